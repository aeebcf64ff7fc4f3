"""Seeded synthetic filterbank workloads shared by the tests, the benchmark and the smoke check.

This module only describes workloads and draws random numbers: observing-band layout, DM
grids, Gaussian (float32) or 8-bit filterbank noise, and the placement of injected pulses at
per-channel sample offsets that the *caller* supplies.  It contains none of the
dedispersion arithmetic (no dispersion delays, no Fourier transforms, no phasors): callers
compute the arrival offsets of an injected pulse with whatever implementation they are
testing against and pass them in.

The shapes follow the workloads of the paper's performance study (Section 4.1: 1024 channels,
64 us sampling, a few hundred MHz of bandwidth near 1.4 GHz, trial DMs from zero in uniform
steps), which are simulated data that are not available here; the recipes below stand in for
them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Workload",
    "channel_centres",
    "small_fp32",
    "paper_shaped_u8",
    "precision_sweep",
    "periodicity",
    "batched_beams",
    "gaussian_f32",
    "gaussian_u8",
    "inject_pulse_f32",
    "inject_pulse_u8",
    "inject_periodic_f32",
    "tiny_random",
]


@dataclasses.dataclass
class Workload:
    """One dedispersion problem: band layout, DM trials, geometry and input encoding."""

    name: str
    n_chan: int
    f_lo_mhz: float          # lower band edge
    f_hi_mhz: float          # upper band edge
    ref_freq_mhz: float      # reference frequency (upper band edge)
    tsamp_s: float
    n_samp: int
    dms: np.ndarray          # float64 trial DMs, pc cm^-3
    chunk_len: int           # FFT length L (power of two)
    overlap: int             # 0 = let the planner choose ceil(max delay)
    single_chunk: bool       # one zero-padded, circular transform of length L
    input_kind: str          # "u8" (time-major [n_samp][n_chan]) or "f32" ([n_chan][n_samp])
    seed: int = 0

    @property
    def freqs(self) -> np.ndarray:
        return channel_centres(self.f_lo_mhz, self.f_hi_mhz, self.n_chan)

    @property
    def n_dm(self) -> int:
        return int(self.dms.shape[0])


def channel_centres(f_lo_mhz: float, f_hi_mhz: float, n_chan: int) -> np.ndarray:
    """Centres of n_chan equal-width channels covering [f_lo, f_hi], ascending."""
    bw = (f_hi_mhz - f_lo_mhz) / n_chan
    return f_lo_mhz + (np.arange(n_chan, dtype=np.float64) + 0.5) * bw


# --------------------------------------------------------------------------- configurations

def small_fp32(seed: int = 0) -> Workload:
    """64 channels over 1350-1450 MHz, 64 us, 4096 float samples, 64 DMs 0..63, one circular chunk."""
    return Workload("small_fp32_64ch_4096s_64dm", 64, 1350.0, 1450.0, 1450.0, 64e-6, 4096,
                    np.arange(64, dtype=np.float64), 4096, 0, True, "f32", seed)


def paper_shaped_u8(seed: int = 0, n_dm: int = 2048) -> Workload:
    """1024 channels over 1250-1550 MHz, 64 us, 2^20 8-bit samples, DMs 0..1000, L = 2^16 chunks."""
    return Workload(f"paper_u8_1024ch_2p20s_{n_dm}dm", 1024, 1250.0, 1550.0, 1550.0, 64e-6, 1 << 20,
                    np.linspace(0.0, 1000.0, n_dm), 1 << 16, 0, False, "u8", seed)


def precision_sweep(n_dm: int, seed: int = 0) -> Workload:
    """The small workload with n_dm trials DM_j = j*64/n_dm (keeps DM 30 on the grid)."""
    w = small_fp32(seed)
    w.name = f"precision_64ch_4096s_{n_dm}dm"
    w.dms = np.arange(n_dm, dtype=np.float64) * (64.0 / n_dm)
    return w


def periodicity(seed: int = 0, n_samp: int = 1 << 22, n_dm: int = 4096) -> Workload:
    """512 channels over 1250-1550 MHz, one unchunked transform of 2^22 samples, DMs 0..500."""
    return Workload(f"periodicity_512ch_{n_samp}s_{n_dm}dm", 512, 1250.0, 1550.0, 1550.0, 64e-6, n_samp,
                    np.linspace(0.0, 500.0, n_dm), n_samp, 0, True, "f32", seed)


def batched_beams(n_beams: int = 32, seed: int = 0, max_log_samp: int = 20):
    """Uneven beams: n_chan in {256,512,1024}, n_samp = 2^k (k in 16..max), n_dm = 2^m (m in 9..12).

    Returns a list of (Workload, pulse_dm, t0) with the pulse DM drawn uniformly in [0, 800].
    """
    rng = np.random.default_rng(seed)
    beams = []
    for b in range(n_beams):
        n_chan = int(rng.choice([256, 512, 1024]))
        log_samp = int(rng.integers(16, max_log_samp + 1))
        n_dm = 1 << int(rng.integers(9, 13))
        pulse_dm = float(rng.uniform(0.0, 800.0))
        n_samp = 1 << log_samp
        w = Workload(f"beam{b}_{n_chan}ch_2p{log_samp}s_{n_dm}dm", n_chan, 1250.0, 1550.0, 1550.0, 64e-6,
                     n_samp, np.linspace(0.0, 1000.0, n_dm), 1 << 16, 0, False, "f32", seed * 1000 + b)
        beams.append((w, pulse_dm, n_samp // 4))
    return beams


# --------------------------------------------------------------------------- random inputs

def gaussian_f32(n_chan: int, n_samp: int, seed: int) -> np.ndarray:
    """Channel-major float32 [n_chan][n_samp], iid N(0,1)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_chan, n_samp), dtype=np.float32)


def gaussian_u8(n_samp: int, n_chan: int, seed: int, mean: float = 128.0, sigma: float = 16.0) -> np.ndarray:
    """Time-major uint8 [n_samp][n_chan]: N(mean, sigma), rounded to nearest, clipped to 0..255.

    Generated in blocks of rows so that a 2^20 x 1024 array never needs a float64 copy.
    """
    rng = np.random.default_rng(seed)
    out = np.empty((n_samp, n_chan), dtype=np.uint8)
    block = max(1, (1 << 22) // max(1, n_chan))
    for r0 in range(0, n_samp, block):
        r1 = min(n_samp, r0 + block)
        v = rng.standard_normal((r1 - r0, n_chan), dtype=np.float32)
        v = np.rint(v * np.float32(sigma) + np.float32(mean))
        np.clip(v, 0.0, 255.0, out=v)
        out[r0:r1] = v.astype(np.uint8)
    return out


def inject_pulse_f32(x: np.ndarray, offsets: np.ndarray, t0: int, amp: float,
                     circular: bool) -> None:
    """Add a one-sample pulse of height amp to channel c at sample t0 + offsets[c] (in place).

    x is channel-major [n_chan][n_samp].  With circular=True the index wraps modulo n_samp,
    otherwise samples past the end are dropped.
    """
    n_chan, n_samp = x.shape
    for c in range(n_chan):
        t = int(t0) + int(offsets[c])
        if circular:
            t %= n_samp
        if 0 <= t < n_samp:
            x[c, t] += np.float32(amp)


def inject_pulse_u8(x: np.ndarray, offsets: np.ndarray, t0: int, amp: float) -> None:
    """Add amp to time-major uint8 x[t0 + offsets[c], c], saturating at 255 (in place)."""
    n_samp, n_chan = x.shape
    for c in range(n_chan):
        t = int(t0) + int(offsets[c])
        if 0 <= t < n_samp:
            x[t, c] = np.uint8(min(255, int(x[t, c]) + int(round(amp))))


def inject_periodic_f32(x: np.ndarray, shifts: np.ndarray, period_samples: float, duty: float,
                        amp: float) -> None:
    """Add a top-hat pulse train to channel-major x (in place).

    Channel c is "on" at samples t where frac((t - shifts[c]) / period) < duty; shifts[c] is
    the (fractional) arrival offset of the train in that channel, supplied by the caller.
    """
    n_chan, n_samp = x.shape
    t = np.arange(n_samp, dtype=np.float64)
    for c in range(n_chan):
        ph = (t - float(shifts[c])) / period_samples
        on = (ph - np.floor(ph)) < duty
        x[c, on] += np.float32(amp)


def tiny_random(seed: int, n_chan: int, n_samp: int, n_dm: int, chunk_len: int,
                single_chunk: bool, input_kind: str = "f32", dm_max: Optional[float] = None) -> Workload:
    """A small random problem for property tests (band 1200-1500 MHz, 64 us)."""
    rng = np.random.default_rng(seed)
    if dm_max is None:
        dm_max = float(rng.uniform(1.0, 40.0))
    dms = np.sort(rng.uniform(0.0, dm_max, size=n_dm))
    return Workload(f"tiny{seed}", n_chan, 1200.0, 1500.0, 1500.0, 64e-6, n_samp, dms, chunk_len, 0,
                    single_chunk, input_kind, seed)


def is_pow2(v: int) -> bool:
    return v > 0 and (v & (v - 1)) == 0


def ilog2(v: int) -> int:
    return int(math.log2(v))
