"""FP64 reference implementation of Fourier-domain dedispersion (FDD).  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import or run this
module.  It shares no code with the HIP library (no kernels, tables, constants or helpers),
and the library must never call it.

Paper: Bassa et al., "Fourier-domain dedispersion" (arXiv:2110.03482).

What is computed, in the paper's order and notation:

* Eq. 1 (Sec. 2.1): dispersion delay  dt(nu, DM) = DM * k_DM * (nu^-2 - nu_0^-2).
  In samples: tau[dm, c] = DM_dm * kappa_c with kappa_c = k_DM (nu_c^-2 - nu_ref^-2) / t_samp.
* Eq. 2 (Sec. 2.1): time-domain dedispersion (TDD, "O1"): shift every channel by its delay
  rounded to the nearest sample and sum over channels.
* Eqs. 3-7 (Sec. 2.2): Fourier-domain dedispersion ("O2"): per-channel forward FFT (Eq. 3),
  phasors W = exp(2 pi i f tau / L) (Eq. 4, sign read as an advance, see below), sum over
  channels (Eq. 7), one inverse FFT per DM (Eq. 6), discarding the cyclically contaminated
  end of every series (Sec. 2.2, wrap/discard rule).
* Sec. 5: power spectra |I(f_s, DM)|^2 taken directly from the Fourier-domain result.
* Sec. 2.3, Eq. 8: spin-frequency-scaled DMs.  Scaling a trial DM as DM_ref r / f_s makes the
  phasor of bin f_s equal to that of the reference bin r at DM_ref, so one phasor matrix serves
  a range of bins; the result is then resampled onto the trial DMs (an approximation).

Readings where the paper is silent or inconsistent (all listed in the design notes):

* Direction: output(t) sums input(t + tau): lower frequencies arrive later and must be
  advanced.  With the forward transform of Eq. 3 (kernel exp(-2 pi i f t)), an advance by
  tau is a multiplication by exp(+2 pi i f tau / L).  This matches the paper's statement that
  the *end* of each series is contaminated by the cyclic wrap; Eq. 2/Eq. 4 as printed have
  the opposite sign.
* k_DM = 4.148808e3 MHz^2 pc^-1 cm^3 s (the paper prints the rounded (2.41e-4)^-1).
* nu_ref is the upper band edge; every channel must lie at or below it (tau >= 0).
* "Nearest sample" rounds halves upward: d = floor(tau + 1/2).
* Chunked mode is overlap-save: chunk k covers input samples [kS, kS + L) (zero beyond
  n_samp); its first S = L - D outputs are kept.  Single-chunk mode zero-pads n_samp to L and
  is circular over L.
* The inverse transform drops the imaginary parts of bins 0 and L/2 and scales by 1/L.
* Power spectra keep bins 0 .. L/2 - 1 (DC kept, Nyquist dropped), unnormalised.
* Down-sampling by a shorter inverse transform (Sec. 2.2): a DM with factor d (a power of two)
  is inverted with a real transform of length M = L/d over bins 0 .. M/2, Im of bins 0 and
  M/2 dropped, scaled by 1/L (not 1/M), so that slowly varying series keep their amplitude:
  the series low-passed to |f| < M/2 (half weight at M/2) and sampled every d-th sample.
  Chunk k keeps its first S/d samples at output offset kS/d, so S must be a multiple of d;
  an automatic overlap is rounded up until S is a multiple of the largest factor.

Library primitives used as steps: numpy.fft.rfft / irfft in float64 (pinned against the
direct DFT definition by the tests).
"""
from __future__ import annotations

import math
from typing import Iterable, Optional, Sequence

import numpy as np

__all__ = [
    "K_DM",
    "kappa",
    "delays",
    "nearest_sample",
    "chunk_geometry",
    "tdd",
    "fdd",
    "fdd_power",
    "forward_spectra",
    "phasors",
    "phasor_sum",
    "inverse_real",
    "direct_rdft",
    "explicit_irdft",
    "input_segment",
    "oracle_fdd_rows",
    "inverse_real_short",
    "scaled_phasors",
    "fdd_power_scaled",
]

# Dispersion constant in MHz^2 pc^-1 cm^3 s (Eq. 1).
K_DM = 4.148808e3


# --------------------------------------------------------------------------- Eq. 1: delays

def kappa(freqs_mhz: Sequence[float], ref_freq_mhz: float, tsamp_s: float) -> np.ndarray:
    """Delay in samples per unit DM for each channel: k_DM (nu_c^-2 - nu_ref^-2) / t_samp (Eq. 1)."""
    f = np.asarray(freqs_mhz, dtype=np.float64)
    inv_f2 = 1.0 / (f * f)
    inv_ref2 = 1.0 / (float(ref_freq_mhz) * float(ref_freq_mhz))
    return (K_DM * (inv_f2 - inv_ref2)) / float(tsamp_s)


def delays(dms: Sequence[float], freqs_mhz: Sequence[float], ref_freq_mhz: float,
           tsamp_s: float) -> np.ndarray:
    """tau[dm, c] in samples (float64), Eq. 1: DM times the per-channel delay per unit DM."""
    k = kappa(freqs_mhz, ref_freq_mhz, tsamp_s)
    d = np.asarray(dms, dtype=np.float64)
    return d[:, None] * k[None, :]


def nearest_sample(tau: np.ndarray) -> np.ndarray:
    """Delay rounded to the nearest sample, halves upward (Sec. 2.1, TDD shifts)."""
    return np.floor(np.asarray(tau, dtype=np.float64) + 0.5).astype(np.int64)


def chunk_geometry(n_samp: int, chunk_len: int, overlap: int, single_chunk: bool,
                   max_tau: float, max_factor: int = 1):
    """(stride S, n_chunks, overlap D) of the overlap-save time chunking.

    Sec. 2.2: at least the maximum delay must be discarded at the end of every transformed
    series, so D >= ceil(max tau) and S = L - D samples of each chunk are kept.  overlap <= 0
    picks D = ceil(max tau), enlarged until S is a multiple of max_factor (the largest
    down-sampling factor).  Single-chunk mode transforms one zero-padded series of length L.
    """
    L = int(chunk_len)
    if L <= 0 or (L & (L - 1)) != 0:
        raise ValueError("chunk length must be a power of two")
    if single_chunk:
        if n_samp > L:
            raise ValueError("single-chunk mode needs n_samp <= chunk_len")
        return L, 1, 0
    need = int(math.ceil(max_tau))
    D = need if overlap <= 0 else int(overlap)
    if D < need:
        raise ValueError("overlap shorter than the maximum delay")
    if overlap <= 0:
        while (L - D) % max_factor != 0:
            D += 1
    S = L - D
    if S <= 0:
        raise ValueError("overlap must be shorter than the chunk")
    if S % max_factor != 0:
        raise ValueError("the kept stride must be a multiple of every down-sampling factor")
    return S, -(-int(n_samp) // S), D


# --------------------------------------------------------------------------- input access

def input_segment(x: np.ndarray, kind: str, t0: int, L: int, channels=None) -> np.ndarray:
    """float64 [n_chan, L] holding samples t0 .. t0+L-1 of every channel, zero beyond the data.

    kind "u8": x is time-major uint8 [n_samp][n_chan]; kind "f32": channel-major [n_chan][n_samp].
    """
    if kind == "u8":
        n_samp, n_chan = x.shape
    else:
        n_chan, n_samp = x.shape
    if channels is None:
        channels = slice(None)
    idx = np.arange(n_chan)[channels]
    out = np.zeros((idx.shape[0], L), dtype=np.float64)
    t1 = min(n_samp, t0 + L)
    if t1 > t0:
        if kind == "u8":
            out[:, : t1 - t0] = x[t0:t1, idx].T.astype(np.float64)
        else:
            out[:, : t1 - t0] = x[idx, t0:t1].astype(np.float64)
    return out


def _as_channel_major(x: np.ndarray, kind: str) -> np.ndarray:
    if kind == "u8":
        return np.ascontiguousarray(x.T).astype(np.float64)
    return np.asarray(x, dtype=np.float64)


# --------------------------------------------------------------------------- Eq. 2: TDD (O1)

def tdd(x: np.ndarray, kind: str, d: np.ndarray, circular_len: Optional[int] = None,
        rows: Optional[Iterable[int]] = None) -> np.ndarray:
    """Brute-force time-domain dedispersion with integer delays (Eq. 2, read as an advance).

    y[dm, t] = sum_c xt[c, t + d[dm, c]] for t < n_samp, where xt is x zero-padded to
    circular_len and periodic with that period (circular_len given), or x extended by zeros
    beyond n_samp (circular_len None).
    """
    xc = _as_channel_major(x, kind)
    n_chan, n_samp = xc.shape
    d = np.asarray(d, dtype=np.int64)
    rows = list(range(d.shape[0])) if rows is None else list(rows)
    y = np.zeros((len(rows), n_samp), dtype=np.float64)
    if circular_len is not None:
        L = int(circular_len)
        xp = np.zeros((n_chan, L), dtype=np.float64)
        xp[:, :n_samp] = xc
        t = np.arange(n_samp)
        for i, r in enumerate(rows):
            for c in range(n_chan):
                y[i] += xp[c, (t + d[r, c]) % L]
    else:
        for i, r in enumerate(rows):
            for c in range(n_chan):
                s = int(d[r, c])
                if s < n_samp:
                    y[i, : n_samp - s] += xc[c, s:]
    return y


# --------------------------------------------------------------------------- Eqs. 3-7: FDD (O2)

def forward_spectra(seg: np.ndarray) -> np.ndarray:
    """Eq. 3 on one chunk: X[c, f] = sum_t seg[c, t] exp(-2 pi i f t / L), f = 0 .. L/2."""
    return np.fft.rfft(seg, axis=-1)


def phasors(tau_row: np.ndarray, L: int, mode: str) -> np.ndarray:
    """Eq. 4 for one DM: W[c, f] = exp(+2 pi i f tau_c / L), f = 0 .. L/2.

    mode "round" uses the nearest-sample delay d and the exact phase ((f d) mod L) / L;
    mode "exact" uses the fractional delay with the phase frac(f tau / L) in float64.
    """
    f = np.arange(L // 2 + 1, dtype=np.int64)
    if mode == "round":
        dd = nearest_sample(tau_row)
        ph = ((dd[:, None] * f[None, :]) % L).astype(np.float64) / L
    elif mode == "exact":
        v = np.asarray(tau_row, dtype=np.float64)[:, None] * f[None, :].astype(np.float64) / L
        ph = v - np.floor(v)
    else:
        raise ValueError(mode)
    return np.exp(2j * np.pi * ph)


def phasor_sum(W: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Eq. 7: Y[f] = sum over channels of W[c, f] * X[c, f]."""
    return np.sum(W * X, axis=0)


def inverse_real(Y: np.ndarray, L: int) -> np.ndarray:
    """Eq. 6 inverse: real series of length L from bins 0 .. L/2, scaled by 1/L.

    The imaginary parts of bins 0 and L/2 are dropped (they do not belong to a real series).
    """
    Yc = np.array(Y, dtype=np.complex128, copy=True)
    Yc[..., 0] = Yc[..., 0].real
    Yc[..., -1] = Yc[..., -1].real
    return np.fft.irfft(Yc, n=L, axis=-1)


def inverse_real_short(Y: np.ndarray, L: int, d: int) -> np.ndarray:
    """Down-sampled inverse (Sec. 2.2): real series of length M = L/d from bins 0 .. M/2 of a
    length-L spectrum, Im of bins 0 and M/2 dropped, scaled by 1/L."""
    M = L // d
    return inverse_real(np.asarray(Y)[..., : M // 2 + 1], M) * (M / L)


def oracle_fdd_rows(x: np.ndarray, kind: str, tau: np.ndarray, L: int, stride: int,
                    n_chunks: int, single_chunk: bool, mode: str,
                    rows: Optional[Iterable[int]] = None, power: bool = False,
                    factors: Optional[Sequence[int]] = None):
    """Fourier-domain dedispersion of the requested DM rows (all rows by default).

    Returns float64 [len(rows), n_samp] dedispersed series, or with power=True the power
    spectra [len(rows), L/2] of the single chunk.  With `factors` (one down-sampling factor
    per DM of tau) it returns a list with one float64 series of ceil(n_samp / d) samples per
    requested row.
    """
    n_samp = x.shape[0] if kind == "u8" else x.shape[1]
    rows = list(range(tau.shape[0])) if rows is None else list(rows)
    ds = [1] * len(rows) if factors is None else [int(factors[r]) for r in rows]
    if power:
        if not single_chunk:
            raise ValueError("power spectra need single-chunk mode")
        out = np.zeros((len(rows), L // 2), dtype=np.float64)
    elif factors is None:
        out = np.zeros((len(rows), n_samp), dtype=np.float64)
    else:
        out = [np.zeros(-(-n_samp // d), dtype=np.float64) for d in ds]
    W = [phasors(tau[r], L, mode) for r in rows]      # the phasors do not depend on the chunk
    keep = n_samp if single_chunk else stride
    for k in range(n_chunks):
        t0 = k * stride
        X = forward_spectra(input_segment(x, kind, t0, L))
        for i in range(len(rows)):
            Y = phasor_sum(W[i], X)
            if power:
                out[i] = (Y.real ** 2 + Y.imag ** 2)[: L // 2]
                continue
            d = ds[i]
            y = inverse_real(Y, L) if d == 1 else inverse_real_short(Y, L, d)
            if not single_chunk and stride % d != 0:
                raise ValueError("the kept stride must be a multiple of every down-sampling factor")
            o0 = t0 // d                                  # output samples of this chunk start here
            n = min(-(-keep // d), out[i].shape[0] - o0)
            out[i][o0: o0 + n] = y[:n]
    return out


def fdd(x: np.ndarray, kind: str, dms, freqs_mhz, ref_freq_mhz: float, tsamp_s: float,
        chunk_len: int, overlap: int = 0, single_chunk: bool = False, mode: str = "exact",
        rows: Optional[Iterable[int]] = None, factors: Optional[Sequence[int]] = None):
    """Fourier-domain dedispersion from the observation description (Eqs. 1, 3-7), with
    optional per-DM down-sampling factors (Sec. 2.2)."""
    tau = delays(dms, freqs_mhz, ref_freq_mhz, tsamp_s)
    n_samp = x.shape[0] if kind == "u8" else x.shape[1]
    max_tau = float(tau.max()) if tau.size else 0.0
    dmax = 1 if factors is None else int(max(factors))
    S, n_chunks, _ = chunk_geometry(n_samp, chunk_len, overlap, single_chunk, max_tau, dmax)
    return oracle_fdd_rows(x, kind, tau, chunk_len, S, n_chunks, single_chunk, mode, rows, factors=factors)


def fdd_power(x: np.ndarray, kind: str, dms, freqs_mhz, ref_freq_mhz: float, tsamp_s: float,
              chunk_len: int, mode: str = "exact", rows: Optional[Iterable[int]] = None) -> np.ndarray:
    """Power spectra |Y[dm, f]|^2, f < L/2, of the single-chunk FDD (Sec. 5)."""
    tau = delays(dms, freqs_mhz, ref_freq_mhz, tsamp_s)
    return oracle_fdd_rows(x, kind, tau, chunk_len, chunk_len, 1, True, mode, rows, power=True)


# --------------------------------------------------------------------------- Sec. 2.3, Eq. 8: scaled DMs

def scaled_phasors(kappa_c: np.ndarray, dm: np.ndarray, ref_bin: int, L: int) -> np.ndarray:
    """Eq. 8: the phasor of reference bin r at DM, exp(+2 pi i frac(r DM kappa_c / L)), which by
    the substitution DM_f = DM r / f is also the phasor of every bin f at DM r / f.
    Returns [len(dm), n_chan]."""
    tau = np.asarray(dm, dtype=np.float64)[:, None] * np.asarray(kappa_c, dtype=np.float64)[None, :]
    v = tau * float(ref_bin) / L
    return np.exp(2j * np.pi * (v - np.floor(v)))


def fdd_power_scaled(x: np.ndarray, kind: str, dms, freqs_mhz, ref_freq_mhz: float, tsamp_s: float,
                     chunk_len: int, f_min: int, block: int = 64, halo: int = 32,
                     rows: Optional[Iterable[int]] = None, bins: Optional[Sequence[int]] = None) -> np.ndarray:
    """Power spectra of one chunk with spin-frequency-scaled DMs (Sec. 2.3, Eq. 8).

    Bins below f_min are exact (as fdd_power).  From f_min on, bins form blocks of `block`
    with reference bin r = block start + block/2; the scaled grid DM'_s = DM_0 + s dDM
    (s = -halo .. n_dm + halo - 1) of a block is evaluated with the phasors of bin r, which
    at bin f belong to the DM DM'_s r / f.  Trial DM_j at bin f therefore lies at the
    fractional row s* = (DM_j f / r - DM_0) / dDM, and its power is interpolated linearly
    between rows floor(s*) and floor(s*) + 1:
        P[j, f] = (1 - w) |Ytilde[floor(s*), f]|^2 + w |Ytilde[floor(s*) + 1, f]|^2.
    The DM list must be uniform (DM_0 + j dDM).  Returns float64 [len(rows), len(bins)]
    (all trials and bins 0 .. L/2 - 1 by default).
    """
    L = int(chunk_len)
    dms = np.asarray(dms, dtype=np.float64)
    n_dm = dms.size
    dm0 = float(dms[0])
    step = (float(dms[-1]) - dm0) / (n_dm - 1)
    kap = kappa(freqs_mhz, ref_freq_mhz, tsamp_s)
    rows = list(range(n_dm)) if rows is None else list(rows)
    bins = np.arange(L // 2) if bins is None else np.asarray(bins, dtype=np.int64)
    X = forward_spectra(input_segment(x, kind, 0, L))             # [n_chan, L/2 + 1], Eq. 3
    out = np.zeros((len(rows), bins.size), dtype=np.float64)
    low = bins < f_min
    if np.any(low):
        fl = bins[low]
        for i, j in enumerate(rows):
            W = phasors(dms[j] * kap, L, "exact")[:, fl]             # Eq. 4 at the trial DM
            Y = np.sum(W * X[:, fl], axis=0)
            out[i, low] = Y.real ** 2 + Y.imag ** 2
    tr = dms[rows]
    for k in np.nonzero(~low)[0]:
        f = int(bins[k])
        r = f_min + (f - f_min) // block * block + block // 2
        ss = (tr * f / r - dm0) / step                               # fractional scaled rows
        s0 = np.floor(ss)
        w = ss - s0
        if np.any(s0 < -halo) or np.any(s0 + 1 >= n_dm + halo):
            raise ValueError("trial outside the scaled grid's halo")
        p = []
        for s in (s0, s0 + 1):
            Yt = scaled_phasors(kap, dm0 + s * step, r, L) @ X[:, f]
            p.append(Yt.real ** 2 + Yt.imag ** 2)
        out[:, k] = (1.0 - w) * p[0] + w * p[1]
    return out


# --------------------------------------------------------------------------- definitions used as pins

def direct_rdft(seg: np.ndarray) -> np.ndarray:
    """Eq. 3 written out as a direct sum (O(L^2)); for small L only."""
    L = seg.shape[-1]
    t = np.arange(L)
    f = np.arange(L // 2 + 1)
    ph = ((f[:, None] * t[None, :]) % L) / L
    return seg @ np.exp(-2j * np.pi * ph).T


def explicit_irdft(Y: np.ndarray, L: int) -> np.ndarray:
    """Inverse real DFT written out: y[t] = (1/L)[Re Y_0 + (-1)^t Re Y_{L/2}
    + 2 sum_{f=1}^{L/2-1} Re(Y_f exp(2 pi i f t / L))]; for small L only."""
    t = np.arange(L)
    f = np.arange(1, L // 2)
    ph = ((f[:, None] * t[None, :]) % L) / L
    E = np.exp(2j * np.pi * ph)
    mid = 2.0 * np.real(Y[..., 1: L // 2] @ E)
    sgn = np.where(t % 2 == 0, 1.0, -1.0)
    return (Y[..., :1].real + sgn * Y[..., L // 2: L // 2 + 1].real + mid) / L
