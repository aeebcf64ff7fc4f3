"""GPU parity of long transforms (L > 2^16: multi-pass FFT) against the FP64 oracle.

Covers the periodicity workload of Sec. 5 (power spectra straight from the Fourier domain):
512 channels, one unchunked 2^22-sample transform, 4096 DMs, at full size on sampled rows.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from parity import check_power, check_rows, raw_start_of

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdd = pytest.importorskip("paper_2110_03482_amd")

TOL = 1e-5


def plan_for(w, mode, precision="fp32", power_only=False):
    return fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, overlap=w.overlap,
                    single_chunk=w.single_chunk, input=w.input_kind, mode=mode, precision=precision,
                    power_only=power_only)


LONG = [
    # n_chan, n_samp, n_dm, L, single, kind           pass radices (log2): 2^17: 4,4,4,4
    (6, 131072, 5, 131072, True, "f32"),      # 2^17, one chunk
    (4, 262144, 3, 262144, True, "f32"),      # 2^18: 4,4,4,5 (radix-32 pass)
    (3, 1 << 22, 2, 1 << 22, True, "f32"),    # 2^22: 4,4,4,4,5
    (5, 300000, 7, 1 << 19, True, "f32"),     # 2^19 > n_samp (zero padding)
    (4, 1 << 20, 3, 1 << 20, True, "u8"),     # 2^20, 8-bit, zero point restored
    (6, 400000, 9, 131072, False, "f32"),     # chunked with long chunks
]


@pytest.mark.parametrize("case", LONG, ids=[f"{c[0]}ch_{c[1]}s_{c[2]}dm_L{c[3]}_{'single' if c[4] else 'chunked'}_{c[5]}"
                                            for c in LONG])
@pytest.mark.parametrize("mode", ["exact", "round"])
def test_long_execute(case, mode):
    n_chan, n_samp, n_dm, L, single, kind = case
    w = W.tiny_random(n_chan + n_dm, n_chan, n_samp, n_dm, L, single_chunk=single, input_kind=kind, dm_max=30.0)
    x = W.gaussian_u8(n_samp, n_chan, 5) if kind == "u8" else W.gaussian_f32(n_chan, n_samp, 5)
    print(f"long case {case} mode={mode}", flush=True)
    with plan_for(w, mode) as p:
        y = p.execute(torch.from_numpy(np.ascontiguousarray(x)).cuda())
        torch.cuda.synchronize()
        y = y.cpu().numpy()
        g = p.geometry
    ref = O.fdd(x, kind, w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, L, single_chunk=single, mode=mode)
    check_rows(y, ref, TOL, raw_from=raw_start_of(kind, g, n_samp, single), label=f"long {case} {mode}")


@pytest.mark.parametrize("precision", ["fp32", "fp16_split", "bf16_split"])
def test_long_power(precision):
    w = W.tiny_random(41, 8, 1 << 20, 12, 1 << 20, single_chunk=True, dm_max=50.0)
    x = W.gaussian_f32(w.n_chan, w.n_samp, 41)
    with plan_for(w, "exact", precision, power_only=True) as p:
        P = p.power_spectrum(torch.from_numpy(x).cuda())
        torch.cuda.synchronize()
        P = P.cpu().numpy()
        with pytest.raises(fdd.FddError):
            p.execute(torch.from_numpy(x).cuda())
    tau = O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s)
    ref = O.oracle_fdd_rows(x, "f32", tau, w.chunk_len, w.chunk_len, 1, True, "exact", power=True)
    check_power(P, ref, {"fp32": TOL, "fp16_split": TOL, "bf16_split": 1e-4}[precision],
                label=f"{precision} long power")


def test_periodicity_workload_sampled_rows():
    """512 ch x 2^22 samples x 4096 DMs (0..500), power spectra; pulsar at DM 57, P = 33 ms."""
    w = W.periodicity()
    x = W.gaussian_f32(w.n_chan, w.n_samp, 0)
    tau57 = O.delays([57.0], w.freqs, w.ref_freq_mhz, w.tsamp_s)[0]
    period = 33.0e-3 / w.tsamp_s                                   # 515.625 samples
    W.inject_periodic_f32(x, tau57, period, 0.03, 0.3)
    print("periodicity workload: running", flush=True)
    f1 = w.n_samp / period                                          # spin frequency: 8134.4 bins
    idx = []
    for h in range(1, 9):                                           # first 8 harmonics, +-2 bins
        c = int(round(h * f1))
        idx.extend(range(c - 2, c + 3))
    rows = [0, 467, 4095]
    with plan_for(w, "exact", "fp16_split", power_only=True) as p:
        P = p.power_spectrum(torch.from_numpy(x).cuda())
        torch.cuda.synchronize()
        finite = bool(torch.isfinite(P).all().item())
        hs = P[:, idx].double().sum(dim=1).cpu().numpy()
        Ps = P[rows].cpu().numpy()
    del P
    print(f"finite={finite} harmonic sums: trial 0 {hs[0]:.4e}, trial 467 {hs[467]:.4e}, max {hs.max():.4e} "
          f"at {int(np.argmax(hs))}", flush=True)
    tau = O.delays(w.dms[rows], w.freqs, w.ref_freq_mhz, w.tsamp_s)
    ref = O.oracle_fdd_rows(x, "f32", tau, w.chunk_len, w.chunk_len, 1, True, "exact", power=True)
    print(f"oracle harmonic sums: {ref[:, idx].sum(axis=1)}", flush=True)
    assert finite
    check_power(Ps, ref, TOL, label=f"periodicity rows {rows}")
    best = int(np.argmax(hs))
    assert abs(w.dms[best] - 57.0) < 1.0
