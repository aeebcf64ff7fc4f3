"""GPU parity of the split-precision phasor sums (FP16 and BF16 head/tail on MFMA, FP32 accumulation).

The error of each form is measured against the FP64 oracle and printed; rows are checked
element by element by `parity.check_rows` (row norm, centred norm, per-sample bound; 8-bit
rows on the centred norm, see tests/parity.py).  The bounds sit above the measured values
with margin and are derived in the design notes:
 - FP16 split: head + tail carry ~22 significant bits and only the tail x tail product
   (~2^-22) is dropped, so the path is as accurate as FP32 (bound 1e-5, the FP32 bar);
 - BF16 split: head + tail carry ~16 bits; the dropped tail x tail product and the bf16
   rounding of the tails leave ~2^-17 per product (bound 1e-4).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from parity import check_power, check_rows, raw_start_of

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdd = pytest.importorskip("paper_2110_03482_amd")

BOUND = {"fp16_split": 1e-5, "bf16_split": 1e-4}


def run_gpu(w, x, mode, precision, power=False, geometry=False):
    with fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, overlap=w.overlap,
                  single_chunk=w.single_chunk, input=w.input_kind, mode=mode, precision=precision) as p:
        xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        out = p.power_spectrum(xd) if power else p.execute(xd)
        torch.cuda.synchronize()
        if geometry:
            return out.cpu().numpy(), p.kernel, p.geometry
        return out.cpu().numpy(), p.kernel


@pytest.mark.parametrize("precision", ["fp16_split", "bf16_split"])
@pytest.mark.parametrize("mode", ["exact", "round"])
def test_split_small(precision, mode):
    w = W.small_fp32(0)
    x = W.gaussian_f32(w.n_chan, w.n_samp, 0)
    offs = O.nearest_sample(O.delays([30.0], w.freqs, w.ref_freq_mhz, w.tsamp_s))[0]
    W.inject_pulse_f32(x, offs, 1000, 5.0, circular=True)
    y, kernel = run_gpu(w, x, mode, precision)
    ref = O.fdd(x, "f32", w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len, single_chunk=True, mode=mode)
    check_rows(y, ref, BOUND[precision], label=f"{precision} {mode} small kernel={kernel}")
    assert int(np.argmax(y[:, 1000])) == 30


_SWEEP_REF = {}


def sweep_reference(w, x):
    """Oracle rows of the sweep workload (every trial up to 2048 trials, then every
    n_dm/2048-th), computed once per DM count."""
    if w.n_dm not in _SWEEP_REF:
        _SWEEP_REF.clear()
        rows = list(range(0, w.n_dm, max(1, w.n_dm // 2048)))
        _SWEEP_REF[w.n_dm] = rows, O.fdd(x, "f32", w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len,
                                         single_chunk=True, mode="exact", rows=rows)
    return _SWEEP_REF[w.n_dm]


@pytest.mark.parametrize("precision", ["fp16_split", "bf16_split"])
@pytest.mark.parametrize("n_dm", [256, 512, 1024, 2048, 4096, 8192])
def test_precision_sweep(precision, n_dm):
    """The small band with n_dm trials DM_j = j 64 / n_dm: error per DM count."""
    w = W.precision_sweep(n_dm)
    x = W.gaussian_f32(w.n_chan, w.n_samp, 0)
    offs = O.nearest_sample(O.delays([30.0], w.freqs, w.ref_freq_mhz, w.tsamp_s))[0]
    W.inject_pulse_f32(x, offs, 1000, 5.0, circular=True)
    y, kernel = run_gpu(w, x, "exact", precision)
    y32, _ = run_gpu(w, x, "exact", "fp32")
    rows, ref = sweep_reference(w, x)
    s32 = check_rows(y32[rows], ref, 1e-5)
    st = check_rows(y[rows], ref, BOUND[precision])
    print(f"sweep {precision} n_dm={n_dm} kernel={kernel}: {st.line()} "
          f"(fp32 path: rel {s32.rel:.3e}, centred {s32.centred:.3e}, max abs {s32.max_abs:.3e})")
    # fine grids resolve DM 30 only to within the delay smearing of a few trials
    assert abs(w.dms[int(np.argmax(y[:, 1000]))] - 30.0) <= 0.25


CHUNKED = [
    (13, 20000, 70, 2048, "f32", 10.0),   # 11 chunks, 2 column tiles
    (64, 50001, 64, 8192, "u8", 40.0),    # 7 chunks, 8-bit
    (40, 30000, 100, 4096, "f32", 2.0),   # 8 chunks
    (32, 30000, 33, 2048, "u8", 8.0),     # 21 chunks, 3 column tiles
]


@pytest.mark.parametrize("case", CHUNKED, ids=[f"{c[0]}ch_{c[1]}s_{c[2]}dm_L{c[3]}_{c[4]}" for c in CHUNKED])
@pytest.mark.parametrize("precision", ["fp16_split", "bf16_split"])
def test_split_chunked(case, precision):
    n_chan, n_samp, n_dm, L, kind, dm_max = case
    seed = n_chan + n_dm
    w = W.tiny_random(seed, n_chan, n_samp, n_dm, L, single_chunk=False, input_kind=kind, dm_max=dm_max)
    x = W.gaussian_u8(n_samp, n_chan, seed) if kind == "u8" else W.gaussian_f32(n_chan, n_samp, seed)
    for mode in ("exact", "round"):
        y, kernel, g = run_gpu(w, x, mode, precision, geometry=True)
        ref = O.fdd(x, kind, w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, L, mode=mode)
        check_rows(y, ref, BOUND[precision], raw_from=raw_start_of(kind, g, n_samp, False),
                   label=f"{precision} {mode} {case} kernel={kernel} chunks={g.n_chunks}")


@pytest.mark.parametrize("precision", ["fp16_split", "bf16_split"])
def test_split_power(precision):
    w = W.small_fp32(3)
    x = W.gaussian_f32(w.n_chan, w.n_samp, 3)
    P, _ = run_gpu(w, x, "exact", precision, power=True)
    tau = O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s)
    ref = O.oracle_fdd_rows(x, "f32", tau, w.chunk_len, w.chunk_len, 1, True, "exact", power=True)
    check_power(P, ref, BOUND[precision], label=f"{precision} power")


@pytest.mark.parametrize("precision", ["fp16_split", "bf16_split"])
def test_split_paper_shaped_rows(precision):
    w = W.paper_shaped_u8()
    x = W.gaussian_u8(w.n_samp, w.n_chan, 0)
    for dm, t0 in ((100.0, 1 << 18), (450.0, 1 << 19), (900.0, 3 << 18)):
        offs = O.nearest_sample(O.delays([dm], w.freqs, w.ref_freq_mhz, w.tsamp_s))[0]
        W.inject_pulse_u8(x, offs, t0, 80.0)
    y, kernel, g = run_gpu(w, x, "exact", precision, geometry=True)
    rows = [0, 3, 921, 1842, 2047]
    ref = O.fdd(x, "u8", w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len, mode="exact", rows=rows)
    check_rows(y[rows], ref, BOUND[precision], raw_from=raw_start_of("u8", g, w.n_samp, False),
               label=f"{precision} paper-shaped rows {rows} kernel={kernel}")
    for trial, t0 in ((205, 1 << 18), (921, 1 << 19), (1842, 3 << 18)):
        assert abs(int(np.argmax(y[:, t0 - 2: t0 + 3].max(axis=1))) - trial) <= 2
