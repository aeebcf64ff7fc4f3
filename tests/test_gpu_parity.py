"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element by element.

Tolerance (FP32 path): 1e-5, checked per DM row by `parity.check_rows` as a row norm, a
mean-removed (centred) norm plus the float32 storage floor, and a per-sample bound of ten
times the allowed RMS error, so that the 128 n_chan zero-point offset of 8-bit rows cannot hide
a seam or tail defect.  8-bit chunks that run past the end of the data keep their zero point
(the 128 -> 0 step there is not a pure DC term); their samples are held to the same 1e-5
relative to their own uncentred norm (derivation in tests/parity.py).
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity import check_power, check_rows, raw_start_of

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdd = pytest.importorskip("paper_2110_03482_amd")

TOL = 1e-5


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run_gpu(w, x, mode, power=False):
    with fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, overlap=w.overlap,
                  single_chunk=w.single_chunk, input=w.input_kind, mode=mode) as p:
        xd = to_dev(x)
        out = p.power_spectrum(xd) if power else p.execute(xd)
        torch.cuda.synchronize()
        return out.cpu().numpy(), p.kernel, p.geometry


def run_oracle(w, x, mode, rows=None):
    return O.fdd(x, w.input_kind, w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len, overlap=w.overlap,
                 single_chunk=w.single_chunk, mode=mode, rows=rows)


def small_input(seed=0):
    w = W.small_fp32(seed)
    x = W.gaussian_f32(w.n_chan, w.n_samp, seed)
    offs = O.nearest_sample(O.delays([30.0], w.freqs, w.ref_freq_mhz, w.tsamp_s))[0]
    W.inject_pulse_f32(x, offs, 1000, 5.0, circular=True)
    return w, x


# ----------------------------------------------------------------------------- small workload

@pytest.mark.parametrize("mode", ["exact", "round"])
def test_small_matches_oracle(mode):
    w, x = small_input()
    print(f"small workload, mode={mode}", flush=True)
    y, kernel, _ = run_gpu(w, x, mode)
    ref = run_oracle(w, x, mode)
    check_rows(y, ref, TOL, label=f"small {mode} kernel={kernel}")
    assert int(np.argmax(y[:, 1000])) == 30


def test_small_round_equals_circular_tdd():
    w, x = small_input(1)
    y, _, _ = run_gpu(w, x, "round")
    d = O.nearest_sample(O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s))
    ref = O.tdd(x, "f32", d, circular_len=w.chunk_len)
    check_rows(y, ref, TOL, label="small round vs circular TDD")


def test_dm_zero_row_is_channel_sum():
    w, x = small_input(2)
    y, _, _ = run_gpu(w, x, "exact")
    ref = x.astype(np.float64).sum(axis=0)
    check_rows(y[:1], ref[None], TOL, label="DM 0 vs channel sum")


@pytest.mark.parametrize("n_dm", [256, 1024])
def test_precision_sweep_workload_fp32(n_dm):
    w = W.precision_sweep(n_dm)
    x = W.gaussian_f32(w.n_chan, w.n_samp, 0)
    y, _, _ = run_gpu(w, x, "exact")
    rows = list(range(0, n_dm, max(1, n_dm // 64)))
    ref = run_oracle(w, x, "exact", rows=rows)
    check_rows(y[rows], ref, TOL, label=f"precision sweep workload fp32 n_dm={n_dm}")


# ----------------------------------------------------------------------------- chunked shapes

CHUNKED = [
    # n_chan, n_samp, n_dm, L, kind, dm_max          chunks: VALU (1-2) and MFMA (>= 3) paths
    (8, 3000, 5, 4096, "f32", 20.0),      # 1 chunk + ragged (VALU)
    (16, 6000, 9, 4096, "f32", 20.0),     # 2 chunks (VALU)
    (13, 20000, 70, 2048, "f32", 10.0),   # many chunks, odd channel count, DM tile ragged (MFMA)
    (64, 50001, 64, 8192, "u8", 40.0),    # 8-bit input, ragged tail (MFMA)
    (32, 30000, 130, 4096, "u8", 25.0),   # (MFMA, 3 DM tiles)
    (40, 9000, 33, 1024, "f32", 3.0),     # short chunks, many of them (MFMA, 2 column tiles)
    (5, 700, 3, 64, "f32", 0.05),         # shortest transform
    (16, 20000, 700, 2048, "u8", 8.0),    # 700 DMs, 11 chunks (MFMA, 11 DM tiles)
    (12, 9000, 1100, 1024, "f32", 4.0),   # 1100 DMs, 10 chunks (MFMA, ragged last DM tile)
]


@pytest.mark.parametrize("case", CHUNKED, ids=[f"{c[0]}ch_{c[1]}s_{c[2]}dm_L{c[3]}_{c[4]}" for c in CHUNKED])
@pytest.mark.parametrize("mode", ["exact", "round"])
def test_chunked_matches_oracle(case, mode):
    n_chan, n_samp, n_dm, L, kind, dm_max = case
    seed = n_chan * 7 + n_dm
    w = W.tiny_random(seed, n_chan, n_samp, n_dm, L, single_chunk=False, input_kind=kind, dm_max=dm_max)
    x = W.gaussian_u8(n_samp, n_chan, seed) if kind == "u8" else W.gaussian_f32(n_chan, n_samp, seed)
    print(f"chunked case {case} mode={mode}", flush=True)
    y, kernel, g = run_gpu(w, x, mode)
    ref = run_oracle(w, x, mode)
    raw = raw_start_of(kind, g, n_samp, False)
    check_rows(y, ref, TOL, raw_from=raw, label=f"kernel={kernel} chunks={g.n_chunks}")
    if mode == "round":
        d = O.nearest_sample(O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s))
        check_rows(y, O.tdd(x, kind, d), TOL, raw_from=raw, label="  vs zero-extended TDD")


def test_single_chunk_shorter_than_transform():
    w = W.tiny_random(3, 12, 2500, 17, 4096, single_chunk=True)
    x = W.gaussian_f32(w.n_chan, w.n_samp, 3)
    for mode in ("exact", "round"):
        y, _, _ = run_gpu(w, x, mode)
        check_rows(y, run_oracle(w, x, mode), TOL, label=f"single chunk shorter than L, {mode}")


def test_single_channel_single_dm():
    w = W.tiny_random(4, 1, 4096, 1, 4096, single_chunk=True)
    x = W.gaussian_f32(1, 4096, 4)
    y, _, _ = run_gpu(w, x, "exact")
    check_rows(y, run_oracle(w, x, "exact"), TOL, label="one channel, one DM")


# ----------------------------------------------------------------------------- power spectra

@pytest.mark.parametrize("mode", ["exact", "round"])
def test_power_spectrum_small(mode):
    w, x = small_input(5)
    P, _, _ = run_gpu(w, x, mode, power=True)
    tau = O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s)
    ref = O.oracle_fdd_rows(x, "f32", tau, w.chunk_len, w.chunk_len, 1, True, mode, power=True)
    # power is quadratic: its relative error is twice that of the amplitudes
    check_power(P, ref, TOL, label=f"power small {mode}")


def test_power_spectrum_u8_full_transform():
    w = W.tiny_random(6, 24, 8192, 40, 8192, single_chunk=True, input_kind="u8")
    x = W.gaussian_u8(w.n_samp, w.n_chan, 6)
    P, _, _ = run_gpu(w, x, "exact", power=True)
    tau = O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s)
    ref = O.oracle_fdd_rows(x, "u8", tau, w.chunk_len, w.chunk_len, 1, True, "exact", power=True)
    check_power(P, ref, TOL, skip_dc=True, label="power 8-bit full transform")
    np.testing.assert_allclose(P[:, 0], ref[:, 0], rtol=2e-6)


def test_power_rejects_chunked_plan():
    w = W.tiny_random(7, 8, 9000, 4, 1024, single_chunk=False, dm_max=2.0)
    with fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len) as p:
        x = to_dev(W.gaussian_f32(w.n_chan, w.n_samp, 7))
        with pytest.raises(fdd.FddError) as e:
            p.power_spectrum(x, out=torch.empty((w.n_dm, 512), device="cuda"))
        assert e.value.status == 3


# ----------------------------------------------------------------------------- paper-shaped, full size

@pytest.fixture(scope="module")
def paper_input():
    w = W.paper_shaped_u8()
    x = W.gaussian_u8(w.n_samp, w.n_chan, 0)
    for dm, t0 in ((100.0, 1 << 18), (450.0, 1 << 19), (900.0, 3 << 18)):
        offs = O.nearest_sample(O.delays([dm], w.freqs, w.ref_freq_mhz, w.tsamp_s))[0]
        W.inject_pulse_u8(x, offs, t0, 80.0)
    return w, x


@pytest.mark.parametrize("factor", ["default", "wide", "linear"])
def test_paper_shaped_sampled_rows(paper_input, factor):
    """1024 ch x 2^20 8-bit samples x 2048 DMs, L = 2^16 (21 chunks): rows checked against the
    oracle, on the direct FP32 kernel (the default), on the chunked DM-factorised FP32 kernel
    (FDD_FACTOR=wide) and on the direct kernel with per-channel linear increments
    (FDD_PHASE_TABLE=linear)."""
    w, x = paper_input
    print(f"paper-shaped workload, exact mode, {factor} kernel", flush=True)
    env = {"wide": ("FDD_FACTOR", "wide"), "linear": ("FDD_PHASE_TABLE", "linear")}.get(factor)
    if env is not None:
        os.environ[env[0]] = env[1]
    try:
        y, kernel, g = run_gpu(w, x, "exact")
    finally:
        if env is not None:
            os.environ.pop(env[0], None)
    assert kernel == ("facw_f32" if factor == "wide" else "mfma_f32") and g.n_chunks == 21
    rows = [0, 1, 921, 1842, 2047]
    ref = run_oracle(w, x, "exact", rows=rows)
    check_rows(y[rows], ref, TOL, raw_from=raw_start_of("u8", g, w.n_samp, False),
               label=f"paper-shaped exact rows {rows}")
    # properties over every row: finite, DM 0 is the channel sum, pulses found at their trials
    assert np.isfinite(y).all()
    for trial, t0 in ((205, 1 << 18), (921, 1 << 19), (1842, 3 << 18)):
        win = y[:, t0 - 2: t0 + 3].max(axis=1)
        assert abs(int(np.argmax(win)) - trial) <= 2, (trial, int(np.argmax(win)))


def test_paper_shaped_round_vs_tdd(paper_input):
    w, x = paper_input
    y, _, g = run_gpu(w, x, "round")
    rows = [0, 1, 921, 1842, 2047]
    d = O.nearest_sample(O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s))
    ref = O.tdd(x, "u8", d, rows=rows)
    check_rows(y[rows], ref, TOL, raw_from=raw_start_of("u8", g, w.n_samp, False),
               label=f"paper-shaped round rows {rows} vs TDD")
