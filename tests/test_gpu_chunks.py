"""GPU parity of the direct matrix-core phasor sums on plans with more than 24 chunks.

The direct kernels hold at most 24 chunks (48 real columns) per workgroup; a wider plan runs
them over balanced chunk groups, each launch reading X and writing the Y planes at its group's
first chunk with rows strided by the plan's chunk count (Eq. 7 over the overlap-save chunks of
Sec. 2.2).  Random DM lists and nearest-sample delays keep these plans off the DM-factorised
kernels.  Every sampled row spans all chunk groups, so a chunk read from or written to the wrong
row, or a group seam, fails the per-sample bound of check_rows.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from parity import check_rows, raw_start

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdd = pytest.importorskip("paper_2110_03482_amd")

TOL = {"fp32": 1e-5, "fp16_split": 1e-5, "bf16_split": 1e-4}
KERNEL = {"fp32": "mfma_f32", "fp16_split": "mfma_f16_split", "bf16_split": "mfma_bf16_split"}

CASES = [
    # seed, n_chan, n_samp, n_dm, L, kind, dm_max, mode         chunks (groups)
    (31, 32, 59000, 200, 2048, "u8", 40.0, "exact"),             # 42 (2 x 21), ragged 8-bit tail
    (32, 24, 90000, 150, 2048, "f32", 40.0, "round"),            # 64 (22, 21, 21)
    (33, 20, 140000, 100, 2048, "u8", 20.0, "round"),            # 81 (21, 20, 20, 20)
    (34, 40, 130000, 300, 4096, "f32", 60.0, "exact"),           # 42 at L = 4096
]


def run(w, x, precision, mode):
    with fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, overlap=w.overlap,
                  single_chunk=False, input=w.input_kind, mode=mode, precision=precision) as p:
        y = p.execute(torch.from_numpy(np.ascontiguousarray(x)).cuda())
        torch.cuda.synchronize()
        return y.cpu().numpy(), p.kernel, p.geometry


@pytest.mark.parametrize("case", CASES, ids=[f"{c[1]}ch_{c[2]}s_L{c[4]}_{c[5]}_{c[7]}" for c in CASES])
@pytest.mark.parametrize("precision", ["fp32", "fp16_split", "bf16_split"])
def test_direct_kernels_over_chunk_groups(case, precision):
    seed, n_chan, n_samp, n_dm, L, kind, dm_max, mode = case
    w = W.tiny_random(seed, n_chan, n_samp, n_dm, L, single_chunk=False, input_kind=kind, dm_max=dm_max)
    x = W.gaussian_u8(n_samp, n_chan, seed) if kind == "u8" else W.gaussian_f32(n_chan, n_samp, seed)
    print(f"chunk groups {precision} {case}", flush=True)
    y, kernel, g = run(w, x, precision, mode)
    assert kernel == KERNEL[precision] and g.n_chunks > 24, (kernel, g.n_chunks)
    rows = sorted({0, 1, n_dm // 3, n_dm // 2, n_dm - 2, n_dm - 1})
    ref = O.fdd(x, kind, w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, L, mode=mode, rows=rows)
    raw = raw_start(kind, n_samp, L, int(g.stride), int(g.n_chunks), False)
    check_rows(y[rows], ref, TOL[precision], raw_from=raw,
               label=f"{precision} {g.n_chunks} chunks vs oracle rows {rows}")
    assert np.isfinite(y).all()


@pytest.fixture(scope="module")
def band_2p21():
    """The paper-shaped band at twice the length: 1024 channels x 2^21 8-bit samples x 2048 DMs,
    L = 2^16, 42 chunks, with three dispersed pulses."""
    w = W.paper_shaped_u8()
    w.n_samp = 1 << 21
    x = W.gaussian_u8(w.n_samp, w.n_chan, 5)
    for dm, t0 in ((100.0, 1 << 19), (450.0, 1 << 20), (900.0, 3 << 19)):
        offs = O.nearest_sample(O.delays([dm], w.freqs, w.ref_freq_mhz, w.tsamp_s))[0]
        W.inject_pulse_u8(x, offs, t0, 80.0)
    return w, x


@pytest.mark.parametrize("precision,mode", [("fp32", "exact"), ("fp16_split", "round")])
def test_paper_band_42_chunks(band_2p21, precision, mode):
    w, x = band_2p21
    print(f"paper band 2^21 samples, {precision} {mode}", flush=True)
    y, kernel, g = run(w, x, precision, mode)
    assert kernel == KERNEL[precision] and g.n_chunks == 42, (kernel, g.n_chunks)
    rows = [0, 1, 921, 1842, 2047]
    ref = O.fdd(x, "u8", w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len, mode=mode, rows=rows)
    check_rows(y[rows], ref, TOL[precision],
               raw_from=raw_start("u8", w.n_samp, w.chunk_len, int(g.stride), int(g.n_chunks), False),
               label=f"paper band 2^21 {precision} {mode} rows {rows}")
    assert np.isfinite(y).all()
    for trial, t0 in ((205, 1 << 19), (921, 1 << 20), (1842, 3 << 19)):
        win = y[:, t0 - 2: t0 + 3].max(axis=1)
        assert abs(int(np.argmax(win)) - trial) <= 2, (trial, int(np.argmax(win)))
