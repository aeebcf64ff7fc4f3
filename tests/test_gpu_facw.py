"""GPU parity of the chunked DM-factorised phasor sums (overlap-save plans, uniform DM grids,
exact delays).

Trial a B + b has the delay of coarse trial a plus that of fine offset b (Eq. 1 is linear in
DM), so per bin the sum is a matrix product with B x N (chunk, fine DM) columns.  These tests
run plans on which the planner picks those kernels (checked through the plan's factors) against
the FP64 oracle, which evaluates every phasor from its own delay, on sampled rows that include
the first and last fine trial of coarse rows, the edges of the 128-row tiles and the last
trial; and on every row against the direct kernels of the same plan (FDD_FACTOR=direct).
Covered: channel counts that are not a multiple of the 16-channel stage, DM counts that leave
a coarse row or a row tile partial, 8 and 16 fine trials, several column-group widths, 8-bit
input with a ragged last chunk, every precision.
"""
import dataclasses
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity import check_rows, raw_start

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdd = pytest.importorskip("paper_2110_03482_amd")

TOL = {"fp32": 1e-5, "fp16_split": 1e-5, "bf16_split": 1e-4}


def make(seed, n_chan, n_samp, n_dm, L, kind, dm_hi):
    w = W.tiny_random(seed, n_chan, n_samp, n_dm, L, single_chunk=False, input_kind=kind)
    w = dataclasses.replace(w, dms=np.linspace(0.0, dm_hi, n_dm))
    x = W.gaussian_u8(n_samp, n_chan, seed) if kind == "u8" else W.gaussian_f32(n_chan, n_samp, seed)
    return w, x


def plan(w, precision, factor=None):
    old = os.environ.get("FDD_FACTOR")
    if factor is None and precision == "fp32":
        factor = "wide"                                      # FP32 takes these kernels on request
    if factor is not None:
        os.environ["FDD_FACTOR"] = factor
    try:
        return fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, overlap=w.overlap,
                        single_chunk=False, input=w.input_kind, mode="exact", precision=precision)
    finally:
        if old is None:
            os.environ.pop("FDD_FACTOR", None)
        else:
            os.environ["FDD_FACTOR"] = old


def run(p, x):
    y = p.execute(torch.from_numpy(np.ascontiguousarray(x)).cuda())
    torch.cuda.synchronize()
    return y.cpu().numpy()


def sample_rows(n_dm, fine):
    rows = {0, 1, fine - 1, fine, 2 * fine - 1, n_dm // 2, n_dm - 2, n_dm - 1}
    for t in range(128 * fine, n_dm, 128 * fine):          # row-tile edges
        rows |= {t - 1, t}
    return sorted(r for r in rows if 0 <= r < n_dm)


CASES = [
    # seed, n_chan, n_samp, n_dm, L, kind, dm_hi      -> (fine, coarse, tiles), chunks
    (11, 48, 21900, 2048, 2048, "f32", 40.0),         # 16 fine, 1 row tile, 16 chunks
    (12, 37, 29000, 2000, 2048, "u8", 30.0),          # 37 channels, partial coarse row, ragged last chunk
    (13, 32, 30000, 3000, 2048, "f32", 20.0),         # 2 row tiles, the second partial
    (14, 40, 23000, 1024, 2048, "f32", 25.0),         # 8 fine trials per coarse row
    (15, 16, 50000, 2048, 4096, "u8", 60.0),          # 16 channels (one stage), L = 4096
    (16, 32, 59000, 2048, 2048, "u8", 40.0),          # 42 chunks (above the direct kernels' 24)
    (17, 24, 90000, 2048, 2048, "f32", 40.0),         # 64 chunks
    (18, 40, 5500, 2048, 2048, "f32", 40.0),          # 4 chunks: one group of 4 tiles
    (19, 24, 9000, 1024, 2048, "u8", 25.0),           # 6 chunks, 8 fine trials: 4 tiles, ragged 8-bit tail
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[1]}ch_{c[2]}s_{c[3]}dm_L{c[4]}_{c[5]}" for c in CASES])
@pytest.mark.parametrize("precision", ["fp32", "fp16_split", "bf16_split"])
def test_facw_matches_oracle_and_direct(case, precision):
    seed, n_chan, n_samp, n_dm, L, kind, dm_hi = case
    w, x = make(seed, n_chan, n_samp, n_dm, L, kind, dm_hi)
    with plan(w, precision) as p:
        fine, coarse, tiles = p.factors
        g = p.geometry
        print(f"facw {precision} {case}: kernel={p.kernel} factors={p.factors} chunks={g.n_chunks}", flush=True)
        assert p.kernel.startswith("facw_") and fine in (8, 16) and tiles > 0
        assert coarse == -(-n_dm // fine)
        y = run(p, x)
    raw = raw_start(kind, n_samp, L, int(g.stride), int(g.n_chunks), False)
    rows = sample_rows(n_dm, fine)
    ref = O.fdd(x, kind, w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, L, mode="exact", rows=rows)
    check_rows(y[rows], ref, TOL[precision], raw_from=raw, label=f"facw {precision} vs oracle rows {rows}")
    if precision != "fp32" and g.n_chunks > 24:
        return                                               # no direct split kernel for so many chunks
    with plan(w, precision, "direct") as pd:
        assert not pd.kernel.startswith("fac")
        yd = run(pd, x)
    check_rows(y, yd, 2 * TOL[precision], raw_from=raw, label=f"facw {precision} vs direct kernel, all rows")


def test_facw_paper_shaped_rows_split():
    """The paper-shaped workload (1024 ch, 2^20 8-bit samples, 2048 DMs, 21 chunks) on the
    chunked factorised kernels in FP16 split, against the oracle on sampled rows; pulses found."""
    w = W.paper_shaped_u8()
    x = W.gaussian_u8(w.n_samp, w.n_chan, 0)
    for dm, t0 in ((100.0, 1 << 18), (450.0, 1 << 19), (900.0, 3 << 18)):
        offs = O.nearest_sample(O.delays([dm], w.freqs, w.ref_freq_mhz, w.tsamp_s))[0]
        W.inject_pulse_u8(x, offs, t0, 80.0)
    with plan(w, "fp16_split") as p:
        assert p.kernel == "facw_f16_split" and p.factors == (16, 128, 7)
        g = p.geometry
        y = run(p, x)
    rows = [0, 15, 16, 921, 1842, 2047]
    ref = O.fdd(x, "u8", w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len, mode="exact", rows=rows)
    check_rows(y[rows], ref, TOL["fp16_split"], raw_from=raw_start("u8", w.n_samp, w.chunk_len, int(g.stride),
                                                                    int(g.n_chunks), False),
               label=f"facw fp16_split paper-shaped rows {rows}")
    assert np.isfinite(y).all()
    for trial, t0 in ((205, 1 << 18), (921, 1 << 19), (1842, 3 << 18)):
        assert abs(int(np.argmax(y[:, t0 - 2: t0 + 3].max(axis=1))) - trial) <= 2
