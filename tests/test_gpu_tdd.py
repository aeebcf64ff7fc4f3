"""GPU parity of the brute-force time-domain dedispersion kernel (Eq. 2, fdd_tdd_execute).

With nearest-sample delays the oracle's time-domain shift-and-sum is the definition.  8-bit
sums are integers below 2^24 and must match the oracle bit for bit; float sums are checked to
float32 rounding.  Zero extension (chunked plans) and the circular convention (single-chunk
plans) are both covered, with ragged sample counts (the byte-wise load path), channel counts
that are not a multiple of the channel stage, DM counts that are not a multiple of the DM
tile, and the full paper-shaped workload on sampled rows.  The FDD path in ROUND mode must
agree with it to the FP32 bar.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity import check_rows, raw_start

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdd = pytest.importorskip("paper_2110_03482_amd")


def plan_of(w, mode="round", power_only=False):
    return fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, overlap=w.overlap,
                    single_chunk=w.single_chunk, input=w.input_kind, mode=mode, power_only=power_only)


def nearest(w):
    return O.nearest_sample(O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s))


CASES = [
    # seed, n_chan, n_samp, n_dm, L, single, kind, dm_max
    (1, 37, 20000, 45, 4096, False, "u8", 12.0),      # 37 channels, 45 DMs: partial stage and tile
    (2, 16, 30001, 9, 2048, False, "u8", 5.0),        # odd n_samp: byte-wise loads
    (3, 64, 9000, 64, 2048, False, "f32", 8.0),
    (4, 24, 4000, 33, 4096, True, "u8", 20.0),        # circular, n_samp < L
    (5, 40, 4096, 64, 4096, True, "f32", 30.0),       # circular, n_samp = L
    (6, 300, 5000, 17, 1024, False, "u8", 2.0),       # > 256 channels: u16 partial sums flushed
    (7, 20, 12000, 12, 8192, False, "u8", 60.0),      # coarse DM grid: wide windows
    (8, 21, 12000, 12, 8192, False, "f32", 60.0),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[1]}ch_{c[2]}s_{c[3]}dm_{'circ' if c[5] else 'zero'}_{c[6]}"
                                            for c in CASES])
def test_tdd_matches_oracle(case):
    seed, n_chan, n_samp, n_dm, L, single, kind, dm_max = case
    w = W.tiny_random(seed, n_chan, n_samp, n_dm, L, single_chunk=single, input_kind=kind, dm_max=dm_max)
    w = dataclasses.replace(w, dms=np.sort(w.dms))
    x = W.gaussian_u8(n_samp, n_chan, seed) if kind == "u8" else W.gaussian_f32(n_chan, n_samp, seed)
    print(f"tdd case {case}", flush=True)
    with plan_of(w) as p:
        y = p.tdd(torch.from_numpy(np.ascontiguousarray(x)).cuda())
        torch.cuda.synchronize()
        y = y.cpu().numpy()
    ref = O.tdd(x, kind, nearest(w), circular_len=L if single else None)
    if kind == "u8":
        assert np.array_equal(y.astype(np.float64), ref), f"max abs diff {np.abs(y - ref).max()}"
    else:
        check_rows(y, ref, 1e-6, label=f"tdd {case}")


@pytest.mark.parametrize("kind", ["u8", "f32"])
def test_tdd_equals_fdd_round(kind):
    w = W.tiny_random(9, 48, 40000, 50, 4096, single_chunk=False, input_kind=kind, dm_max=15.0)
    w = dataclasses.replace(w, dms=np.sort(w.dms))
    x = W.gaussian_u8(w.n_samp, w.n_chan, 9) if kind == "u8" else W.gaussian_f32(w.n_chan, w.n_samp, 9)
    with plan_of(w) as p:
        xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        yt = p.tdd(xd).cpu().numpy()
        yf = p.execute(xd).cpu().numpy()
    raw = raw_start(kind, w.n_samp, w.chunk_len, int(p.geometry.stride), int(p.geometry.n_chunks), False)
    check_rows(yf, yt, 1e-5, raw_from=raw, label=f"{kind}: FDD (round) vs TDD")


def test_tdd_paper_shaped_sampled_rows():
    w = W.paper_shaped_u8()
    x = W.gaussian_u8(w.n_samp, w.n_chan, 0)
    d = nearest(w)
    for dm, t0 in ((100.0, 1 << 18), (450.0, 1 << 19), (900.0, 3 << 18)):
        offs = O.nearest_sample(O.delays([dm], w.freqs, w.ref_freq_mhz, w.tsamp_s))[0]
        W.inject_pulse_u8(x, offs, t0, 80.0)
    print("tdd paper-shaped", flush=True)
    with plan_of(w, mode="exact", power_only=True) as p:
        y = p.tdd(torch.from_numpy(x).cuda())
        torch.cuda.synchronize()
        rows = [0, 205, 921, 1842, 2047]
        yr = y[rows].cpu().numpy()
        for trial, t0 in ((205, 1 << 18), (921, 1 << 19), (1842, 3 << 18)):
            assert int(torch.argmax(y[:, t0])) == trial
    ref = O.tdd(x, "u8", d, rows=rows)
    assert np.array_equal(yr.astype(np.float64), ref)


def test_tdd_rejects_wide_dm_steps():
    w = W.tiny_random(3, 16, 5000, 3, 2048, single_chunk=False, input_kind="f32", dm_max=3.0)
    w = dataclasses.replace(w, dms=np.array([0.0, 150.0, 300.0]))   # delays of one tile spread > 4088 samples
    w = dataclasses.replace(w, chunk_len=1 << 14)
    with plan_of(w) as p:
        with pytest.raises(fdd.FddError) as e:
            p.tdd(torch.zeros((w.n_chan, w.n_samp), dtype=torch.float32, device="cuda"))
        assert e.value.status == 3
