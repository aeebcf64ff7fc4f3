"""GPU parity of down-sampled output (Sec. 2.2: a shorter inverse transform for DMs whose
smearing spans several samples) against the FP64 oracle, row by row.

Tolerances as in the full-resolution parity tests (1e-5 per row, element by element through
`parity.check_rows`: row norm, centred norm, per-sample bound, and the raw-region rule for
8-bit chunks past the end of the data).  The oracle evaluates the same definition, the
length-L/d real inverse of bins 0 .. L/(2d) scaled by 1/L, in float64.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from parity import check_rows, raw_start_of

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdd = pytest.importorskip("paper_2110_03482_amd")

TOL = 1e-5


def make_input(w, seed):
    if w.input_kind == "u8":
        return W.gaussian_u8(w.n_samp, w.n_chan, seed)
    return W.gaussian_f32(w.n_chan, w.n_samp, seed)


def run(w, x, mode, precision, factors):
    with fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, overlap=w.overlap,
                  single_chunk=w.single_chunk, input=w.input_kind, precision=precision, mode=mode,
                  downsample=factors) as p:
        out = p.execute(torch.from_numpy(np.ascontiguousarray(x)).cuda())
        torch.cuda.synchronize()
        flat = out.cpu().numpy()
        off = p.output_offsets()
        rows = [flat[off[j]: off[j + 1]] if p.downsampled else flat[j] for j in range(w.n_dm)]
        return rows, p.geometry, p.kernel


def check(w, x, mode, rows, g, factors, label, tol=TOL):
    ref = O.fdd(x, w.input_kind, w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len, overlap=int(g.overlap),
                single_chunk=w.single_chunk, mode=mode, factors=factors)
    raw = [raw_start_of(w.input_kind, g, w.n_samp, w.single_chunk, int(factors[j])) for j in range(w.n_dm)]
    check_rows(list(rows), list(ref), tol, raw_from=raw, label=label)


CASES = [
    # label, (n_chan, n_samp, n_dm, L, single, kind, dm_max), mode, precision, factor pattern
    ("chunked_f32_fp32", (16, 20000, 40, 2048, False, "f32", 10.0), "exact", "fp32", [1] * 10 + [2] * 10 + [4] * 10 + [8] * 10),
    ("chunked_u8_f16split", (32, 30001, 24, 4096, False, "u8", 25.0), "exact", "fp16_split",
     [2] * 6 + [1] * 6 + [16] * 6 + [4] * 6),
    ("chunked_f32_bf16split_round", (13, 9001, 18, 1024, False, "f32", 3.0), "round", "bf16_split",
     [1, 1, 2, 2, 2, 4, 4, 4, 4, 8, 8, 8, 16, 16, 16, 16, 16, 16]),
    ("single_u8_full_valu", (8, 4096, 9, 4096, True, "u8", 20.0), "round", "fp32", [1, 2, 4, 8, 16, 32, 64, 64, 1]),
    ("single_f32_ragged_bf16", (12, 3000, 5, 4096, True, "f32", 15.0), "exact", "bf16_split", [4] * 5),
    ("chunked_f32_one_segment", (24, 70000, 33, 8192, False, "f32", 40.0), "exact", "fp32", [2] * 33),
    ("chunked_f32_shortest", (5, 2000, 3, 128, False, "f32", 0.05), "exact", "fp32", [2, 1, 2]),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_downsampled_matches_oracle(case):
    label, shape, mode, precision, factors = case
    n_chan, n_samp, n_dm, L, single, kind, dm_max = shape
    w = W.tiny_random(len(label), n_chan, n_samp, n_dm, L, single, kind, dm_max=dm_max)
    x = make_input(w, 3)
    print(f"{label}: {shape} {mode} {precision} factors {sorted(set(factors))}", flush=True)
    rows, g, kernel = run(w, x, mode, precision, np.asarray(factors, dtype=np.int32))
    print(f"{label}: kernel {kernel}, overlap {g.overlap}, chunks {g.n_chunks}, segments {g.n_segments}", flush=True)
    check(w, x, mode, rows, g, factors, label)


def test_downsampled_linear_increments(monkeypatch):
    """A uniform DM grid with exact delays on the direct FP32 kernel with per-channel linear
    increments (FDD_PHASE_TABLE=linear): each segment's trials are offset by its first DM index."""
    import dataclasses
    w = W.tiny_random(43, 16, 20000, 40, 2048, False, "f32", dm_max=10.0)
    w = dataclasses.replace(w, dms=np.linspace(0.0, 10.0, 40))
    x = make_input(w, 5)
    factors = np.asarray([1] * 10 + [2] * 10 + [4] * 10 + [8] * 10, dtype=np.int32)
    monkeypatch.setenv("FDD_PHASE_TABLE", "linear")
    rows, g, kernel = run(w, x, "exact", "fp32", factors)
    assert kernel == "mfma_f32" and g.n_segments == 4
    check(w, x, "exact", rows, g, factors, "linear increments, 4 segments")


def test_factor_one_everywhere_is_bitwise_full_resolution():
    w = W.tiny_random(41, 16, 20000, 40, 2048, False, "u8", dm_max=10.0)
    x = make_input(w, 4)
    rows, g, _ = run(w, x, "exact", "fp32", np.ones(w.n_dm, dtype=np.int32))
    full, g2, _ = run(w, x, "exact", "fp32", None)
    assert g.n_segments == 1 and g.out_samples == w.n_dm * w.n_samp
    for j in range(w.n_dm):
        assert np.array_equal(rows[j], full[j])


def test_downsampled_pulse_peaks_at_its_dm_and_time():
    w = W.small_fp32()
    x = W.gaussian_f32(w.n_chan, w.n_samp, 9)
    dm_true, t0, width = 30.0, 1000, 8
    offs = O.nearest_sample(O.delays([dm_true], w.freqs, w.ref_freq_mhz, w.tsamp_s))[0]
    for k in range(width):
        W.inject_pulse_f32(x, offs, t0 + k, 2.0, circular=True)
    factors = fdd.fdd_smearing_factors(w.freqs, w.tsamp_s, w.dms, 8)
    factors = np.maximum(factors, 4).astype(np.int32)    # every row down-sampled by 4 or more
    rows, g, _ = run(w, x, "exact", "fp32", factors)
    j_true = int(np.argmin(np.abs(w.dms - dm_true)))
    peak = [float(r.max()) for r in rows]
    assert abs(int(np.argmax(peak)) - j_true) <= 2
    d = int(factors[j_true])
    assert abs(int(np.argmax(rows[j_true])) - (t0 + width // 2) // d) <= 1
    check(w, x, "exact", rows, g, factors, "small workload, smearing factors")


@pytest.mark.slow
def test_paper_shaped_downsampled_sampled_rows():
    """The paper-shaped workload (1024 channels, 2^20 8-bit samples, 2048 DMs) with the
    smearing factors bench.py uses (1 .. 16): sampled rows from every segment against the
    oracle, which computes them one by one."""
    w = W.paper_shaped_u8()
    x = W.gaussian_u8(w.n_samp, w.n_chan, 0)
    factors = fdd.fdd_smearing_factors(w.freqs, w.tsamp_s, w.dms, 16)
    print(f"paper-shaped, factors {np.unique(factors, return_counts=True)}", flush=True)
    with fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, input="u8",
                  downsample=factors) as p:
        flat = p.execute(torch.from_numpy(x).cuda())
        torch.cuda.synchronize()
        off = p.output_offsets()
        flat = flat.cpu().numpy()
        g = p.geometry
    sample = []
    for d in np.unique(factors):
        idx = np.nonzero(factors == d)[0]
        sample += [int(idx[0]), int(idx[-1])]
    ref = O.fdd(x, "u8", w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len, overlap=int(g.overlap),
                mode="exact", rows=sample, factors=factors)
    rows = [flat[off[j]: off[j + 1]] for j in sample]
    raw = [raw_start_of("u8", g, w.n_samp, False, int(factors[j])) for j in sample]
    check_rows(rows, list(ref), TOL, raw_from=raw, label=f"paper-shaped down-sampled rows {sample}")
