"""C-ABI checks that need no GPU: exported symbols, dry-run planning, validation errors.

The planner's float64 delays and chunk geometry are compared with the oracle's own
implementation of Eq. 1 and the Sec. 2.2 discard rule.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import workloads as W

fdd = pytest.importorskip("paper_2110_03482_amd")

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fdd.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = fdd.library()
    declared = _declared_functions()
    assert "fdd_plan" in declared and "fdd_execute" in declared and "fdd_power_spectrum" in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(fdd.exported_symbols()) >= set(declared)
    assert fdd.fdd_version().startswith("fdd-gfx950")


def _dry(w, **kw):
    args = dict(overlap=w.overlap, single_chunk=w.single_chunk, input=w.input_kind, dry_run=True)
    args.update(kw)
    return fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, **args)


@pytest.mark.parametrize("maker", [W.small_fp32, W.paper_shaped_u8, W.periodicity])
def test_dry_run_delays_equal_oracle(maker):
    w = maker()
    p = _dry(w) if w.chunk_len <= (1 << 16) else None
    tau_o = O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s)
    one = fdd.fdd_dispersion_delays(w.freqs, w.ref_freq_mhz, w.tsamp_s, float(w.dms[-1]))
    np.testing.assert_array_equal(one, tau_o[-1])
    if p is None:
        return
    tau = p.delays()
    np.testing.assert_array_equal(tau, tau_o)
    np.testing.assert_array_equal(O.nearest_sample(tau), O.nearest_sample(tau_o))
    p.close()


def test_dry_run_geometry_paper_shaped():
    w = W.paper_shaped_u8()
    p = _dry(w)
    g = p.geometry
    tau = O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s)
    S, n, D = O.chunk_geometry(w.n_samp, w.chunk_len, 0, False, float(tau.max()))
    assert (g.stride, g.n_chunks, g.overlap) == (S, n, D)
    assert g.n_bins == w.chunk_len // 2 + 1
    assert g.bins_padded % 64 == 0 and g.bins_padded >= g.n_bins
    assert g.max_delay == pytest.approx(float(tau.max()), rel=0, abs=0)
    assert g.n_valid == w.n_samp - int(np.ceil(tau.max()))
    # X (c64) + two Y planes (f32) + transposed input + phase table (16 B per channel and DM)
    expect = (w.n_chan * n * g.bins_padded * 8 + 2 * w.n_dm * n * g.bins_padded * 4 + w.n_chan * w.n_samp
              + 16 * w.n_chan * w.n_dm)
    assert expect <= g.workspace_bytes < expect + (1 << 24)
    assert p.kernel == "mfma_f32" and p.factors == (0, 0, 0)      # FP32: direct kernel by default
    p.close()
    # uniform grid, exact delays, 21 chunks, split precision: DM-factorised chunked kernels, 16
    # fine trials per coarse row (128 rows), 7 tiles per column group (3 groups of 112 columns)
    p = _dry(w, precision="fp16_split")
    assert p.kernel == "facw_f16_split" and p.factors == (16, 128, 7)
    p.close()
    os.environ["FDD_FACTOR"] = "wide"
    try:
        p = _dry(w)
        assert p.kernel == "facw_f32" and p.factors == (16, 128, 7)
        p.close()
    finally:
        del os.environ["FDD_FACTOR"]


@pytest.mark.parametrize("seed", range(6))
def test_dry_run_geometry_random(seed):
    rng = np.random.default_rng(seed)
    L = int(2 ** rng.integers(8, 14))
    w = W.tiny_random(seed, n_chan=int(rng.integers(1, 40)), n_samp=int(rng.integers(100, 20000)),
                      n_dm=int(rng.integers(1, 50)), chunk_len=L, single_chunk=False, dm_max=float(rng.uniform(0.5, 5)))
    tau = O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s)
    try:
        S, n, D = O.chunk_geometry(w.n_samp, L, 0, False, float(tau.max()))
    except ValueError:
        with pytest.raises(fdd.FddError):
            _dry(w)
        return
    g = _dry(w).geometry
    assert (g.stride, g.n_chunks, g.overlap) == (S, n, D)


def _desc_kwargs():
    w = W.small_fp32()
    return w, dict(input="f32", dry_run=True)


def test_validation_errors():
    w = W.paper_shaped_u8()
    with pytest.raises(fdd.FddError) as e:
        _dry(w, overlap=14000)
    assert e.value.status == 2                                     # FDD_E_OVERLAP
    with pytest.raises(fdd.FddError) as e:
        fdd.Plan(w.freqs, 1400.0, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, dry_run=True)
    assert e.value.status == 1 and "reference" in str(e.value)
    with pytest.raises(fdd.FddError) as e:
        fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, 3000, dry_run=True)
    assert e.value.status == 1
    with pytest.raises(fdd.FddError) as e:
        fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, 1 << 23, dry_run=True)
    assert e.value.status == 3
    with pytest.raises(fdd.FddError) as e:
        fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, 5000, 4096, single_chunk=True, dry_run=True)
    assert e.value.status == 1
    with pytest.raises(fdd.FddError) as e:
        fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, np.array([1.0, -2.0]), w.n_samp, w.chunk_len, dry_run=True)
    assert e.value.status == 1
    with pytest.raises(fdd.FddError) as e:
        fdd.Plan(w.freqs, w.ref_freq_mhz, -1.0, w.dms, w.n_samp, w.chunk_len, dry_run=True)
    assert e.value.status == 1
    with pytest.raises(fdd.FddError) as e:
        fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, 1 << 16, overlap=1 << 16, dry_run=True)
    assert e.value.status == 2


def test_null_and_dry_run_execution_rejected():
    lib = fdd.library()
    assert lib.fdd_plan(None, None) == 1
    assert lib.fdd_execute(None, None, None, None) == 1
    assert lib.fdd_plan_info(None, None) == 1
    assert lib.fdd_destroy(None) == 0
    w = W.small_fp32()
    p = _dry(w)
    st = lib.fdd_execute(p.handle, ctypes.c_void_p(16), ctypes.c_void_p(16), None)
    assert st == 1 and "dry-run" in fdd.fdd_last_error()
    assert lib.fdd_set_workspace(p.handle, ctypes.c_void_p(256), ctypes.c_size_t(1 << 30)) == 1
    p.close()
    assert fdd.fdd_status_string(2).startswith("overlap")


def test_kernel_selection():
    w = W.small_fp32()
    # one chunk, uniform DMs, exact delays: the DM-factorised matrix-core kernels
    assert _dry(w).kernel == "fac_f32"
    assert _dry(w, precision="fp16_split").kernel == "fac_f16_split"
    assert _dry(w, mode="round").kernel == "valu"        # nearest-sample delays do not factorise
    w2 = W.tiny_random(1, 16, 5000, 8, 1024, False, dm_max=3.0)
    p = _dry(w2)                                         # random (non-uniform) DMs
    assert p.geometry.n_chunks >= 3 and p.kernel == "mfma_f32"
    w3 = W.paper_shaped_u8()
    assert _dry(w3).kernel == "mfma_f32"                 # 21 chunks, FP32: direct kernel
    assert _dry(w3, precision="fp16_split").kernel == "facw_f16_split"   # split: chunked factorised
    assert _dry(w3, precision="bf16_split").kernel == "facw_bf16_split"
    assert _dry(w3, precision="fp16_split", mode="round").kernel == "mfma_f16_split"   # rounding does not factorise
    assert _dry(w3, precision="fp16_split", power_only=True).kernel == "mfma_f16_split"   # needs the Y buffer
    assert _dry(w3, mode="round").factors == (0, 0, 0)
    os.environ["FDD_FACTOR"] = "direct"
    try:
        assert _dry(w3, precision="fp16_split").kernel == "mfma_f16_split"
    finally:
        del os.environ["FDD_FACTOR"]


def test_chunked_factorised_selection():
    """Chunked plans on uniform grids with exact delays take the DM-factorised chunked kernels in
    split precision at any chunk count, with a column-group width of 4 to 7 tiles (the planner
    weighs the measured time per tile against the padding of the last group)."""
    import dataclasses
    seen, chunks = set(), []
    for n_samp in (21900, 15000, 9000, 40000, 90000):
        w = W.tiny_random(11, 48, n_samp, 2048, 2048, single_chunk=False, input_kind="f32")
        w = dataclasses.replace(w, dms=np.linspace(0.0, 40.0, 2048))
        p = _dry(w, precision="fp16_split")
        assert p.kernel == "facw_f16_split" and p.factors[0] in (8, 16), (n_samp, p.kernel)
        assert 4 <= p.factors[2] <= 7
        seen.add(p.factors[2])
        chunks.append(int(p.geometry.n_chunks))
        p.close()
        r = fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, input="f32",
                     precision="fp16_split", mode="round", dry_run=True) if n_samp <= 30000 else None
        if r is not None:
            assert r.kernel == "mfma_f16_split"
            r.close()
    assert 7 in seen and max(chunks) > 24, (seen, chunks)


def test_direct_kernels_take_any_chunk_count():
    """Plans that do not factorise (random DMs, or nearest-sample delays) stay on the direct
    matrix-core kernels above 24 chunks: those run over balanced groups of at most 24 chunks."""
    for n_samp in (60000, 90000, 140000):
        w = W.tiny_random(11, 48, n_samp, 256, 2048, single_chunk=False, input_kind="f32")   # random DMs
        assert _dry(w).kernel == "mfma_f32"
        for prec in ("fp16_split", "bf16_split"):
            p = _dry(w, precision=prec)
            assert p.geometry.n_chunks > 24 and p.kernel == ("mfma_f16_split" if prec == "fp16_split"
                                                               else "mfma_bf16_split"), (n_samp, prec, p.kernel)
            p.close()
        assert _dry(w, mode="round").kernel == "mfma_f32"


def test_direct_fp32_kernel_needs_a_small_descriptor_window():
    """The FP32 matrix-core kernel reads X through descriptors over the rows of up to 16 channels,
    which must stay below 2 GiB (16 x chunks x pitch x 8 bytes): a 2^24-sample band at
    L = 2^16 (329 chunks) fits, a 2^25-sample one (658 chunks) goes to the VALU kernel."""
    for log_n, kernel in ((24, "mfma_f32"), (25, "valu")):
        w = W.tiny_random(12, 16, 1 << log_n, 64, 1 << 16, single_chunk=False, input_kind="f32", dm_max=50.0)
        p = _dry(w)
        g = p.geometry
        assert p.kernel == kernel, (log_n, g.n_chunks, p.kernel)
        assert (16 * 8 * g.n_chunks * g.bins_padded <= 0x7fffffff) == (kernel == "mfma_f32")
        p.close()

def test_facw_gpu_cases_cover_the_tile_counts_in_use():
    """The factorised GPU parity cases (tests/test_gpu_facw.py) must reach every column-group width
    the planner picks for them: 4, 5 and 7 tiles of 32 columns (6 is never the cheapest)."""
    import dataclasses
    import test_gpu_facw as F
    seen = set()
    for seed, n_chan, n_samp, n_dm, L, kind, dm_hi in F.CASES:
        w = W.tiny_random(seed, n_chan, n_samp, n_dm, L, single_chunk=False, input_kind=kind)
        w = dataclasses.replace(w, dms=np.linspace(0.0, dm_hi, n_dm))
        p = _dry(w, mode="exact", precision="fp16_split")
        assert p.kernel == "facw_f16_split", (seed, p.kernel)
        seen.add(p.factors[2])
        p.close()
    assert {4, 5, 7} <= seen, seen

def test_batch_rejects_without_device_calls():
    lib = fdd.library()
    d = fdd.BatchDesc()
    out = ctypes.c_void_p()
    assert lib.fdd_batch_create(0, None, ctypes.byref(d), ctypes.byref(out)) == 1
    assert lib.fdd_batch_create(1, None, None, None) == 1
    w = W.small_fp32()
    p = _dry(w)
    with pytest.raises(fdd.FddError) as e:
        fdd.fdd_batch_create([p.handle], d)
    assert e.value.status == 1 and "dry-run" in str(e.value)
    d.flags = 1 << 9
    with pytest.raises(fdd.FddError) as e:
        fdd.fdd_batch_create([p.handle], d)
    assert e.value.status == 1 and "flags" in str(e.value)
    assert lib.fdd_batch_execute(None, None, None, None) == 1
    assert lib.fdd_batch_info(None, None, None, None) == 1
    assert lib.fdd_batch_destroy(None) == 0
    p.close()


# ----------------------------------------------------------------------------- down-sampled output (Sec. 2.2)

def test_downsampled_geometry_and_offsets():
    w = W.paper_shaped_u8()
    ds = np.ones(w.n_dm, dtype=np.int32)
    ds[100:300] = 4
    ds[300:] = 16
    ds[50] = 2                                           # runs need not be monotone
    p = _dry(w, downsample=ds)
    g = p.geometry
    assert (g.chunk_len - g.overlap) % 16 == 0 and g.stride % 16 == 0
    n_out = -(-w.n_samp // ds.astype(np.int64))
    assert g.out_samples == int(n_out.sum()) and p.downsampled
    assert g.n_segments == 5                             # 1 | 2 | 1 | 4 | 16
    off = p.output_offsets()
    np.testing.assert_array_equal(off, np.concatenate([[0], np.cumsum(n_out)]))
    assert p.kernel == "mfma_f32"
    p.close()
    flat = _dry(w, downsample=np.ones(w.n_dm, dtype=np.int32))
    assert not flat.downsampled and flat.geometry.n_segments == 1
    assert flat.geometry.out_samples == w.n_dm * w.n_samp
    flat.close()
    # ceil(max tau) = 14496 already leaves S = 51040 = 16 x 3190: the overlap stays
    assert _dry(w).geometry.overlap == 14496 and g.overlap == 14496


def test_downsampled_overlap_rounding_and_rejections():
    w = W.small_fp32()
    n = w.n_dm
    auto = fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, 20000, 4096, input="f32", dry_run=True,
                    downsample=np.full(n, 8, dtype=np.int32))
    base = fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, 20000, 4096, input="f32", dry_run=True)
    D0 = base.geometry.overlap
    assert auto.geometry.overlap == 4096 - (4096 - D0) // 8 * 8 and auto.geometry.stride % 8 == 0
    assert auto.kernel != "fac_f32"                      # the factorised tables serve one segment of factor 1
    cases = [
        (dict(downsample=np.full(n, 3, dtype=np.int32)), 1),             # not a power of two
        (dict(downsample=np.zeros(n, dtype=np.int32)), 1),               # below 1
        (dict(downsample=np.full(n, 4096 // 32, dtype=np.int32)), 1),    # L/d below 64
        (dict(downsample=np.full(n, 2, dtype=np.int32), power_only=True, single_chunk=True), 1),
        (dict(downsample=np.full(n, 8, dtype=np.int32), overlap=D0 + 1 if (4096 - D0 - 1) % 8 else D0 + 2), 1),
    ]
    for kw, status in cases:
        args = dict(input="f32", dry_run=True)
        args.update(kw)
        ns = 4096 if args.get("single_chunk") else 20000
        with pytest.raises(fdd.FddError) as e:
            fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, ns, 4096, **args)
        assert e.value.status == status, kw
    with pytest.raises(fdd.FddError) as e:              # shortened inverses use the one-workgroup transforms
        fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, 1 << 17, 1 << 17, single_chunk=True, input="f32",
                 dry_run=True, downsample=np.full(n, 2, dtype=np.int32))
    assert e.value.status == 3
    many = np.tile(np.array([1, 2], dtype=np.int32), 200)
    dms = np.linspace(0.0, 10.0, many.size)
    with pytest.raises(fdd.FddError) as e:
        fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, dms, 20000, 4096, input="f32", dry_run=True, downsample=many)
    assert e.value.status == 3 and "runs" in str(e.value)
    with pytest.raises(ValueError):
        fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, 20000, 4096, input="f32", dry_run=True,
                 downsample=np.ones(n + 1, dtype=np.int32))


def test_batch_rejects_downsampled_plans():
    w = W.small_fp32()
    p = _dry(w, downsample=np.full(w.n_dm, 2, dtype=np.int32))
    # planned without a device, so the batch stops at the dry-run check first; the factor
    # check sits behind it and is exercised on the GPU
    with pytest.raises(fdd.FddError):
        fdd.fdd_batch_create([p.handle], fdd.BatchDesc())
    p.close()


def test_smearing_factors():
    # two channels 1 MHz apart at 400.5 / 401.5 MHz: the lowest channel spans 400 .. 401 MHz
    freqs = np.array([401.5, 400.5])
    tsamp = 1e-4
    per_dm = 4.148808e3 * (1.0 / 400.0 ** 2 - 1.0 / 401.0 ** 2) / tsamp     # samples per unit DM
    dms = np.array([0.0, 0.99 / per_dm, 1.0 / per_dm * 1.000001, 3.99 / per_dm, 4.0 / per_dm * 1.000001,
                    1000.0 / per_dm])
    got = fdd.fdd_smearing_factors(freqs, tsamp, dms, 64)
    np.testing.assert_array_equal(got, [1, 1, 1, 2, 4, 64])
    np.testing.assert_array_equal(fdd.fdd_smearing_factors(freqs, tsamp, dms, 8), [1, 1, 1, 2, 4, 8])
    np.testing.assert_array_equal(fdd.fdd_smearing_factors([1400.0], tsamp, dms, 64), np.ones(6))
    w = W.paper_shaped_u8()
    f = fdd.fdd_smearing_factors(w.freqs, w.tsamp_s, w.dms, 16)
    assert f[0] == 1 and f[-1] == 16 and np.all(np.diff(f) >= 0)          # ascending DMs: runs ascend
    with pytest.raises(fdd.FddError):
        fdd.fdd_smearing_factors(freqs, tsamp, dms, 3)


# ----------------------------------------------------------------------------- scaled DMs (Sec. 2.3, Eq. 8)

def _scaled_shift(dms, f_lo, f_hi, r):
    """Largest |s* - j| over trials j and bins f_lo..f_hi of a block with reference bin r."""
    step = (dms[-1] - dms[0]) / (dms.size - 1)
    f = np.arange(f_lo, f_hi + 1, dtype=np.float64)
    ss = (dms[:, None] * f[None, :] / r - dms[0]) / step
    return float(np.abs(ss - np.arange(dms.size)[:, None]).max())


@pytest.mark.parametrize("n_dm,dm0,dm1,L", [(4096, 0.0, 500.0, 1 << 22), (64, 0.0, 30.0, 4096),
                                            (100, 20.0, 60.0, 8192), (3, 0.0, 1.0, 128)])
def test_scaled_first_bin_rule(n_dm, dm0, dm1, L):
    w = W.small_fp32()
    dms = np.linspace(dm0, dm1, n_dm)
    p = fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, dms, L, L, single_chunk=True, input="f32", dry_run=True,
                 power_only=True, scaled_dm=True)
    fmin = int(p.geometry.scaled_min_bin)
    assert fmin % 64 == 0 and 0 <= fmin <= L // 2
    if fmin < L // 2:
        assert _scaled_shift(dms, fmin, fmin + 63, fmin + 32) <= 31.0 + 1e-9
    assert fmin >= min(64, L // 2)                      # bin 0 always runs exactly
    if fmin > 64:
        assert _scaled_shift(dms, fmin - 64, fmin - 1, fmin - 32) > 31.0
    plain = fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, dms, L, L, single_chunk=True, input="f32", dry_run=True,
                     power_only=True)
    assert plain.geometry.scaled_min_bin == 0
    n_blocks = -(-(L // 2 - fmin) // 64)
    assert p.geometry.workspace_bytes >= plain.geometry.workspace_bytes + (n_dm + 64) * n_blocks * 64 * 4


def test_scaled_rejections():
    w = W.small_fp32()
    base = dict(input="f32", dry_run=True, scaled_dm=True)
    cases = [
        (dict(single_chunk=False), 20000, 4096, w.dms),                       # chunked
        (dict(single_chunk=True, mode="round"), 4096, 4096, w.dms),          # nearest-sample delays
        (dict(single_chunk=True), 64, 64, w.dms),                            # L below 128
        (dict(single_chunk=True), 4096, 4096, np.array([0.0, 1.0, 3.0])),    # not uniform
        (dict(single_chunk=True), 4096, 4096, np.array([5.0])),              # one DM
    ]
    for kw, ns, L, dms in cases:
        args = dict(base)
        args.update(kw)
        with pytest.raises(fdd.FddError) as e:
            fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, dms, ns, L, **args)
        assert e.value.status == 3, kw
