"""CPU checks of the parity helpers: defects that a row norm misses must fail them."""
import numpy as np
import pytest

from parity import check_power, check_rows, f32_rounding_rms, raw_start


def _row_8bit_like(n=1 << 16, seed=0):
    # a dedispersed 8-bit row at 1024 channels: offset 128 x 1024, fluctuations 16 sqrt(1024)
    rng = np.random.default_rng(seed)
    return 131072.0 + 512.0 * rng.standard_normal(n)


def test_clean_row_passes():
    ref = _row_8bit_like()
    y = (ref + 512.0 * 2e-7 * np.random.default_rng(1).standard_normal(ref.size)).astype(np.float32)
    st = check_rows(y[None], ref[None], 1e-5)
    assert st.rel < 1e-6 and st.centred < 1e-5


def test_seam_defect_hidden_by_row_norm_fails():
    ref = _row_8bit_like(1 << 20)
    y = ref.copy()
    y[51040 - 4: 51040 + 4] += 300.0          # a bad seam of 8 samples in a 2^20-sample row
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-5   # the plain row norm misses it
    with pytest.raises(AssertionError):
        check_rows(y[None], ref[None], 1e-5)


def test_spread_offset_hidden_by_row_norm_fails_centred():
    ref = _row_8bit_like()
    y = ref + 23.0 * np.sign(np.sin(np.arange(ref.size)))   # 4.5 % of the fluctuations
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 2e-4
    with pytest.raises(AssertionError):
        check_rows(y[None], ref[None], 1e-5)


def test_raw_region_bound_is_confined():
    ref = _row_8bit_like()
    cut = ref.size - 4096
    y = ref.copy()
    y[cut:] += 0.3 * np.random.default_rng(2).standard_normal(4096)   # raw-chunk rounding level
    check_rows(y[None], ref[None], 1e-5, raw_from=cut)
    with pytest.raises(AssertionError):
        check_rows(y[None], ref[None], 1e-5)                             # not allowed elsewhere
    y2 = y.copy()
    y2[cut - 1] += 2.0                                                   # just before the raw region
    with pytest.raises(AssertionError):
        check_rows(y2[None], ref[None], 1e-5, raw_from=cut)


def test_float32_storage_floor():
    ref = _row_8bit_like()
    fl = f32_rounding_rms(ref)
    assert 0.002 < fl < 0.005                          # ulp 2^-7 .. 2^-6 near 2^17, / sqrt(12)
    y = ref.astype(np.float32)                         # the best float32 answer passes
    check_rows(y[None], ref[None], 1e-5)


def test_raw_start_geometry():
    # paper-shaped: 2^20 samples, L = 2^16, S = 51040: chunks 0..19 are whole, chunk 20 is raw
    assert raw_start("u8", 1 << 20, 1 << 16, 51040, 21, False) == 20 * 51040
    assert raw_start("u8", 1 << 20, 1 << 16, 51040, 21, False, factor=4) == 20 * 51040 // 4
    assert raw_start("f32", 1 << 20, 1 << 16, 51040, 21, False) is None
    assert raw_start("u8", 4000, 4096, 4096, 1, True) == 0
    assert raw_start("u8", 4096, 4096, 4096, 1, True) is None
    assert raw_start("u8", 3000, 4096, 2000, 2, False) == 0


def test_power_check_catches_a_bad_bin():
    rng = np.random.default_rng(3)
    ref = rng.exponential(100.0, size=(2, 4096))
    P = ref * (1 + 1e-7 * rng.standard_normal(ref.shape))
    check_power(P, ref, 1e-5)
    P[1, 77] *= 1.01
    with pytest.raises(AssertionError):
        check_power(P, ref, 1e-5)


def test_power_check_scales_with_the_bin():
    # a bin holding a large coherent power is held to its own size: 2e-7 relative there passes,
    # while the same absolute error in a typical bin fails
    rng = np.random.default_rng(4)
    ref = rng.exponential(1e9, size=(1, 8192))
    ref[0, 0] = 3.7e14
    P = ref.copy()
    P[0, 0] *= 1 + 2e-7
    check_power(P, ref, 1e-5)
    P = ref.copy()
    P[0, 5] += 3.7e14 * 2e-7
    with pytest.raises(AssertionError):
        check_power(P, ref, 1e-5)
