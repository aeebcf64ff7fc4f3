"""Pins of the FP64 oracle to facts fixed by physics, closed forms and brute force (CPU only).

Each test names the passage of the paper it checks.  None of them re-types the oracle's own
formula: they use physical constants, analytic sums, direct O(L^2) definitions or explicit
loops, chosen so that a dropped term, a flipped sign, a wrong index or a transposed operand
in the oracle fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W


GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- Eq. 1 (Sec. 2.1)

def test_dispersion_constant_from_physical_constants():
    """Eq. 1: k_DM = e^2 / (2 pi m_e c), expressed in MHz^2 pc^-1 cm^3 s (CODATA 2018)."""
    with open(os.path.join(GOLDEN, "physical_constants.json")) as fh:
        pc = json.load(fh)
    e, me, c, parsec = (pc["electron_charge_esu"], pc["electron_mass_g"],
                        pc["speed_of_light_cm_s"], pc["parsec_cm"])
    k_cgs = e * e / (2.0 * math.pi * me * c)          # s Hz^2 cm^2 (per cm^-2 column)
    k_mhz = k_cgs * parsec / 1e12                      # per (pc cm^-3), MHz^2
    # The literature value 4.148808e3 was derived from older constants; CODATA 2018 gives
    # 4148.8064, 3.8e-7 below it.  The paper's rounded (2.41e-4)^-1 is 1.4e-4 off and fails.
    assert abs(k_mhz - O.K_DM) / O.K_DM < 1e-6


def test_delay_equals_cold_plasma_group_delay():
    """Eq. 1 against the group delay of a cold-plasma slab, integrated from v_g = c sqrt(1 - nu_p^2/nu^2).

    Pins the nu^-2 law, the constant and the sign (lower frequencies arrive later).
    """
    with open(os.path.join(GOLDEN, "physical_constants.json")) as fh:
        pc = json.load(fh)
    e, me, c, parsec = (pc["electron_charge_esu"], pc["electron_mass_g"],
                        pc["speed_of_light_cm_s"], pc["parsec_cm"])
    n_e = 0.03            # cm^-3
    length_pc = 1000.0    # slab thickness
    dm = n_e * length_pc  # pc cm^-3
    nu_p2 = n_e * e * e / (math.pi * me)   # plasma frequency squared, Hz^2
    ell = length_pc * parsec

    def travel_excess(nu_hz):
        # ell / v_g - ell / c, computed without cancellation
        x = nu_p2 / (nu_hz * nu_hz)
        return (ell / c) * math.expm1(-0.5 * math.log1p(-x))

    freqs = np.array([1250.3, 1333.0, 1400.0, 1499.9])
    ref = 1550.0
    tsamp = 64e-6
    tau = O.delays([dm], freqs, ref, tsamp)[0]
    for f, t in zip(freqs, tau):
        want = (travel_excess(f * 1e6) - travel_excess(ref * 1e6)) / tsamp
        assert want > 0
        assert abs(t - want) / want < 1e-6


def test_nearest_sample_rule():
    """Sec. 2.1: shifts go to the nearest sample; halves round up (reading)."""
    got = O.nearest_sample(np.array([0.0, 0.49999, 0.5, 1.5, 2.4, 2.5, 2.6, 14495.9958]))
    assert got.tolist() == [0, 0, 1, 2, 2, 3, 3, 14496]


def test_chunk_geometry_paper_shaped():
    """Sec. 2.2 wrap/discard: 1024 ch 1250-1550 MHz, 64 us, DM <= 1000, L = 2^16 -> D = 14496."""
    w = W.paper_shaped_u8()
    tau = O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s)
    S, n, D = O.chunk_geometry(w.n_samp, w.chunk_len, 0, False, float(tau.max()))
    assert (S, n, D) == (51040, 21, 14496)
    with pytest.raises(ValueError):
        O.chunk_geometry(w.n_samp, w.chunk_len, 14000, False, float(tau.max()))
    with pytest.raises(ValueError):
        O.chunk_geometry(5000, 4096, 0, True, 10.0)
    with pytest.raises(ValueError):
        O.chunk_geometry(5000, 3000, 0, False, 10.0)


# ----------------------------------------------------------------------------- Eq. 3 / Eq. 6 steps

@pytest.mark.parametrize("L", [8, 64, 256, 1024])
def test_forward_step_is_the_dft(L):
    """Eq. 3 on a chunk: the FFT step equals the direct O(L^2) sum."""
    rng = np.random.default_rng(L)
    seg = rng.standard_normal((3, L))
    np.testing.assert_allclose(O.forward_spectra(seg), O.direct_rdft(seg), rtol=0, atol=1e-10 * L)


@pytest.mark.parametrize("L", [8, 64, 512])
def test_inverse_step_is_the_explicit_formula(L):
    """Eq. 6 inverse: drops Im of bins 0 and L/2 and scales by 1/L, as the written-out sum."""
    rng = np.random.default_rng(L + 1)
    Y = rng.standard_normal((4, L // 2 + 1)) + 1j * rng.standard_normal((4, L // 2 + 1))
    np.testing.assert_allclose(O.inverse_real(Y, L), O.explicit_irdft(Y, L), rtol=0, atol=1e-12)


def test_inverse_undoes_forward():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((5, 4096))
    np.testing.assert_allclose(O.inverse_real(O.forward_spectra(x), 4096), x, atol=1e-12)


# ----------------------------------------------------------------------------- closed forms, Eqs. 3-7

def _tone_problem(L, n_samp, k0, seed, n_chan=7, n_dm=5):
    rng = np.random.default_rng(seed)
    freqs = np.sort(rng.uniform(1200.0, 1500.0, n_chan))
    dms = rng.uniform(0.0, 30.0, n_dm)
    theta = rng.uniform(0, 2 * np.pi, n_chan)
    t = np.arange(n_samp)
    x = np.cos(2 * np.pi * k0 * t[None, :] / L + theta[:, None]).astype(np.float64)
    return freqs, dms, theta, x


@pytest.mark.parametrize("k0", [1, 5, 333, 1023])
def test_tone_closed_form_single_chunk(k0):
    """Eqs. 3-7, fractional delays: a tone at bin k0 comes out advanced by tau, summed over channels."""
    L = 2048
    freqs, dms, theta, x = _tone_problem(L, L, k0, seed=k0)
    tau = O.delays(dms, freqs, 1500.0, 64e-6)
    assert np.any(np.abs(tau - np.rint(tau)) > 0.1)          # genuinely fractional
    y = O.oracle_fdd_rows(x, "f64", tau, L, L, 1, True, "exact")
    t = np.arange(L)
    want = np.cos(2 * np.pi * k0 * (t[None, None, :] + tau[:, :, None]) / L
                  + theta[None, :, None]).sum(axis=1)
    np.testing.assert_allclose(y, want, atol=1e-9)


def test_tone_closed_form_chunked():
    """Overlap-save chunks that lie inside the data reproduce the tone closed form exactly."""
    L, k0 = 1024, 37
    n_samp = 5000
    freqs, dms, theta, x = _tone_problem(L, n_samp, k0, seed=3)
    tau = O.delays(dms, freqs, 1500.0, 64e-6)
    S, n_chunks, D = O.chunk_geometry(n_samp, L, 0, False, float(tau.max()))
    y = O.oracle_fdd_rows(x, "f64", tau, L, S, n_chunks, False, "exact")
    t = np.arange(n_samp)
    want = np.cos(2 * np.pi * k0 * (t[None, None, :] + tau[:, :, None]) / L
                  + theta[None, :, None]).sum(axis=1)
    inside = np.zeros(n_samp, dtype=bool)
    for k in range(n_chunks):
        if k * S + L <= n_samp:
            inside[k * S: k * S + S] = True
    assert inside.sum() > 2 * S
    np.testing.assert_allclose(y[:, inside], want[:, inside], atol=1e-9)


# ----------------------------------------------------------------------------- down-sampled inverse, Sec. 2.2

@pytest.mark.parametrize("d,k0", [(2, 1), (2, 255), (4, 100), (8, 63), (16, 3)])
def test_downsampled_tone_closed_form_single_chunk(d, k0):
    """A tone below the shortened band (k0 < L/(2d)) comes out advanced by tau and sampled
    every d-th sample, with its full amplitude (the 1/L scaling)."""
    L = 2048
    assert k0 < L // (2 * d)
    freqs, dms, theta, x = _tone_problem(L, L, k0, seed=10 + k0)
    tau = O.delays(dms, freqs, 1500.0, 64e-6)
    z = O.oracle_fdd_rows(x, "f64", tau, L, L, 1, True, "exact", factors=[d] * len(dms))
    m = np.arange(L // d)
    want = np.cos(2 * np.pi * k0 * (d * m[None, None, :] + tau[:, :, None]) / L
                  + theta[None, :, None]).sum(axis=1)
    for i in range(len(dms)):
        assert z[i].shape == (L // d,)
        np.testing.assert_allclose(z[i], want[i], atol=1e-9)


@pytest.mark.parametrize("d", [2, 4, 8])
def test_downsampled_tone_closed_form_chunked(d):
    """Overlap-save with a kept stride that is a multiple of d: chunks inside the data give
    the closed form at every d-th sample; the rows hold ceil(n_samp / d) samples."""
    L, k0 = 1024, 21
    n_samp = 5001
    freqs, dms, theta, x = _tone_problem(L, n_samp, k0, seed=4)
    tau = O.delays(dms, freqs, 1500.0, 64e-6)
    S, n_chunks, D = O.chunk_geometry(n_samp, L, 0, False, float(tau.max()), d)
    assert S % d == 0 and D >= np.ceil(tau.max())
    z = O.oracle_fdd_rows(x, "f64", tau, L, S, n_chunks, False, "exact", factors=[d] * len(dms))
    n_out = -(-n_samp // d)
    m = np.arange(n_out)
    want = np.cos(2 * np.pi * k0 * (d * m[None, None, :] + tau[:, :, None]) / L
                  + theta[None, :, None]).sum(axis=1)
    inside = np.zeros(n_out, dtype=bool)
    for k in range(n_chunks):
        if k * S + L <= n_samp:
            inside[k * S // d: (k + 1) * S // d] = True
    assert inside.sum() >= 2 * S // d
    for i in range(len(dms)):
        assert z[i].shape == (n_out,)
        np.testing.assert_allclose(z[i][inside], want[i][inside], atol=1e-9)


def test_downsampled_equals_decimated_full_resolution_when_band_limited():
    """Random spectra confined to bins 1 .. L/(2d) - 1: the shortened inverse is exactly every
    d-th sample of the full-resolution series, for mixed factors in one DM list."""
    L, d_list = 1024, [1, 2, 2, 8, 4, 1]
    rng = np.random.default_rng(5)
    n_chan = 6
    spec = np.zeros((n_chan, L // 2 + 1), dtype=np.complex128)
    top = L // (2 * max(d_list))
    spec[:, 1:top] = rng.standard_normal((n_chan, top - 1)) + 1j * rng.standard_normal((n_chan, top - 1))
    x = np.fft.irfft(spec, n=L, axis=-1)
    freqs = np.sort(rng.uniform(1200.0, 1500.0, n_chan))
    dms = rng.uniform(0.0, 20.0, len(d_list))
    tau = O.delays(dms, freqs, 1500.0, 64e-6)
    full = O.oracle_fdd_rows(x, "f64", tau, L, L, 1, True, "exact")
    z = O.oracle_fdd_rows(x, "f64", tau, L, L, 1, True, "exact", factors=d_list)
    for i, d in enumerate(d_list):
        np.testing.assert_allclose(z[i], full[i][::d], atol=1e-12 * np.abs(full[i]).max())


def test_downsampled_cutoff_bin_half_weight_and_above_removed():
    """Reading of the cutoff: a tone at bin M/2 = L/(2d) keeps half its amplitude; one bin
    above it is removed entirely."""
    L, d = 512, 4
    M = L // d
    t = np.arange(L)
    tau = np.zeros((1, 1))
    at = np.cos(2 * np.pi * (M // 2) * t / L)[None, :]
    above = np.cos(2 * np.pi * (M // 2 + 1) * t / L)[None, :]
    z_at = O.oracle_fdd_rows(at, "f64", tau, L, L, 1, True, "exact", factors=[d])[0]
    z_above = O.oracle_fdd_rows(above, "f64", tau, L, L, 1, True, "exact", factors=[d])[0]
    m = np.arange(M)
    np.testing.assert_allclose(z_at, 0.5 * np.where(m % 2 == 0, 1.0, -1.0), atol=1e-12)
    np.testing.assert_allclose(z_above, 0.0, atol=1e-12)


def test_downsampled_stride_rule():
    """An automatic overlap grows until S is a multiple of the largest factor; an explicit
    overlap that does not give that is rejected."""
    S, n, D = O.chunk_geometry(10000, 1024, 0, False, 100.3, 16)
    assert D == 112 and S == 912 and n == -(-10000 // 912)
    with pytest.raises(ValueError):
        O.chunk_geometry(10000, 1024, 101, False, 100.3, 16)


@pytest.mark.parametrize("t0,tau", [(100, 3.25), (0, 0.5), (511, 17.75), (37, 200.1)])
def test_dirichlet_closed_form(t0, tau):
    """A delta advanced by a fractional delay: closed-form periodic sinc, incl. the Nyquist term."""
    L = 512
    x = np.zeros((1, L))
    x[0, t0] = 1.0
    y = O.oracle_fdd_rows(x, "f64", np.array([[tau]]), L, L, 1, True, "exact")[0]
    M = L // 2
    t = np.arange(L)
    u = 2 * np.pi * (t - t0 + tau) / L
    s = np.sin(u / 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        dsum = np.where(np.abs(s) > 1e-12, np.sin((M - 0.5) * u) / (2 * s) - 0.5, M - 1.0)
    want = (1.0 + np.where(t % 2 == 0, 1.0, -1.0) * np.cos(np.pi * (t0 - tau)) + 2 * dsum) / L
    np.testing.assert_allclose(y, want, atol=1e-12)


# ----------------------------------------------------------------------------- Sec. 2.2 invariants

def _brute_tdd(xc, d, circular_len):
    """Eq. 2 as plain loops (tiny inputs only)."""
    n_chan, n_samp = xc.shape
    y = np.zeros((d.shape[0], n_samp))
    for m in range(d.shape[0]):
        for t in range(n_samp):
            acc = 0.0
            for c in range(n_chan):
                s = t + int(d[m, c])
                if circular_len is not None:
                    s %= circular_len
                    acc += xc[c, s] if s < n_samp else 0.0
                elif s < n_samp:
                    acc += xc[c, s]
            y[m, t] = acc
    return y


@pytest.mark.parametrize("circular", [True, False])
def test_tdd_matches_loops(circular):
    rng = np.random.default_rng(11)
    xc = rng.standard_normal((5, 40))
    d = rng.integers(0, 30, size=(4, 5))
    got = O.tdd(xc, "f64", d, circular_len=64 if circular else None)
    np.testing.assert_allclose(got, _brute_tdd(xc, d, 64 if circular else None), atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_round_fdd_equals_circular_tdd(seed):
    """Sec. 2.2: with the correct phasors FDD gives the time-domain result (single circular chunk)."""
    w = W.tiny_random(seed, n_chan=9, n_samp=900, n_dm=6, chunk_len=1024, single_chunk=True)
    x = W.gaussian_f32(w.n_chan, w.n_samp, seed)
    y = O.fdd(x, "f32", w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len, single_chunk=True,
              mode="round")
    d = O.nearest_sample(O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s))
    np.testing.assert_allclose(y, _brute_tdd(x.astype(np.float64), d, 1024), atol=1e-10)


@pytest.mark.parametrize("seed,L,n_samp", [(3, 256, 1500), (4, 512, 3001), (5, 1024, 1024)])
def test_round_fdd_equals_zero_extended_tdd_chunked(seed, L, n_samp):
    """Sec. 2.2 wrap/discard: overlap >= max delay -> chunked FDD equals TDD with zero extension."""
    w = W.tiny_random(seed, n_chan=6, n_samp=n_samp, n_dm=5, chunk_len=L, single_chunk=False,
                      dm_max=4.0)
    x = W.gaussian_f32(w.n_chan, w.n_samp, seed)
    y = O.fdd(x, "f32", w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, L, mode="round")
    d = O.nearest_sample(O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s))
    np.testing.assert_allclose(y, O.tdd(x, "f32", d), atol=1e-10)
    np.testing.assert_allclose(y, _brute_tdd(x.astype(np.float64), d, None), atol=1e-10)


def test_exact_equals_round_for_integer_delays():
    """Eq. 4 with integer delays: the fractional-phase path reduces to the nearest-sample path."""
    rng = np.random.default_rng(5)
    x = rng.standard_normal((4, 700))
    tau = rng.integers(0, 40, size=(3, 4)).astype(np.float64)
    for single, S, n in [(True, 1024, 1), (False, 256 - 40, -(-700 // (256 - 40)))]:
        L = 1024 if single else 256
        a = O.oracle_fdd_rows(x, "f64", tau, L, S, n, single, "exact")
        b = O.oracle_fdd_rows(x, "f64", tau, L, S, n, single, "round")
        np.testing.assert_allclose(a, b, atol=1e-10)


@pytest.mark.parametrize("mode", ["exact", "round"])
def test_dm_zero_is_channel_sum(mode):
    """Eq. 4 with dt = 0: every phasor is 1, so DM 0 returns the plain channel sum."""
    w = W.small_fp32()
    x = W.gaussian_f32(w.n_chan, w.n_samp, 0)
    y = O.fdd(x, "f32", [0.0], w.freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len, single_chunk=True,
              mode=mode)
    np.testing.assert_allclose(y[0], x.astype(np.float64).sum(axis=0), atol=1e-10)


def test_single_channel_amplitudes_preserved():
    """Sec. 2.2: a pure phase rotation leaves the spectral amplitudes unchanged."""
    rng = np.random.default_rng(9)
    x = rng.standard_normal((1, 2048))
    X = O.forward_spectra(x)[0]
    tau = np.array([[123.456]])
    P = O.oracle_fdd_rows(x, "f64", tau, 2048, 2048, 1, True, "exact", power=True)[0]
    np.testing.assert_allclose(P, (np.abs(X) ** 2)[:1024], rtol=1e-12)


def test_power_is_spectrum_of_circular_tdd():
    """Sec. 5: power taken in the Fourier domain equals |DFT|^2 of the dedispersed series."""
    w = W.tiny_random(21, n_chan=8, n_samp=1024, n_dm=4, chunk_len=1024, single_chunk=True)
    x = W.gaussian_f32(w.n_chan, w.n_samp, 21)
    tau = O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s)
    P = O.oracle_fdd_rows(x, "f32", tau, 1024, 1024, 1, True, "round", power=True)
    y = _brute_tdd(x.astype(np.float64), O.nearest_sample(tau), 1024)
    want = np.abs(O.direct_rdft(y)) ** 2
    np.testing.assert_allclose(P, want[:, :512], rtol=1e-9, atol=1e-8)


def test_linearity_and_channel_permutation():
    w = W.tiny_random(31, n_chan=6, n_samp=1000, n_dm=4, chunk_len=512, single_chunk=False,
                      dm_max=3.0)
    rng = np.random.default_rng(31)
    a = rng.standard_normal((w.n_chan, w.n_samp))
    b = rng.standard_normal((w.n_chan, w.n_samp))

    def run(x, freqs):
        return O.fdd(x, "f64", w.dms, freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len, mode="exact")

    np.testing.assert_allclose(run(2.0 * a - 3.0 * b, w.freqs), 2.0 * run(a, w.freqs) - 3.0 * run(b, w.freqs),
                               atol=1e-10)
    perm = rng.permutation(w.n_chan)
    np.testing.assert_allclose(run(a[perm], w.freqs[perm]), run(a, w.freqs), atol=1e-10)


@pytest.mark.parametrize("mode", ["exact", "round"])
def test_injected_pulse_peaks_at_its_dm(mode):
    """Small workload: a 5-sigma pulse at t = 1000 dispersed at DM 30 peaks at trial 30."""
    w = W.small_fp32()
    x = W.gaussian_f32(w.n_chan, w.n_samp, 0)
    offs = O.nearest_sample(O.delays([30.0], w.freqs, w.ref_freq_mhz, w.tsamp_s))[0]
    W.inject_pulse_f32(x, offs, 1000, 5.0, circular=True)
    y = O.fdd(x, "f32", w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len, single_chunk=True,
              mode=mode)
    assert int(np.argmax(y[:, 1000])) == 30
    assert y[30, 1000] > 250.0


# ----------------------------------------------------------------------------- scaled DMs, Sec. 2.3 / Eq. 8

def _scaled_f_min(n_dm, dm_max, block=64, halo=32):
    step = dm_max / (n_dm - 1)
    rmin = 32.0 * dm_max / ((halo - 1) * step)
    return max(block, int(np.ceil(max(0.0, rmin - block // 2) / block) * block))


def test_scaled_phasor_is_the_exact_phasor_at_the_scaled_dm():
    """Eq. 8: the reference bin's phasor at DM equals bin f's phasor (Eq. 4) at DM r / f."""
    rng = np.random.default_rng(21)
    L = 8192
    freqs = np.sort(rng.uniform(1200.0, 1500.0, 9))
    kap = O.kappa(freqs, 1500.0, 64e-6)
    for r, f in [(100, 97), (2080, 2111), (3000, 2970), (4000, 4031)]:
        dm = rng.uniform(0.0, 80.0, 5)
        Ws = O.scaled_phasors(kap, dm, r, L)
        for i in range(dm.size):
            We = O.phasors((dm[i] * r / f) * kap, L, "exact")[:, f]
            np.testing.assert_allclose(Ws[i], We, atol=1e-9)


def test_scaled_equals_exact_at_reference_bins_and_below_f_min():
    rng = np.random.default_rng(22)
    L, n_chan, n_dm = 4096, 12, 40
    freqs = np.sort(rng.uniform(1200.0, 1500.0, n_chan))
    dms = np.linspace(3.0, 45.0, n_dm)
    x = rng.standard_normal((n_chan, L))
    f_min = _scaled_f_min(n_dm, 45.0) + 64          # some exact bins, then blocks
    refs = np.arange(f_min + 32, L // 2, 64)
    bins = np.concatenate([np.arange(0, f_min, 7), refs])
    got = O.fdd_power_scaled(x, "f64", dms, freqs, 1500.0, 64e-6, L, f_min, bins=bins)
    want = O.fdd_power(x, "f64", dms, freqs, 1500.0, 64e-6, L)[:, bins]
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-9 * want.max())


def test_scaled_dm_independent_channel_is_exact_everywhere():
    """A channel at the reference frequency has no delay: every scaled row equals |X|^2, so the
    interpolation weights must sum to one at every bin."""
    rng = np.random.default_rng(23)
    L = 2048
    x = rng.standard_normal((1, L))
    dms = np.linspace(0.0, 30.0, 33)
    got = O.fdd_power_scaled(x, "f64", dms, [1400.0], 1400.0, 64e-6, L, 64)
    X = np.fft.rfft(x[0])[: L // 2]
    np.testing.assert_allclose(got, np.broadcast_to(np.abs(X) ** 2, got.shape), rtol=1e-12)


def test_scaled_two_channel_closed_form():
    """A delta in a delay-free channel and in one with a small delay per unit DM: the exact power
    is 2 + 2 cos(2 pi f DM kappa / L).  The scaled rows sample that cosine in DM at phase steps
    below 0.01 rad, so linear resampling reproduces it to 1e-4, which fixes the direction of the
    stretch (f / r), the reference bin and the row offset."""
    L, n_dm = 4096, 64
    x = np.zeros((2, L))
    x[:, 0] = 1.0
    ref_mhz = 1500.0
    tsamp = 64e-6
    dms = np.linspace(0.0, 60.0, n_dm)
    step = dms[1] - dms[0]
    # kappa with pi * step * kappa = 0.0095 rad per row at the highest reference bin
    kap_target = 0.0095 / (np.pi * step)
    nu = 1.0 / np.sqrt(kap_target * tsamp / 4.148808e3 + 1.0 / ref_mhz ** 2)
    freqs = [ref_mhz, nu]
    kap = O.kappa(freqs, ref_mhz, tsamp)[1]
    f_min = _scaled_f_min(n_dm, 60.0)
    got = O.fdd_power_scaled(x, "f64", dms, freqs, ref_mhz, tsamp, L, f_min)
    f = np.arange(L // 2)
    want = 2.0 + 2.0 * np.cos(2 * np.pi * f[None, :] * dms[:, None] * kap / L)
    np.testing.assert_allclose(got, want, atol=1e-4)
    # the approximation is not trivially exact here: rows move by whole steps within a block
    assert np.abs(dms[-1] * (f_min + 1) / (f_min + 32) - dms[-1]) > step


# ----------------------------------------------------------------------------- 8-bit time-major input (Sec. 3)
#
# The paper's 8-bit filterbanks are sample-major and need a transpose before the per-channel
# transforms (Sec. 3).  These pins build such an array from an explicit formula of (t, c) and
# check every 8-bit path of the oracle against the same formula read channel-major, so that a
# transposed, offset or mis-strided read of the time-major layout fails.

def _u8_value(t, c):
    return (37 * t + 11 * c + 5) % 256


def _u8_time_major(n_samp, n_chan):
    x = np.zeros((n_samp, n_chan), dtype=np.uint8)
    for t in range(n_samp):
        for c in range(n_chan):
            x[t, c] = _u8_value(t, c)
    return x


def _f32_channel_major(n_samp, n_chan):
    x = np.zeros((n_chan, n_samp), dtype=np.float32)
    for c in range(n_chan):
        for t in range(n_samp):
            x[c, t] = float(_u8_value(t, c))
    return x


@pytest.mark.parametrize("t0,L", [(0, 16), (7, 20), (20, 8), (23, 4)])
def test_u8_reader_against_formula(t0, L):
    """input_segment on time-major uint8 [n_samp][n_chan]: out[c, j] = x(t0 + j, c), zero past the data."""
    n_samp, n_chan = 23, 5
    x = _u8_time_major(n_samp, n_chan)
    seg = O.input_segment(x, "u8", t0, L)
    assert seg.shape == (n_chan, L) and seg.dtype == np.float64
    for c in range(n_chan):
        for j in range(L):
            want = float(_u8_value(t0 + j, c)) if t0 + j < n_samp else 0.0
            assert seg[c, j] == want, (c, j)
    sub = O.input_segment(x, "u8", t0, L, channels=slice(1, 4))
    for i, c in enumerate(range(1, 4)):
        for j in range(L):
            want = float(_u8_value(t0 + j, c)) if t0 + j < n_samp else 0.0
            assert sub[i, j] == want


@pytest.mark.parametrize("circular", [True, False])
def test_u8_tdd_against_loops(circular):
    """Eq. 2 on 8-bit time-major input, written out over (t, c) with the formula's values."""
    n_samp, n_chan = 29, 3
    x = _u8_time_major(n_samp, n_chan)
    d = np.array([[0, 1, 4], [2, 0, 7], [5, 3, 1]])
    Lc = 32 if circular else None
    got = O.tdd(x, "u8", d, circular_len=Lc)
    for m in range(d.shape[0]):
        for t in range(n_samp):
            acc = 0.0
            for c in range(n_chan):
                s = t + int(d[m, c])
                if circular:
                    s %= 32
                if s < n_samp:
                    acc += _u8_value(s, c)
            assert got[m, t] == acc, (m, t)


@pytest.mark.parametrize("mode", ["exact", "round"])
@pytest.mark.parametrize("single,L,n_samp", [(True, 64, 50), (True, 64, 64), (False, 64, 300)])
def test_u8_fdd_equals_channel_major_float(mode, single, L, n_samp):
    """FDD of 8-bit time-major input equals FDD of the same values given channel-major as float."""
    n_chan = 6
    w = W.tiny_random(3, n_chan=n_chan, n_samp=n_samp, n_dm=4, chunk_len=L, single_chunk=single, dm_max=0.3)
    xu = _u8_time_major(n_samp, n_chan)
    xf = _f32_channel_major(n_samp, n_chan)
    a = O.fdd(xu, "u8", w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, L, single_chunk=single, mode=mode)
    b = O.fdd(xf, "f32", w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, L, single_chunk=single, mode=mode)
    assert a.shape == (4, n_samp)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-9)
    if mode == "round":
        d = O.nearest_sample(O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s))
        np.testing.assert_allclose(a, _brute_tdd(xf.astype(np.float64), d, L if single else None), atol=1e-9)
    if single:
        tau = O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s)
        pu = O.oracle_fdd_rows(xu, "u8", tau, L, L, 1, True, mode, power=True)
        pf = O.oracle_fdd_rows(xf, "f32", tau, L, L, 1, True, mode, power=True)
        np.testing.assert_allclose(pu, pf, rtol=1e-12, atol=1e-6)
