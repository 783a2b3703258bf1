"""Pins of the oracle's frequency-dependent shapelet coefficients: the
coefficients at frequency nu are C(nu) = sum_q C_q ln(nu/nu_ref)^q, the form
in which the paper proposes fitting the coefficients as a function of
frequency (Sec. 7) so that the spectral index may vary across a source."""
import dataclasses
import math

import numpy as np

import oracle
import synth


def _obs(freqs):
    obs, _ = synth.make_config(0, n_tiles=8, n_time=2, n_chan=len(freqs), n_point=1, n_gauss=1,
                               shapelet_nmax=[4])
    return dataclasses.replace(obs, freq_hz=np.asarray(freqs, np.float64), n_chan=len(freqs))


def test_single_term_equals_the_plain_model():
    obs, sky = synth.make_config(0, n_tiles=8, n_time=1, n_chan=3, shapelet_nmax=[12, 5])
    one = dataclasses.replace(sky, s_nterm=np.ones(sky.n_shp, np.int32))
    assert np.array_equal(oracle.predict(obs, sky), oracle.predict(obs, one))


def test_reference_frequency_sees_the_first_term_only():
    _, sky = synth.make_config(0, n_tiles=8, n_time=1, n_chan=3, shapelet_nmax=[12])
    obs = _obs([sky.nu_ref_hz, 1.1 * sky.nu_ref_hz])
    multi = synth.with_spectral_terms(sky, np.random.default_rng(3), 3, scale=0.5)
    v_multi = oracle.predict(obs, multi)
    v_plain = oracle.predict(obs, sky)
    assert np.array_equal(v_multi[..., 0], v_plain[..., 0])
    assert not np.allclose(v_multi[..., 1], v_plain[..., 1])


def test_order_zero_shapelet_is_a_gaussian_times_the_spectral_polynomial():
    # a (0,0) shapelet with beta = FWHM at the phase centre equals the
    # Gaussian envelope times C_00 phi_0(0)^2 = C_00 / sqrt(pi); with terms
    # the factor becomes (c0 + c1 x + c2 x^2) / sqrt(pi), x = ln(nu/nu_ref)
    freqs = np.array([150e6, 165e6, 180e6, 197e6])
    obs = _obs(freqs)
    ref = synth.empty_sky()
    c = np.array([1.7, -0.6, 2.3])
    maj, mn, pa = math.radians(0.3), math.radians(0.2), 0.4
    shp = dataclasses.replace(
        ref, s_ra=np.array([obs.ra0]), s_dec=np.array([obs.dec0]), s_sref=np.array([3.0]),
        s_alpha=np.array([-0.7]), s_beta1=np.array([maj]), s_beta2=np.array([mn]), s_pa=np.array([pa]),
        s_nmax=np.array([0], np.int32), s_coeff_off=np.array([0], np.int64), coeffs=c,
        s_nterm=np.array([3], np.int32))
    gau = dataclasses.replace(
        ref, g_ra=np.array([obs.ra0]), g_dec=np.array([obs.dec0]), g_sref=np.array([3.0]),
        g_alpha=np.array([-0.7]), g_maj=np.array([maj]), g_min=np.array([mn]), g_pa=np.array([pa]))
    v_s = oracle.predict(obs, shp)
    v_g = oracle.predict(obs, gau)
    x = np.log(freqs / ref.nu_ref_hz)
    factor = (c[0] + c[1] * x + c[2] * x * x) / math.sqrt(math.pi)
    assert np.max(np.abs(v_s - v_g * factor)) < 1e-13 * np.max(np.abs(v_g))


def test_each_term_enters_with_its_power_of_the_log_frequency():
    _, sky = synth.make_config(0, n_tiles=8, n_time=1, n_chan=3, n_point=0, n_gauss=0, shapelet_nmax=[9])
    obs = _obs([140e6, 170e6, 200e6])
    multi = synth.with_spectral_terms(sky, np.random.default_rng(4), 2, scale=1.0)
    cnt = 55
    c0, c1 = multi.coeffs[:cnt], multi.coeffs[cnt:2 * cnt]
    v = oracle.predict(obs, multi)
    v0 = oracle.predict(obs, dataclasses.replace(sky, coeffs=c0))
    v1 = oracle.predict(obs, dataclasses.replace(sky, coeffs=c1))
    x = np.log(np.asarray(obs.freq_hz) / sky.nu_ref_hz)
    assert np.max(np.abs(v - (v0 + v1 * x))) < 1e-12 * np.max(np.abs(v))
