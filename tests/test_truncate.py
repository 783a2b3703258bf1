"""CPU checks of the model truncation (Sec. 5.3)."""
import math

import numpy as np
import pytest

import synth
from paper_2005_09316_amd import truncate


def test_hermite_l1_closed_forms():
    l1 = truncate.hermite_l1(2)
    # phi_0 = pi^(-1/4) e^(-x^2/2); phi_1 = sqrt(2) x phi_0; phi_2 = (2x^2 - 1) phi_0 / sqrt(2)
    assert abs(l1[0] - math.sqrt(2.0) * math.pi ** 0.25) < 1e-6
    assert abs(l1[1] - 2.0 * math.sqrt(2.0) * math.pi ** -0.25) < 1e-6
    a = 1.0 / math.sqrt(2.0)
    g = math.sqrt(2.0 * math.pi) * math.erf(a / math.sqrt(2.0))
    i2 = math.sqrt(2.0 * math.pi) + 8.0 * a * math.exp(-a * a / 2.0) - 2.0 * g
    assert abs(l1[2] - i2 * math.pi ** -0.25 / math.sqrt(2.0)) < 1e-6


def test_hermite_l1_grows_like_quarter_power():
    l1 = truncate.hermite_l1(96)
    r = l1[96] / l1[24]
    assert abs(r - 4.0 ** 0.25) < 0.05 * 4.0 ** 0.25


def test_single_gaussian_term_counts_its_flux():
    import dataclasses
    sky = dataclasses.replace(synth.empty_sky(), s_ra=np.array([0.0]), s_dec=np.array([-0.6]), s_sref=np.array([7.0]),
                              s_alpha=np.array([0.0]), s_beta1=np.array([1e-3]), s_beta2=np.array([1e-3]),
                              s_pa=np.array([0.0]), s_nmax=np.array([0], np.int32),
                              s_coeff_off=np.array([0], np.int64), coeffs=np.array([math.sqrt(math.pi)]))
    flux, kind, comp, coef = truncate.component_flux(sky)
    # C_00 phi_0(0)^2 = 1: the image of the term is a Gaussian of flux S
    assert flux.size == 1 and abs(flux[0] - 7.0) < 1e-5


def test_keep_count_follows_the_cumulative_rule():
    flux = np.array([5.0, 3.0, 2.0, 1.0, -4.0])
    assert truncate.keep_count(flux, 1.0) == 5
    assert truncate.keep_count(flux, 0.6) == 2     # 5 + 4 = 9 <= 9 < 12
    assert truncate.keep_count(flux, 0.59) == 1    # 5 <= 8.85 < 9
    assert truncate.keep_count(flux, 0.1) == 1     # at least one
    with pytest.raises(ValueError):
        truncate.keep_count(flux, 0.0)


def test_truncate_by_flux_keeps_the_largest_and_stays_within_f():
    obs, sky = synth.make_config(0)
    full, kind, comp, coef = truncate.component_flux(sky)
    for f in (1.0, 0.9, 0.5, 0.2):
        t, n, ntot, frac = truncate.truncate_by_flux(sky, f)
        assert ntot == full.size and frac <= f + 1e-12
        tf, _, _, _ = truncate.component_flux(t)
        kept = tf[tf > 0]
        assert kept.size == n or f == 1.0
        # every dropped component is no larger than the smallest kept one
        assert np.sort(full)[::-1][n - 1] <= kept.min() + 1e-12
    t, n, ntot, frac = truncate.truncate_by_flux(sky, 1.0)
    assert n == ntot and abs(frac - 1.0) < 1e-12
    assert np.array_equal(t.coeffs, sky.coeffs) and t.n_point == sky.n_point


def test_truncate_by_order_zeroes_high_orders():
    obs, sky = synth.make_config(0)
    t = truncate.truncate_by_order(sky, 4)
    n1, n2 = truncate._orders(int(sky.s_nmax[0]))
    c = t.coeffs[:n1.size]
    assert np.all(c[n1 + n2 > 4] == 0.0)
    assert np.array_equal(c[n1 + n2 <= 4], sky.coeffs[:n1.size][n1 + n2 <= 4])


def test_spectral_term_skies_are_refused():
    _, sky = synth.make_config(0, n_tiles=8, n_chan=2, shapelet_nmax=[6])
    multi = synth.with_spectral_terms(sky, np.random.default_rng(1), 2)
    with pytest.raises(ValueError):
        truncate.truncate_by_flux(multi, 0.9)
    with pytest.raises(ValueError):
        truncate.truncate_by_order(multi, 3)
