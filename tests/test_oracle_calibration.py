"""Pins of the oracle's calibration (Sec. 5.1): recovery of known gains from
noise-free data, the unit-gain fixed point, the minimum-norm gauge of the
step, and agreement with a generic least-squares optimiser on noisy data."""
import numpy as np
import pytest

import oracle
import synth


def _cell(rng, n_ant, noise=0.0):
    a1, a2 = synth.antenna_pairs(n_ant)
    model = rng.lognormal(0.0, 0.5, a1.size) * np.exp(2j * np.pi * rng.random(a1.size))
    g = synth.random_gains(rng, 1, 1, n_ant)[0, 0]
    v = g[a1] * np.conj(g[a2]) * model
    if noise:
        v = v + noise * (rng.standard_normal(a1.size) + 1j * rng.standard_normal(a1.size))
    return a1, a2, model, g, v


def test_noise_free_gains_are_recovered():
    rng = np.random.default_rng(11)
    a1, a2, model, g_true, v = _cell(rng, 12)
    g = oracle.calibrate_cell(v, model, a1, a2, 12, n_iter=10)
    # the data fix g_i g_j^* (the global phase of g is free)
    prod = g[a1] * np.conj(g[a2])
    assert np.max(np.abs(prod - g_true[a1] * np.conj(g_true[a2]))) < 1e-10
    res = v - prod * model
    assert np.max(np.abs(res)) < 1e-10 * np.max(np.abs(v))
    # one global phase relates the solution to the truth
    rot = g / g_true
    assert np.max(np.abs(np.abs(rot) - 1.0)) < 1e-10
    assert np.max(np.abs(rot / rot[0] - 1.0)) < 1e-10


def test_unit_gains_are_a_fixed_point():
    rng = np.random.default_rng(12)
    a1, a2 = synth.antenna_pairs(8)
    model = rng.standard_normal(a1.size) + 1j * rng.standard_normal(a1.size)
    g = oracle.calibrate_cell(model, model, a1, a2, 8, n_iter=3)
    assert np.array_equal(g, np.ones(8, np.complex128))


def test_step_is_minimum_norm_in_the_global_phase():
    # from g = 1 the undetermined direction is i (1, ..., 1): the step has no
    # component along it
    rng = np.random.default_rng(13)
    a1, a2, model, g_true, v = _cell(rng, 10)
    g1 = oracle.calibrate_cell(v, model, a1, a2, 10, n_iter=1)
    e = g1 - 1.0
    assert abs(np.sum(e.imag)) < 1e-12 * np.sum(np.abs(e))


def test_noisy_solution_matches_a_generic_least_squares_fit():
    scipy_opt = pytest.importorskip("scipy.optimize")
    rng = np.random.default_rng(14)
    n = 10
    a1, a2, model, g_true, v = _cell(rng, n, noise=0.05)
    g = oracle.calibrate_cell(v, model, a1, a2, n, n_iter=10)

    def resid(x):
        gg = x[:n] + 1j * x[n:]
        r = v - gg[a1] * np.conj(gg[a2]) * model
        return np.concatenate([r.real, r.imag])

    x0 = np.concatenate([np.ones(n), np.zeros(n)])
    fit = scipy_opt.least_squares(resid, x0, method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15)
    gl = fit.x[:n] + 1j * fit.x[n:]
    cost_oracle = np.sum(resid(np.concatenate([g.real, g.imag])) ** 2)
    cost_lm = np.sum(fit.fun ** 2)
    assert cost_oracle <= cost_lm * (1 + 1e-9)
    p_oracle = g[a1] * np.conj(g[a2])
    p_lm = gl[a1] * np.conj(gl[a2])
    assert np.max(np.abs(p_oracle - p_lm)) < 1e-7


def test_peel_subtracts_the_gain_corrupted_model():
    rng = np.random.default_rng(15)
    n, T, K = 6, 2, 3
    a1, a2 = synth.antenna_pairs(n)
    model = rng.standard_normal((T, a1.size, K)) + 1j * rng.standard_normal((T, a1.size, K))
    gt = synth.random_gains(rng, T, K, n)
    data = np.empty_like(model)
    for t in range(T):
        for k in range(K):
            data[t, :, k] = gt[t, k, a1] * np.conj(gt[t, k, a2]) * model[t, :, k]
    gains, res = oracle.peel(data, model, a1, a2, n)
    assert gains.shape == (T, K, n)
    assert np.max(np.abs(res)) < 1e-10 * np.max(np.abs(data))


def test_two_tiles_closed_form():
    # one baseline: the data fix g_0 g_1^* = V / I exactly; from unit gains the
    # minimum-norm steps keep the mean phase at zero, so g_1 = conj(g_0) up
    # to amplitude: |g_0| = |g_1| = sqrt(|V / I|), arg g_0 = -arg g_1
    a1, a2 = np.array([0], np.int32), np.array([1], np.int32)
    m = np.array([2.0 - 1.0j])
    v = np.array([(1.3 * np.exp(0.4j)) * m[0]])
    g = oracle.calibrate_cell(v, m, a1, a2, 2, n_iter=30)
    ratio = v[0] / m[0]
    assert abs(g[0] * np.conj(g[1]) - ratio) < 1e-12
    assert abs(abs(g[0]) - abs(g[1])) < 1e-12
    assert abs(np.angle(g[0]) + np.angle(g[1])) < 1e-12


try:
    from hypothesis import given, settings, strategies as st
except ImportError:  # pragma: no cover
    given = None

if given is not None:
    @settings(max_examples=25, deadline=None, derandomize=True)
    @given(n=st.integers(3, 9), seed=st.integers(0, 2 ** 31 - 1))
    def test_noise_free_recovery_random_arrays(n, seed):
        """Any connected array with all pairs, random model and gains within
        the linear regime: the calibrated products g_i g_j^* reproduce the
        true ones and the step gauge keeps the mean phase change at zero."""
        rng = np.random.default_rng(seed)
        a1, a2 = synth.antenna_pairs(n)
        model = rng.lognormal(0.0, 0.3, a1.size) * np.exp(2j * np.pi * rng.random(a1.size))
        g_true = synth.random_gains(rng, 1, 1, n, amp_sigma=0.1, phase_sigma=0.3)[0, 0]
        v = g_true[a1] * np.conj(g_true[a2]) * model
        g = oracle.calibrate_cell(v, model, a1, a2, n, n_iter=15)
        prod = g[a1] * np.conj(g[a2])
        assert np.max(np.abs(prod - g_true[a1] * np.conj(g_true[a2]))) < 1e-9
