"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test ties one piece of the oracle to something fixed independently of
its code: the paper's printed counts (tests/golden), closed forms of the
Hermite functions, library routines (scipy, numpy's Gauss-Hermite rule),
brute-force pixel DFTs of the image-plane models of Sec. 2 and Sec. 3.2, and
a 50-digit mpmath evaluation of the whole sum on a sample of visibilities.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest
import scipy.special as sps

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
KAPPA = math.pi / math.sqrt(2.0 * math.log(2.0))
FWHM_TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))


# --------------------------------------------------------------------------
# paper counts (Sec. 2 p_tot, Sec. 5.3)
# --------------------------------------------------------------------------

def test_basis_counts_match_paper():
    """Sec. 2: p_tot = (p_max+2)(p_max+1)/2 for n1+n2 <= p_max; Sec. 5.3 prints
    7656 basis functions for two p_max = 86 models."""
    gold = json.load(open(os.path.join(HERE, "golden", "paper_counts.json")))
    for case in gold["cases"]:
        n = case["pmax"]
        brute = sum(1 for a in range(n + 1) for b in range(n + 1) if a + b <= n)
        assert brute * case["models"] == case["basis_total"]
        # the oracle consumes exactly that many coefficients
        c = np.zeros(brute)
        oracle.shapelet_envelope_ab(n, c, 0.3, -0.2)
        with pytest.raises(ValueError):
            oracle.shapelet_envelope_ab(n, np.zeros(brute + 1), 0.3, -0.2)
    ms = gold["ms_clean"]
    assert ms["point"] + ms["gaussian"] == ms["total"]


def test_every_coefficient_reaches_the_envelope():
    """Every packed (n1, n2) term must contribute: perturbing coefficient i alone
    changes xi by exactly phi_n1(a) phi_n2(b) (sign i)^(n1+n2)."""
    n = 7
    n1, n2 = synth.shapelet_orders(n)
    a, b = 0.7, -1.3
    pa, pb = oracle.hermite(n, a), oracle.hermite(n, b)
    for i in range(n1.size):
        c = np.zeros(n1.size)
        c[i] = 1.0
        got = oracle.shapelet_envelope_ab(n, c, a, b, sign=-1)
        want = pa[n1[i]] * pb[n2[i]] * (-1j) ** int(n1[i] + n2[i])
        assert abs(got - want) < 1e-15


# --------------------------------------------------------------------------
# Hermite functions (Sec. 2 Eq. basis_1D, orthonormal reading)
# --------------------------------------------------------------------------

def test_hermite_matches_scipy_polynomials():
    for x in [-7.3, -2.0, -0.1, 0.0, 0.4, 1.7, 5.5]:
        phi = oracle.hermite(40, x)
        for n in range(41):
            ref = sps.eval_hermite(n, x) * math.exp(-x * x / 2) / math.sqrt(
                2.0 ** n * math.factorial(n) * math.sqrt(math.pi))
            assert abs(phi[n] - ref) <= 1e-12 * max(1.0, abs(ref))


def test_hermite_orthonormal_gauss_hermite_quadrature():
    """With 120 Gauss-Hermite nodes the rule is exact for H_m H_n, m, n <= 96."""
    x, w = np.polynomial.hermite.hermgauss(120)
    nmax = 96
    P = np.stack([oracle.hermite(nmax, xi) for xi in x])  # [nodes, n]
    G = (P * (w * np.exp(x * x))[:, None]).T @ P
    assert np.max(np.abs(G - np.eye(nmax + 1))) < 1e-11


def test_hermite_orthonormal_trapezoid():
    xs = np.arange(-40.0, 40.0 + 1e-9, 0.004)
    nmax = 80
    P = np.stack([oracle.hermite(nmax, xi) for xi in xs])
    G = P.T @ P * 0.004
    assert np.max(np.abs(G - np.eye(nmax + 1))) < 1e-10


def test_hermite_at_origin_closed_form():
    phi = oracle.hermite(96, 0.0)
    for n in range(97):
        if n % 2:
            assert phi[n] == 0.0
        else:
            k = n // 2
            ref = (-1) ** k * math.sqrt(math.factorial(n)) / (2.0 ** k * math.factorial(k) * math.pi ** 0.25)
            assert abs(phi[n] - ref) < 1e-15


def test_hermite_cramer_bound():
    bound = math.pi ** -0.25
    for x in np.linspace(-30, 30, 1201):
        assert np.all(np.abs(oracle.hermite(96, x)) <= bound * (1 + 1e-12))


def test_hermite_derivative_identity():
    """phi_n' = sqrt(n/2) phi_{n-1} - sqrt((n+1)/2) phi_{n+1} vs a central difference."""
    h = 1e-5
    for x in [-4.1, -0.3, 0.9, 3.3, 8.0]:
        p = oracle.hermite(61, x)
        d = (oracle.hermite(61, x + h) - oracle.hermite(61, x - h)) / (2 * h)
        for n in range(60):
            lad = (math.sqrt(n / 2) * p[n - 1] if n else 0.0) - math.sqrt((n + 1) / 2) * p[n + 1]
            assert abs(d[n] - lad) < 1e-8


def test_hermite_mpmath_high_orders():
    mpmath.mp.dps = 50
    for x in [0.37, 4.9, 11.0, 13.2, 16.0]:
        phi = oracle.hermite(90, x)
        for n in [0, 1, 2, 17, 54, 70, 80, 90]:
            ref = mpmath.hermite(n, x) * mpmath.exp(-mpmath.mpf(x) ** 2 / 2) / mpmath.sqrt(
                mpmath.mpf(2) ** n * mpmath.factorial(n) * mpmath.sqrt(mpmath.pi))
            assert abs(phi[n] - float(ref)) < 1e-13 * max(1.0, abs(float(ref))) + 1e-300


# --------------------------------------------------------------------------
# positions and frames
# --------------------------------------------------------------------------

def _dir(ra, dec):
    return np.array([math.cos(dec) * math.cos(ra), math.cos(dec) * math.sin(ra), math.sin(dec)])


def test_lmn_textbook_formula_and_unit_norm():
    ra0, dec0 = 0.3, math.radians(-37)
    rng = np.random.default_rng(7)
    for _ in range(50):
        ra = ra0 + rng.uniform(-0.3, 0.3)
        dec = dec0 + rng.uniform(-0.2, 0.2)
        l, m, n1 = oracle.lmn(ra0, dec0, ra, dec)
        da = ra - ra0
        lt = math.cos(dec) * math.sin(da)
        mt = math.sin(dec) * math.cos(dec0) - math.cos(dec) * math.sin(dec0) * math.cos(da)
        nt = math.sin(dec) * math.sin(dec0) + math.cos(dec) * math.cos(dec0) * math.cos(da)
        assert abs(l - lt) < 1e-15 and abs(m - mt) < 1e-15
        assert abs((n1 + 1) - nt) < 1e-15
        assert abs(l * l + m * m + (n1 + 1) ** 2 - 1) < 1e-15
    assert np.all(oracle.lmn(ra0, dec0, ra0, dec0) == 0.0)


def test_n_minus_one_without_cancellation():
    mpmath.mp.dps = 40
    ra0, dec0 = 0.0, math.radians(-37)
    for eps in [1e-9, 1e-7, 1e-5]:
        l, m, n1 = oracle.lmn(ra0, dec0, ra0 + eps, dec0 + eps)
        ref = -(mpmath.mpf(l) ** 2 + mpmath.mpf(m) ** 2) / (1 + mpmath.sqrt(1 - mpmath.mpf(l) ** 2 - mpmath.mpf(m) ** 2))
        assert abs(n1 - float(ref)) <= 1e-15 * abs(float(ref))


def test_rotation_properties():
    ra0, dec0 = 0.0, math.radians(-37)
    assert np.allclose(oracle.rotation(ra0, dec0, ra0, dec0), np.eye(3), atol=1e-16)
    rng = np.random.default_rng(3)
    for _ in range(20):
        ra, dec = ra0 + rng.uniform(-0.2, 0.2), dec0 + rng.uniform(-0.2, 0.2)
        R = oracle.rotation(ra0, dec0, ra, dec)
        assert np.max(np.abs(R @ R.T - np.eye(3))) < 1e-15
        assert abs(np.linalg.det(R) - 1) < 1e-14
        l, m, n1 = oracle.lmn(ra0, dec0, ra, dec)
        # the component's direction, seen from the phase centre, becomes the new w axis
        assert np.max(np.abs(R @ np.array([l, m, n1 + 1]) - np.array([0, 0, 1]))) < 1e-15
        # a baseline's w' towards the component equals b . s_j
        b = rng.normal(size=3) * 1000
        east0 = np.array([-math.sin(ra0), math.cos(ra0), 0])
        north0 = np.array([-math.sin(dec0) * math.cos(ra0), -math.sin(dec0) * math.sin(ra0), math.cos(dec0)])
        uvw = np.array([b @ east0, b @ north0, b @ _dir(ra0, dec0)])
        eastj = np.array([-math.sin(ra), math.cos(ra), 0])
        assert abs((R @ uvw)[2] - b @ _dir(ra, dec)) < 1e-9
        assert abs((R @ uvw)[0] - b @ eastj) < 1e-9


# --------------------------------------------------------------------------
# envelopes against brute-force DFTs of their image-plane models
# --------------------------------------------------------------------------

def _pixel_grid(half_deg=1.2, n=801):
    x = np.linspace(-math.radians(half_deg), math.radians(half_deg), n)
    L, M = np.meshgrid(x, x, indexing="ij")
    return L, M, (x[1] - x[0]) ** 2


def _dft(img, L, M, dA, u, v, sign=-1):
    return np.sum(img * np.exp(sign * 2j * math.pi * (u * L + v * M))) * dA


def test_gauss_envelope_is_dft_of_image_gaussian():
    """Sec. 3.2 Eq. (gauss-def) imaged with major axis at PA (east of north),
    normalised to unit integral, has the transform of Eq. (gauss-env)."""
    L, M, dA = _pixel_grid(0.9, 701)
    for maj, mn, pa in [(12.0, 5.0, 0.0), (15.0, 9.0, 0.7), (8.0, 8.0, 2.2)]:
        maj, mn = maj * synth.ARCMIN, mn * synth.ARCMIN
        x = L * math.sin(pa) + M * math.cos(pa)
        y = L * math.cos(pa) - M * math.sin(pa)
        img = np.exp(-4 * math.log(2) * (x ** 2 / maj ** 2 + y ** 2 / mn ** 2))
        img /= img.sum() * dA
        for u, v in [(0, 0), (120.0, -40.0), (-300.0, 250.0), (60.0, 410.0)]:
            ref = _dft(img, L, M, dA, u, v)
            got = oracle.gauss_envelope(u, v, maj, mn, pa)
            assert abs(got - ref) < 1e-9


def test_gauss_major_axis_runs_north_at_zero_pa():
    """PA = 0: the envelope is narrowest along v (image extended along m)."""
    maj, mn = 20 * synth.ARCMIN, 5 * synth.ARCMIN
    assert oracle.gauss_envelope(0, 200, maj, mn, 0.0) < oracle.gauss_envelope(200, 0, maj, mn, 0.0)


@pytest.mark.parametrize("n1,n2", [(0, 0), (1, 0), (0, 1), (2, 1), (1, 2), (3, 2), (0, 3), (4, 0)])
def test_shapelet_envelope_is_dft_of_image_basis(n1, n2):
    """Image-plane basis phi_n1(x/s1) phi_n2(y/s2) (Sec. 2 Eqs. basis_1D/2D with
    sigma = beta / (2 sqrt(2 ln 2))) in the frame x = l sin(pa) + m cos(pa),
    y = l cos(pa) - m sin(pa); its DFT under exp(-2 pi i (ul + vm)) equals
    2 pi s1 s2 times the oracle's envelope with that single coefficient.  This
    fixes the (-i)^(n1+n2) factor, the kappa scaling and the axis assignment."""
    L, M, dA = _pixel_grid(1.2, 801)
    beta1, beta2, pa = 14 * synth.ARCMIN, 19 * synth.ARCMIN, 0.6
    s1, s2 = beta1 * FWHM_TO_SIGMA, beta2 * FWHM_TO_SIGMA
    x = L * math.sin(pa) + M * math.cos(pa)
    y = L * math.cos(pa) - M * math.sin(pa)
    h1 = sps.eval_hermite(n1, x / s1) * np.exp(-(x / s1) ** 2 / 2) / math.sqrt(2.0 ** n1 * math.factorial(n1) * math.sqrt(math.pi))
    h2 = sps.eval_hermite(n2, y / s2) * np.exp(-(y / s2) ** 2 / 2) / math.sqrt(2.0 ** n2 * math.factorial(n2) * math.sqrt(math.pi))
    img = h1 * h2
    n = n1 + n2
    nm = max(n, 1)
    n1s, n2s = synth.shapelet_orders(nm)
    c = np.zeros(n1s.size)
    c[np.nonzero((n1s == n1) & (n2s == n2))[0][0]] = 1.0
    for u, v in [(0.0, 0.0), (90.0, -30.0), (-150.0, 210.0), (40.0, 260.0)]:
        ref = _dft(img, L, M, dA, u, v, sign=-1)
        a, b = oracle.shapelet_args(u, v, beta1, beta2, pa)
        got = oracle.shapelet_envelope_ab(nm, c, a, b, sign=-1)
        assert abs(got - ref / (2 * math.pi * s1 * s2)) < 1e-8, (u, v, got, ref)


def test_shapelet_00_equals_gaussian():
    """Sec. 3.2: with beta1 = theta_maj, beta2 = theta_min the (0,0) basis
    reproduces the Gaussian envelope (normalised to one at the origin)."""
    maj, mn, pa = 17 * synth.ARCMIN, 6 * synth.ARCMIN, 1.1
    c00 = 1.0 / oracle.hermite(0, 0.0)[0] ** 2
    for u, v in [(0, 0), (33.0, -140.0), (250.0, 75.0), (-500.0, 20.0)]:
        a, b = oracle.shapelet_args(u, v, maj, mn, pa)
        xs = oracle.shapelet_envelope_ab(0, [c00], a, b)
        assert abs(xs - oracle.gauss_envelope(u, v, maj, mn, pa)) < 1e-15


def test_shapelet_sign_flip_is_conjugate():
    n = 12
    c = np.random.default_rng(5).normal(size=(n + 2) * (n + 1) // 2)
    for a, b in [(0.3, 1.9), (-2.2, 0.8), (5.0, -4.0)]:
        assert oracle.shapelet_envelope_ab(n, c, a, b, 1) == np.conj(oracle.shapelet_envelope_ab(n, c, a, b, -1))


# --------------------------------------------------------------------------
# whole predictions: closed forms and identities
# --------------------------------------------------------------------------

def _radec_from_lm(l, m, ra0=synth.RA0_RAD, dec0=synth.DEC0_RAD):
    n = math.sqrt(1 - l * l - m * m)
    east = np.array([-math.sin(ra0), math.cos(ra0), 0])
    north = np.array([-math.sin(dec0) * math.cos(ra0), -math.sin(dec0) * math.sin(ra0), math.cos(dec0)])
    d = l * east + m * north + n * _dir(ra0, dec0)
    return math.atan2(d[1], d[0]), math.asin(d[2])


def _obs(uvw, freqs, beam=0.0):
    uvw = np.asarray(uvw, np.float64).reshape(1, -1, 3)
    f = np.asarray(freqs, np.float64)
    return synth.Obs(n_time=1, n_bl=uvw.shape[1], n_chan=f.size, uvw_m=uvw, freq_hz=f,
                     beam_fwhm_rad=beam, beam_nu_ref_hz=150e6 if beam else 0.0)


def _one(kind, ra, dec, sref=1.0, alpha=0.0, **kw):
    s = synth.empty_sky()
    if kind == "p":
        s.p_ra, s.p_dec, s.p_sref, s.p_alpha = (np.array([x]) for x in (ra, dec, sref, alpha))
    elif kind == "g":
        s.g_ra, s.g_dec, s.g_sref, s.g_alpha = (np.array([x]) for x in (ra, dec, sref, alpha))
        s.g_maj, s.g_min, s.g_pa = (np.array([kw[k]]) for k in ("maj", "mn", "pa"))
    else:
        s.s_ra, s.s_dec, s.s_sref, s.s_alpha = (np.array([x]) for x in (ra, dec, sref, alpha))
        s.s_beta1, s.s_beta2, s.s_pa = (np.array([kw[k]]) for k in ("b1", "b2", "pa"))
        s.s_nmax = np.array([kw["nmax"]], np.int32)
        s.s_coeff_off = np.array([0], np.int64)
        s.coeffs = np.asarray(kw["coeffs"], np.float64)
    return s


def _random_uvw(n, seed=0, scale=1500.0):
    return np.random.default_rng(seed).normal(size=(n, 3)) * scale


def test_point_at_phase_centre_is_its_flux():
    obs = _obs(_random_uvw(64), [150e6, 170e6, 190e6])
    sky = _one("p", synth.RA0_RAD, synth.DEC0_RAD, sref=3.0, alpha=-0.7)
    V = oracle.predict(obs, sky)
    S = 3.0 * (obs.freq_hz / 180e6) ** -0.7
    assert np.max(np.abs(V[0] - S[None, :])) < 1e-14


def test_symmetric_point_pair_is_real_cosine():
    uvw = _random_uvw(40, 1)
    uvw[:, 2] = 0.0
    obs = _obs(uvw, [160e6, 180e6])
    l, m = 0.05, -0.08
    a = _one("p", *_radec_from_lm(l, m), sref=2.0)
    b = _one("p", *_radec_from_lm(-l, -m), sref=2.0)
    V = oracle.predict(obs, synth.concat_skies(a, b))
    lam = synth.C_LIGHT / obs.freq_hz
    u = uvw[:, 0:1] / lam
    v = uvw[:, 1:2] / lam
    ref = 4.0 * np.cos(2 * math.pi * (u * l + v * m))
    # phases reach ~1.4e3 rad here; 1e-11 is a few FP64 ulps of the phase
    assert np.max(np.abs(V[0] - ref)) < 1e-11


def test_gaussian_at_phase_centre_and_zero_width_limit():
    obs = _obs(_random_uvw(30, 2), [175e6])
    g = _one("g", synth.RA0_RAD, synth.DEC0_RAD, sref=1.5, maj=9 * synth.ARCMIN, mn=4 * synth.ARCMIN, pa=0.4)
    V = oracle.predict(obs, g)[0, :, 0]
    lam = synth.C_LIGHT / 175e6
    ref = [1.5 * oracle.gauss_envelope(w[0] / lam, w[1] / lam, 9 * synth.ARCMIN, 4 * synth.ARCMIN, 0.4)
           for w in obs.uvw_m[0]]
    assert np.max(np.abs(V - ref)) < 1e-15
    assert np.max(np.abs(V.imag)) == 0.0
    # a vanishing Gaussian is a point
    ra, dec = _radec_from_lm(0.03, 0.02)
    g0 = _one("g", ra, dec, maj=1e-12, mn=1e-12, pa=0.0)
    p0 = _one("p", ra, dec)
    assert np.max(np.abs(oracle.predict(obs, g0) - oracle.predict(obs, p0))) < 1e-12


def test_shapelet_00_at_phase_centre_equals_gaussian_prediction():
    obs = _obs(_random_uvw(50, 3), [170e6, 185e6])
    maj, mn, pa = 11 * synth.ARCMIN, 7 * synth.ARCMIN, 2.0
    c00 = 1.0 / oracle.hermite(0, 0.0)[0] ** 2
    s = _one("s", synth.RA0_RAD, synth.DEC0_RAD, sref=2.0, alpha=-0.8, b1=maj, b2=mn, pa=pa, nmax=0, coeffs=[c00])
    g = _one("g", synth.RA0_RAD, synth.DEC0_RAD, sref=2.0, alpha=-0.8, maj=maj, mn=mn, pa=pa)
    assert np.max(np.abs(oracle.predict(obs, s) - oracle.predict(obs, g))) < 1e-14


def test_hermitian_symmetry_linearity_sign_and_channel_scaling():
    obs, sky = synth.make_config(0, n_tiles=12)
    V = oracle.predict(obs, sky)
    neg = synth.Obs(**{**obs.__dict__, "uvw_m": -obs.uvw_m})
    assert np.max(np.abs(oracle.predict(neg, sky) - np.conj(V))) < 1e-11
    assert np.max(np.abs(oracle.predict(obs, sky, sign=+1) - np.conj(V))) == 0.0
    a = synth.select_components(sky, points=range(0, 50), gauss=[], shapelets=[])
    b = synth.select_components(sky, points=range(50, 100), gauss=None, shapelets=None)
    assert np.max(np.abs(oracle.predict(obs, a) + oracle.predict(obs, b) - V)) < 1e-11
    # alpha = 0, flat beam: V depends on uvw only through uvw * nu
    flat = synth.select_components(sky)
    flat.p_alpha = np.zeros_like(flat.p_alpha)
    flat.g_alpha = np.zeros_like(flat.g_alpha)
    flat.s_alpha = np.zeros_like(flat.s_alpha)
    obs2 = synth.Obs(**{**obs.__dict__, "uvw_m": obs.uvw_m * 2.0, "freq_hz": obs.freq_hz / 2.0})
    assert np.max(np.abs(oracle.predict(obs2, flat) - oracle.predict(obs, flat))) < 1e-10


def test_beam_reduces_to_flat_at_phase_centre_and_attenuates_off_axis():
    uvw = _random_uvw(8, 4)
    flat, beamed = _obs(uvw, [150e6, 200e6]), _obs(uvw, [150e6, 200e6], beam=math.radians(25))
    p = _one("p", synth.RA0_RAD, synth.DEC0_RAD)
    assert np.max(np.abs(oracle.predict(flat, p) - oracle.predict(beamed, p))) == 0.0
    rho = math.radians(12.5)
    ra, dec = synth.offset_to_radec(np.array([rho]), np.array([0.3]))
    q = _one("p", float(ra[0]), float(dec[0]))
    # FWHM 25 deg at 150 MHz: a source 12.5 deg out sits at half power
    ft = oracle.flux_table(beamed, q)
    assert abs(ft[0, 0] - 0.5) < 1e-12
    assert abs(ft[0, 1] - 2.0 ** -((200 / 150) ** 2)) < 1e-12


def _mp_phi(n, x):
    x = mpmath.mpf(x)
    return [mpmath.hermite(k, x) * mpmath.exp(-x * x / 2) / mpmath.sqrt(mpmath.mpf(2) ** k * mpmath.factorial(k) * mpmath.sqrt(mpmath.pi)) for k in range(n + 1)]


def _mp_frame(ra, dec):
    sa, ca, sd, cd = mpmath.sin(ra), mpmath.cos(ra), mpmath.sin(dec), mpmath.cos(dec)
    return mpmath.matrix([[-sa, ca, 0], [-sd * ca, -sd * sa, cd], [cd * ca, cd * sa, sd]])


def test_whole_sum_against_mpmath_brute_force():
    """50-digit evaluation of the tiny workload on 64 random visibilities."""
    mpmath.mp.dps = 50
    obs, sky = synth.make_config(0)
    rng = np.random.default_rng(11)
    rows = rng.choice(obs.n_time * obs.n_bl, 16, replace=False)
    V = oracle.predict(obs, sky, rows=rows)
    F = oracle.total_flux(obs, sky)
    T0 = _mp_frame(mpmath.mpf(obs.ra0), mpmath.mpf(obs.dec0))
    c = mpmath.mpf(synth.C_LIGHT)
    comps = []
    for kind, n in (("p", sky.n_point), ("g", sky.n_gauss), ("s", sky.n_shp)):
        pre = {"p": "p_", "g": "g_", "s": "s_"}[kind]
        for j in range(n):
            ra, dec = mpmath.mpf(getattr(sky, pre + "ra")[j]), mpmath.mpf(getattr(sky, pre + "dec")[j])
            sv = mpmath.matrix([mpmath.cos(dec) * mpmath.cos(ra), mpmath.cos(dec) * mpmath.sin(ra), mpmath.sin(dec)])
            lmn = T0 * sv
            comps.append((kind, j, lmn, (_mp_frame(ra, dec) * T0.T) if kind == "s" else None))
    kap = mpmath.pi / mpmath.sqrt(2 * mpmath.log(2))
    worst = 0.0
    for ri, row in enumerate(rows):
        t, b = divmod(int(row), obs.n_bl)
        um = [mpmath.mpf(x) for x in obs.uvw_m[t, b]]
        for k in range(obs.n_chan):
            nu = mpmath.mpf(obs.freq_hz[k])
            u, v, w = (x * nu / c for x in um)
            acc = mpmath.mpc(0)
            for kind, j, lmn, R in comps:
                pre = {"p": "p_", "g": "g_", "s": "s_"}[kind]
                S = mpmath.mpf(getattr(sky, pre + "sref")[j]) * (nu / mpmath.mpf(sky.nu_ref_hz)) ** mpmath.mpf(getattr(sky, pre + "alpha")[j])
                l, m, n = lmn[0], lmn[1], lmn[2]
                ph = mpmath.expj(-2 * mpmath.pi * (u * l + v * m + w * (n - 1)))
                env = mpmath.mpf(1)
                if kind == "g":
                    pa = mpmath.mpf(sky.g_pa[j])
                    kx = mpmath.cos(pa) * v + mpmath.sin(pa) * u
                    ky = -mpmath.sin(pa) * v + mpmath.cos(pa) * u
                    env = mpmath.exp(-mpmath.pi ** 2 / (4 * mpmath.log(2)) * (kx ** 2 * mpmath.mpf(sky.g_maj[j]) ** 2 + ky ** 2 * mpmath.mpf(sky.g_min[j]) ** 2))
                elif kind == "s":
                    up = R[0, 0] * u + R[0, 1] * v + R[0, 2] * w
                    vp = R[1, 0] * u + R[1, 1] * v + R[1, 2] * w
                    pa = mpmath.mpf(sky.s_pa[j])
                    a = kap * mpmath.mpf(sky.s_beta1[j]) * (mpmath.cos(pa) * vp + mpmath.sin(pa) * up)
                    bb = kap * mpmath.mpf(sky.s_beta2[j]) * (-mpmath.sin(pa) * vp + mpmath.cos(pa) * up)
                    N = int(sky.s_nmax[j])
                    pa_, pb_ = _mp_phi(N, a), _mp_phi(N, bb)
                    o = int(sky.s_coeff_off[j])
                    env = mpmath.mpc(0)
                    idx = 0
                    for n1 in range(N + 1):
                        for n2 in range(N + 1 - n1):
                            env += mpmath.mpf(sky.coeffs[o + idx]) * (-1j) ** (n1 + n2) * pa_[n1] * pb_[n2]
                            idx += 1
                acc += S * env * ph
            worst = max(worst, abs(complex(acc) - V[ri, k]) / F[k])
    # phases reach ~1e3 rad: FP64 rounding of the phase bounds the oracle at ~1e-13 of total flux
    assert worst < 2e-13


def test_error_metric_definition():
    obs, sky = synth.make_config(0, n_tiles=6)
    V = oracle.predict(obs, sky)
    F = oracle.total_flux(obs, sky)
    W = V.copy()
    W[0, 3, 2] += 0.5 * F[2]
    assert abs(oracle.error_metric(W, V, obs, sky) - 0.5) < 1e-12
    assert oracle.error_metric(V, V, obs, sky) == 0.0


def test_generated_shapelets_are_normalised():
    for idx in (0, 2):
        obs, sky = synth.make_config(idx, n_tiles=4, n_time=1, n_chan=1, n_point=1, n_gauss=1) if idx == 0 else synth.make_config(2, n_tiles=4, n_time=1, n_chan=1)
        x0 = oracle.xi_origin(sky)[sky.n_point + sky.n_gauss:]
        assert np.max(np.abs(x0 - 1.0)) < 1e-12
