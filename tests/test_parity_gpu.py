"""GPU parity: libvp's HIP kernels against the FP64 oracle, element by element,
on seeded synthetic inputs.

Error metric: max over channels of max |V_gpu - V_oracle| / F_k, F_k the total
flux of channel k (sum of |S_j(nu_k)| |xi_j(0)|).  Bars: 1e-11 for the FP64
path, 1e-6 for the mixed paths (FP64 phase, FP32 sincos/envelopes/MFMA
contraction, Kahan sums).  The FP32-only path is reported, not gated.

Sizes here span several 256-row tiles with ragged row and channel tails; the
full-size workloads are checked on sampled rows in test_fullsize_gpu.py."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from paper_2005_09316_amd import vp
from tests.helpers import Handles, run

pytestmark = pytest.mark.gpu

TOL = {vp.VP_PREC_FP64: 1e-11, vp.VP_PREC_MIXED: 1e-6, vp.VP_PREC_MIXED_BF16: 1e-6}


@pytest.fixture(scope="module")
def ctx():
    c = vp.vp_create_ctx(0, 0)
    yield c
    vp.vp_destroy_ctx(c)


def _case(name):
    if name == "tiny":
        return synth.make_config(0)
    if name == "mwa-mid":
        # 24 tiles (276 baselines) x 3 times = 828 rows: 4 row tiles, ragged;
        # 13 channels: ragged against 8- and 4-channel blocks; beam on.
        return synth.make_config(1, n_tiles=24, n_time=3, n_chan=13, n_point=300, n_gauss=60,
                                 shapelet_nmax=[54, 33])
    if name == "fornax-mid":
        return synth.make_config(2, n_tiles=20, n_time=2, n_chan=6)
    if name == "mwa-nonuniform":
        # channels at irregular frequencies: the mixed path evaluates every
        # channel's phasor (no rotation between channels)
        rng = np.random.default_rng(31)
        freqs = np.sort(rng.uniform(170e6, 190e6, 11))
        return synth.make_config(1, n_tiles=20, n_time=2, n_chan=11, n_point=200, n_gauss=40,
                                 shapelet_nmax=[20], freq_hz=freqs)
    if name == "lobes-only":
        # shapelets only: no point/Gaussian pass runs, the shapelet pass starts
        # from zero (the output buffer holds NaN before a predict)
        obs, sky = synth.make_config(2, n_tiles=20, n_time=2, n_chan=6)
        return obs, synth.select_components(sky, points=[], gauss=[])
    if name == "mwa-descending":
        # uniformly spaced channels in decreasing frequency: a negative channel
        # step for the phasor rotations and the FP64 envelope recurrence
        freqs = np.linspace(190e6, 170e6, 11)
        return synth.make_config(1, n_tiles=20, n_time=2, n_chan=11, n_point=200, n_gauss=40,
                                 shapelet_nmax=[20], freq_hz=freqs)
    if name == "mwa-jittered":
        # a grid uniform to 1e-13 of nu: the mixed path rotates phasors, the
        # FP64 path (which rotates only on grids uniform to 1e-15) does not
        rng = np.random.default_rng(32)
        freqs = np.linspace(170e6, 190e6, 11) * (1.0 + 1e-13 * rng.uniform(-1.0, 1.0, 11))
        return synth.make_config(1, n_tiles=20, n_time=2, n_chan=11, n_point=200, n_gauss=40,
                                 shapelet_nmax=[20], freq_hz=freqs)
    if name == "nmax-limit":
        return synth.make_config(0, n_tiles=16, n_time=2, n_chan=5, n_point=3, n_gauss=2,
                                 shapelet_nmax=[96, 0, 1, 31, 32, 63, 64])
    if name == "nmax-chunks":
        # orders on either side of every 16-order boundary below 96 (the FP64
        # kernel's second-axis chunks; 32-order blocks elsewhere), 7 channels
        # (ragged against 4-channel tiles)
        return synth.make_config(0, n_tiles=16, n_time=2, n_chan=7, n_point=3, n_gauss=2,
                                 shapelet_nmax=[15, 16, 17, 47, 48, 49, 79, 80, 81])
    raise KeyError(name)


CASES = ["tiny", "mwa-mid", "fornax-mid", "lobes-only", "mwa-nonuniform", "mwa-descending", "mwa-jittered",
         "nmax-limit", "nmax-chunks"]
_REF = {}


def _ref(name):
    if name not in _REF:
        obs, sky = _case(name)
        _REF[name] = (obs, sky, oracle.predict(obs, sky))
    return _REF[name]


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("prec,dtype", [(vp.VP_PREC_FP64, vp.VP_C128), (vp.VP_PREC_MIXED, vp.VP_C128),
                                        (vp.VP_PREC_MIXED, vp.VP_C64), (vp.VP_PREC_MIXED_BF16, vp.VP_C128)])
def test_predict_matches_oracle(ctx, name, prec, dtype):
    obs, sky, ref = _ref(name)
    _log("case", name, "prec", prec, "dtype", dtype, "vis", obs.n_vis)
    with Handles(ctx, obs, sky) as h:
        got = run(ctx, h.obs, h.sky, obs, prec, dtype)
    err = oracle.error_metric(got, ref, obs, sky)
    _log("  error / total flux = %.3e" % err)
    tol = TOL[prec]
    if dtype == vp.VP_C64:
        tol = max(tol, 1e-6)
    assert np.all(np.isfinite(got))
    assert err <= tol


@pytest.mark.parametrize("name", ["tiny", "fornax-mid", "nmax-limit"])
@pytest.mark.parametrize("prec", [vp.VP_PREC_FP32, vp.VP_PREC_MIXED_BF16X2])
def test_reported_paths(ctx, name, prec):
    """FP32-only and 2-way BF16 contraction paths: their error is reported,
    not held to the 1e-6 target.  The bound here only catches a broken path
    (a dropped term, a wrong sign or index errs by O(1) of the total flux):
    the arithmetic of these paths (FP32 recurrences and sums; a second-axis
    value carried in two BF16 parts, 2^-17 relative) measured at most 1.5e-4
    of the total flux over every Fornax-like visibility."""
    obs, sky, ref = _ref(name)
    with Handles(ctx, obs, sky) as h:
        got = run(ctx, h.obs, h.sky, obs, prec, vp.VP_C64)
    err = oracle.error_metric(got, ref, obs, sky)
    _log("precision %d, case %s: error / total flux = %.3e (reported)" % (prec, name, err))
    assert np.all(np.isfinite(got))
    assert err <= 1e-3


@pytest.mark.parametrize("prec,dtype", [(vp.VP_PREC_FP64, vp.VP_C128), (vp.VP_PREC_MIXED, vp.VP_C64)])
def test_subtract_matches_oracle_residual(ctx, prec, dtype):
    obs, sky, ref = _ref("mwa-mid")
    rng = np.random.default_rng(17)
    data = ref + (rng.standard_normal(ref.shape) + 1j * rng.standard_normal(ref.shape))
    if dtype == vp.VP_C64:
        data = data.astype(np.complex64).astype(np.complex128)
    with Handles(ctx, obs, sky) as h:
        got = run(ctx, h.obs, h.sky, obs, prec, dtype, data=data)
    err = oracle.error_metric(got, data - ref, obs, sky)
    _log("subtract prec %d: error / total flux = %.3e" % (prec, err))
    assert err <= TOL[prec] if dtype == vp.VP_C128 else err <= 1e-6


def test_sign_flip_is_exact_conjugate(ctx):
    obs, sky, _ = _ref("mwa-mid")
    plus = synth.Obs(**{**obs.__dict__, "sign": +1})
    for prec in (vp.VP_PREC_FP64, vp.VP_PREC_MIXED):
        with Handles(ctx, obs, sky) as h, Handles(ctx, plus, sky) as hp:
            a = run(ctx, h.obs, h.sky, obs, prec, vp.VP_C128)
            b = run(ctx, hp.obs, hp.sky, plus, prec, vp.VP_C128)
        assert np.array_equal(a, np.conj(b))


def test_deterministic_bitwise(ctx):
    obs, sky, _ = _ref("fornax-mid")
    with Handles(ctx, obs, sky) as h:
        a = run(ctx, h.obs, h.sky, obs, vp.VP_PREC_MIXED, vp.VP_C64)
        b = run(ctx, h.obs, h.sky, obs, vp.VP_PREC_MIXED, vp.VP_C64)
    assert np.array_equal(a, b)


def test_subtract_of_predict_is_zero_and_linearity(ctx):
    obs, sky, _ = _ref("mwa-mid")
    a = synth.select_components(sky, points=range(0, 150), gauss=range(0, 30), shapelets=[0])
    b = synth.select_components(sky, points=range(150, 300), gauss=range(30, 60), shapelets=[1])
    with Handles(ctx, obs, sky) as h, Handles(ctx, obs, a) as ha, Handles(ctx, obs, b) as hb:
        full = run(ctx, h.obs, h.sky, obs, vp.VP_PREC_FP64, vp.VP_C128)
        va = run(ctx, ha.obs, ha.sky, obs, vp.VP_PREC_FP64, vp.VP_C128)
        vb = run(ctx, hb.obs, hb.sky, obs, vp.VP_PREC_FP64, vp.VP_C128)
        zero = run(ctx, h.obs, h.sky, obs, vp.VP_PREC_FP64, vp.VP_C128, data=full)
    F = oracle.total_flux(obs, sky)
    assert np.max(np.abs(zero) / F) < 1e-13
    assert oracle.error_metric(va + vb, full, obs, sky) < 1e-12


def test_empty_sky_and_edge_shapes(ctx):
    obs, sky = synth.make_config(0, n_tiles=3, n_time=1, n_chan=1)
    empty = synth.empty_sky()
    for prec in (vp.VP_PREC_FP64, vp.VP_PREC_MIXED):
        with Handles(ctx, obs, empty) as h:
            z = run(ctx, h.obs, h.sky, obs, prec, vp.VP_C128)
            assert np.all(z == 0)
            d = np.arange(obs.n_vis).reshape(1, obs.n_bl, 1) * (1 + 2j)
            same = run(ctx, h.obs, h.sky, obs, prec, vp.VP_C128, data=d)
            assert np.array_equal(same, d)
    # one row, one channel, each component kind alone
    for sel in ({"points": [0], "gauss": [], "shapelets": []}, {"points": [], "gauss": [0], "shapelets": []},
                {"points": [], "gauss": [], "shapelets": [0]}):
        s = synth.select_components(sky, **sel)
        one = synth.Obs(**{**obs.__dict__, "n_bl": 1, "uvw_m": obs.uvw_m[:, :1]})
        ref = oracle.predict(one, s)
        for prec in (vp.VP_PREC_FP64, vp.VP_PREC_MIXED):
            with Handles(ctx, one, s) as h:
                got = run(ctx, h.obs, h.sky, one, prec, vp.VP_C128)
            assert oracle.error_metric(got, ref, one, s) <= TOL[prec]


def test_invalid_inputs_rejected(ctx):
    obs, sky = synth.make_config(0, n_tiles=4)
    import torch
    out = torch.empty((obs.n_time * obs.n_bl, obs.n_chan), dtype=torch.complex128, device="cuda")
    with Handles(ctx, obs, sky) as h:
        for prec in (vp.VP_PREC_MIXED_F32MMA, -1, 7):  # retired, below and above the range
            with pytest.raises(vp.VPError) as e:
                vp.vp_predict(ctx, h.sky, h.obs, prec, vp.VP_C128, out.data_ptr(), 0)
            assert e.value.code == vp.VP_EINVAL
    bad = synth.Obs(**{**obs.__dict__, "sign": 2})
    with pytest.raises(vp.VPError) as e:
        vp.vp_create_obs(ctx, bad)
    assert e.value.code == vp.VP_EINVAL
    nan = synth.Obs(**{**obs.__dict__, "uvw_m": obs.uvw_m * np.nan})
    with pytest.raises(vp.VPError):
        vp.vp_create_obs(ctx, nan)
    s2 = synth.select_components(sky)
    s2.s_nmax = np.array([97], np.int32)
    with pytest.raises(vp.VPError):
        vp.vp_create_sky(ctx, s2)
    s3 = synth.select_components(sky)
    s3.s_beta1 = np.array([0.0])
    with pytest.raises(vp.VPError):
        vp.vp_create_sky(ctx, s3)
    with Handles(ctx, obs, sky) as h:
        with pytest.raises(vp.VPError):
            vp.vp_predict(ctx, h.sky, h.obs, 7, vp.VP_C64, 1234, 0)
        with pytest.raises(vp.VPError):
            vp.vp_predict(ctx, h.sky, h.obs, vp.VP_PREC_MIXED, 5, 1234, 0)


def test_effective_order_and_truncation(ctx):
    """A shapelet whose coefficients vanish above order 20 gives the same
    visibilities, bit for bit, whether declared with nmax 40 or 20 (the
    library keeps the effective order); an order-truncated and a flux-truncated
    model match the oracle of the same truncated model."""
    import dataclasses

    from paper_2005_09316_amd import truncate
    obs, sky = synth.make_config(0, n_tiles=16, n_time=2, n_chan=5, n_point=2, n_gauss=1, shapelet_nmax=[40])
    t40 = truncate.truncate_by_order(sky, 20)
    n1, n2 = truncate._orders(40)
    t20 = dataclasses.replace(t40, s_nmax=np.array([20], np.int32), coeffs=t40.coeffs[n1 + n2 <= 20])
    outs = []
    for sk in (t40, t20):
        with Handles(ctx, obs, sk) as h:
            outs.append(run(ctx, h.obs, h.sky, obs, vp.VP_PREC_MIXED, vp.VP_C128))
    assert np.array_equal(outs[0], outs[1])
    ref = oracle.predict(obs, t20)
    err = oracle.error_metric(outs[1], ref, obs, t20)
    _log("order-truncated shapelet (20 of 40): error / total flux = %.3e" % err)
    assert err <= 1e-6
    tf, n, ntot, frac = truncate.truncate_by_flux(sky, 0.8)
    with Handles(ctx, obs, tf) as h:
        got = run(ctx, h.obs, h.sky, obs, vp.VP_PREC_MIXED, vp.VP_C128)
    err = oracle.error_metric(got, oracle.predict(obs, tf), obs, tf)
    _log("flux-truncated model (%d of %d kept): error / total flux = %.3e" % (n, ntot, err))
    assert err <= 1e-6


def test_lookup_table_variant_within_interpolation_bound(ctx):
    """VP_PREC_LUT reads the basis from an FP32 table of phi_n on a uniform
    grid of step h = 32/8192 with linear interpolation (the paper's
    simulator's evaluation, Sec. 3.2).  Bound from the oracle's Hermite
    functions: the interpolation error of phi_n is at most
    h^2/8 max|phi_n''| with phi_n'' = (x^2 - 2n - 1) phi_n, plus FP32
    rounding of the table and the interpolation (3 * 2^-24 * pi^(-1/4));
    with e = the largest of these over the orders used and M = pi^(-1/4)
    (|phi_n| <= M), each shapelet's envelope moves by at most
    sum |C| (2 e M + e^2), and the flux-weighted sum of that over the
    shapelets, against the total flux, bounds the error metric."""
    obs, sky = synth.make_config(0, n_tiles=16, n_time=2, n_chan=3, n_point=2, n_gauss=1,
                                 shapelet_nmax=[30, 12])
    nmax = int(max(sky.s_nmax))
    h = 32.0 / 8192
    xs = np.linspace(0.0, 32.0, 4001)
    phi = np.array([oracle.hermite(nmax, x) for x in xs])           # [x][n]
    n = np.arange(nmax + 1)
    d2 = np.abs((xs[:, None] ** 2 - 2 * n[None, :] - 1) * phi).max()
    M = math.pi ** -0.25
    e = h * h / 8.0 * d2 + 3 * 2.0 ** -24 * M
    ft = np.abs(oracle.flux_table(obs, sky))                        # [J][K]
    j0 = sky.n_point + sky.n_gauss
    bound_abs = np.zeros(obs.n_chan)
    for s in range(sky.n_shp):
        N = int(sky.s_nmax[s])
        c = sky.coeffs[int(sky.s_coeff_off[s]):int(sky.s_coeff_off[s]) + (N + 1) * (N + 2) // 2]
        bound_abs += ft[j0 + s] * np.abs(c).sum() * (2 * e * M + e * e)
    bound = float((bound_abs / oracle.total_flux(obs, sky)).max())
    ref = oracle.predict(obs, sky)
    with Handles(ctx, obs, sky) as hd:
        got = run(ctx, hd.obs, hd.sky, obs, vp.VP_PREC_LUT, vp.VP_C128)
        exact = run(ctx, hd.obs, hd.sky, obs, vp.VP_PREC_FP64, vp.VP_C128)
    err = oracle.error_metric(got, ref, obs, sky)
    err64 = oracle.error_metric(exact, ref, obs, sky)
    _log("lookup-table basis: error / total flux %.3e (bound %.3e); recurrence %.3e" % (err, bound, err64))
    assert np.all(np.isfinite(got))
    assert err <= bound
    assert err64 <= TOL[vp.VP_PREC_FP64]


@pytest.mark.parametrize("prec,dtype", [(vp.VP_PREC_FP64, vp.VP_C128), (vp.VP_PREC_MIXED, vp.VP_C128),
                                        (vp.VP_PREC_MIXED, vp.VP_C64)])
def test_spectral_terms_match_oracle(ctx, prec, dtype):
    """Shapelets whose coefficients vary with frequency, C(nu) = sum_q C_q
    ln(nu/nu_ref)^q (3 terms), over a 150-200 MHz band so that ln(nu/nu_ref)
    reaches +-0.15; same bars as the plain model (error relative to the
    channel's total flux, with xi(0) taken at that channel)."""
    import dataclasses
    obs, sky = synth.make_config(2, n_tiles=16, n_time=2, n_chan=5, shapelet_nmax=[40, 33])
    obs = dataclasses.replace(obs, freq_hz=np.linspace(150e6, 200e6, 5))
    multi = synth.with_spectral_terms(sky, np.random.default_rng(21), 3, scale=0.5)
    ref = oracle.predict(obs, multi)
    _log("spectral terms: prec", prec, "dtype", dtype)
    with Handles(ctx, obs, multi) as h:
        got = run(ctx, h.obs, h.sky, obs, prec, dtype)
    err = oracle.error_metric(got, ref, obs, multi)
    _log("  error / total flux = %.3e" % err)
    tol = TOL[prec] if dtype == vp.VP_C128 else max(TOL[prec], 1e-6)
    assert np.all(np.isfinite(got))
    assert err <= tol


def test_spectral_terms_rejected_outside_limits(ctx):
    obs, sky = synth.make_config(0, n_tiles=6, n_chan=2, shapelet_nmax=[4])
    import dataclasses
    for q in (0, vp.VP_NTERM_LIMIT + 1):
        bad = dataclasses.replace(sky, s_nterm=np.array([q], np.int32),
                                  coeffs=np.tile(sky.coeffs, max(q, 1)))
        with pytest.raises(vp.VPError):
            vp.vp_create_sky(ctx, bad)


def _random_case(seed):
    """A small seeded configuration with irregular sizes: 2-40 tiles, 1-3
    times, 1-13 channels (uniformly or irregularly spaced), 0-300 points,
    0-40 Gaussians, 0-3 shapelets of order 0-96."""
    import dataclasses
    rng = np.random.default_rng(9000 + seed)
    n_tiles = int(rng.integers(2, 41))
    n_time = int(rng.integers(1, 4))
    n_chan = int(rng.integers(1, 14))
    if rng.random() < 0.5:
        freqs = np.linspace(150e6, 200e6, n_chan) if n_chan > 1 else np.array([182e6])
    else:
        freqs = np.sort(rng.uniform(150e6, 200e6, n_chan))
    nmax = [int(x) for x in rng.integers(0, 97, int(rng.integers(0, 4)))]
    obs, sky = synth.make_config(1, seed=9100 + seed, n_tiles=n_tiles, n_time=n_time, n_chan=n_chan,
                                 n_point=int(rng.integers(0, 301)), n_gauss=int(rng.integers(0, 41)),
                                 shapelet_nmax=nmax, freq_hz=freqs)
    if rng.random() < 0.3:
        obs = dataclasses.replace(obs, beam_fwhm_rad=0.0, beam_nu_ref_hz=0.0)
    return obs, sky


@pytest.mark.parametrize("seed", range(12))
def test_random_configurations(ctx, seed):
    obs, sky = _random_case(seed)
    _log("random case %d: tiles %d, times %d, channels %d, points %d, Gaussians %d, shapelet orders %s"
         % (seed, obs.n_tiles, obs.n_time, obs.n_chan, sky.n_point, sky.n_gauss, list(sky.s_nmax)))
    ref = oracle.predict(obs, sky)
    F = oracle.total_flux(obs, sky)
    with Handles(ctx, obs, sky) as h:
        for prec, dtype in ((vp.VP_PREC_FP64, vp.VP_C128), (vp.VP_PREC_MIXED, vp.VP_C64)):
            got = run(ctx, h.obs, h.sky, obs, prec, dtype)
            assert np.all(np.isfinite(got))
            if not np.any(F > 0):
                assert np.max(np.abs(got)) == 0.0
                continue
            err = oracle.error_metric(got, ref, obs, sky)
            _log("  precision %d: error / total flux %.3e" % (prec, err))
            assert err <= (TOL[prec] if dtype == vp.VP_C128 else 1e-6)
