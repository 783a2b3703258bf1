"""CPU checks of the seeded input generator and of bench.py's contract."""
import json
import math
import os
import subprocess
import sys

import numpy as np

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_array_and_uvw_geometry():
    rng = np.random.default_rng(1)
    e, n = synth.tile_layout(rng, 40)
    assert np.all(np.hypot(e, n) <= 1500.0)
    bl = synth.baselines_enu(e, n)
    assert bl.shape == (40 * 39 // 2, 3)
    for ha in (-0.3, 0.0, 0.2):
        uvw = synth.uvw_from_enu(bl, ha)
        # a rotation: lengths are preserved
        assert np.allclose(np.linalg.norm(uvw, axis=1), np.linalg.norm(bl, axis=1), rtol=1e-12)
    obs = synth.make_obs(rng, 12, 3, synth.channels(182e6, 80e3, 5))
    assert obs.uvw_m.shape == (3, 66, 3) and obs.n_vis == 3 * 66 * 5
    assert np.allclose(np.diff(obs.freq_hz), 80e3) and abs(obs.freq_hz.mean() - 182e6) < 1e-3


def test_workload_shapes():
    obs, sky = synth.make_config(0)
    assert (obs.n_time, obs.n_bl, obs.n_chan) == (1, 496, 4)
    assert np.allclose(obs.freq_hz, [171.25e6, 173.75e6, 176.25e6, 178.75e6])
    assert (sky.n_point, sky.n_gauss, sky.n_shp, sky.n_basis()) == (100, 10, 1, 66)
    obs1, sky1 = synth.make_config(1, n_point=10, n_gauss=5)
    assert (obs1.n_time, obs1.n_bl, obs1.n_chan) == (14, 8128, 32)
    assert obs1.beam_fwhm_rad > 0 and sky1.n_basis() == 2 * 1540
    obs4, _ = synth.make_config(4, n_point=1, n_gauss=1, shapelet_nmax=[1])
    assert obs4.n_bl == 32640 and obs4.n_chan == 384 and obs4.n_vis == 12533760


def test_flux_laws_and_positions():
    rng = np.random.default_rng(2)
    s = synth.powerlaw_counts(rng, 200000, 0.05, 50.0, -1.6)
    assert s.min() >= 0.05 and s.max() <= 50.0
    # slope of the log-log histogram of dN/dS
    edges = np.logspace(math.log10(0.05), math.log10(50.0), 25)
    h, _ = np.histogram(s, edges)
    mid = np.sqrt(edges[1:] * edges[:-1])
    good = h > 50
    slope = np.polyfit(np.log(mid[good]), np.log(h[good] / np.diff(edges)[good]), 1)[0]
    assert abs(slope + 1.6) < 0.05
    ra, dec = synth.cap_positions(rng, 5000, math.radians(10))
    for r, d in zip(ra[:200], dec[:200]):
        l, m, n1 = oracle.lmn(synth.RA0_RAD, synth.DEC0_RAD, r, d)
        assert math.asin(min(1.0, math.hypot(l, m))) <= math.radians(10) + 1e-12


def test_shapelet_coefficients_normalised_and_damped():
    rng = np.random.default_rng(3)
    for nmax in (0, 1, 10, 54, 80):
        c, redraws = synth.shapelet_coeffs(rng, nmax, 20.0)
        assert c.size == (nmax + 1) * (nmax + 2) // 2
        assert abs(oracle.shapelet_envelope_ab(nmax, c, 0.0, 0.0) - 1.0) < 1e-12


def test_serving_stream_recipe():
    reqs = synth.make_requests(64)
    t = np.array([r.t_arrival_s for r in reqs])
    assert np.all(np.diff(t) > 0)
    assert 1.5 < t[-1] < 6.0  # 64 arrivals at 20/s
    for r in reqs:
        assert r.obs.n_tiles in (64, 128, 256) and 1 <= r.obs.n_time <= 14 and 8 <= r.obs.n_chan <= 384
        assert r.sky.n_shp <= 4 and all(20 <= n <= 80 for n in r.sky.s_nmax)
    kinds = [r.kind for r in reqs]
    assert 0.25 < kinds.count("predict") / len(kinds) < 0.75


def test_paper_cost_comparison_counts():
    obs, clean, lobes = synth.make_paper_cost_comparison()
    assert (clean.n_point, clean.n_gauss) == (4540, 1791)      # Sec. 5.3
    assert lobes.n_basis() == 7656                              # Sec. 5.3
    assert (obs.n_time, obs.n_bl, obs.n_chan) == (15, 8128, 384)
    assert abs(clean.p_sref.sum() + clean.g_sref.sum() - 500.0) < 1e-9


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
