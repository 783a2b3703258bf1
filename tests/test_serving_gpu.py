"""Serving (continuous batching) on the GPU: jobs submitted together share
the persistent kernel tile by tile; each job's result must equal the same
job run alone through vp_predict / vp_subtract (bitwise: the tile device
functions and per-visibility operation order are the same), admission must
respect the HBM budget in FIFO order, and error paths must isolate."""
import sys
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2005_09316_amd import vp
from tests.helpers import vis_tensor

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _wait(ctx, tickets, timeout=120.0):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for t in tickets:
            if t not in res:
                r = vp.vp_poll(ctx, t)
                if r is not None:
                    res[t] = r
        if time.time() - t0 > timeout:
            raise TimeoutError("serving jobs did not finish in %.0f s" % timeout)
        time.sleep(0.001)
    return res


def _job_specs():
    """Uneven jobs: tiles, channels, times, component mixes, kinds, dtypes, sign."""
    specs = []
    rng = np.random.default_rng(2024)
    for i in range(10):
        tiles = int(rng.choice([6, 12, 24, 40]))
        obs, sky = synth.make_config(1, seed=500 + i, n_tiles=tiles, n_time=int(rng.integers(1, 4)),
                                     n_chan=int(rng.integers(1, 20)), n_point=int(rng.integers(0, 300)),
                                     n_gauss=int(rng.integers(0, 40)),
                                     shapelet_nmax=[int(x) for x in rng.integers(0, 60, int(rng.integers(0, 3)))])
        if i % 3 == 2:
            obs = synth.Obs(**{**obs.__dict__, "sign": +1})
        kind = vp.VP_JOB_SUBTRACT if i % 2 else vp.VP_JOB_PREDICT
        dtype = vp.VP_C64 if i % 4 < 2 else vp.VP_C128
        data = None
        if kind == vp.VP_JOB_SUBTRACT:
            data = synth.noise_c64((obs.n_time, obs.n_bl, obs.n_chan), seed=900 + i)
        specs.append((obs, sky, kind, dtype, data))
    # the phases' edge cases: shapelets alone (the point/Gaussian phase only
    # clears or passes the buffer), and points and Gaussians alone (no
    # shapelet phase), each as a predict and a subtract
    for i, (npt, ng, nmax) in enumerate(((0, 0, [44, 17]), (250, 30, []))):
        obs, sky = synth.make_config(1, seed=530 + i, n_tiles=24, n_time=2, n_chan=11, n_point=npt, n_gauss=ng,
                                     shapelet_nmax=nmax)
        specs.append((obs, sky, vp.VP_JOB_PREDICT, vp.VP_C64, None))
        specs.append((obs, sky, vp.VP_JOB_SUBTRACT, vp.VP_C128,
                      synth.noise_c64((obs.n_time, obs.n_bl, obs.n_chan), seed=940 + i)))
    return specs


@pytest.fixture(scope="module")
def ctx():
    c = vp.vp_create_ctx(0, 0)
    yield c
    vp.vp_destroy_ctx(c)


def _alone(ctx, oh, sh, obs, kind, dtype, data):
    import torch
    t = vis_tensor(obs, dtype, data)
    s = torch.cuda.current_stream()
    if kind == vp.VP_JOB_PREDICT:
        vp.vp_predict(ctx, sh, oh, vp.VP_PREC_MIXED, dtype, t.data_ptr(), s.cuda_stream)
    else:
        vp.vp_subtract(ctx, sh, oh, vp.VP_PREC_MIXED, dtype, t.data_ptr(), s.cuda_stream)
    s.synchronize()
    return t.cpu().numpy()


def test_mix_equals_alone_and_oracle(ctx):
    import torch
    specs = _job_specs()
    handles = [(vp.vp_create_obs(ctx, o), vp.vp_create_sky(ctx, s)) for o, s, _, _, _ in specs]
    alone = [_alone(ctx, oh, sh, o, k, d, x) for (oh, sh), (o, s, k, d, x) in zip(handles, specs)]
    bufs = [vis_tensor(o, d, x) for o, s, k, d, x in specs]
    torch.cuda.synchronize()
    tickets = [vp.vp_submit(ctx, k, sh, oh, vp.VP_PREC_MIXED, d, b.data_ptr())
               for (oh, sh), (o, s, k, d, x), b in zip(handles, specs, bufs)]
    res = _wait(ctx, tickets)
    assert all(r["status"] == vp.VP_OK for r in res.values())
    for i, ((o, s, k, d, x), b, a) in enumerate(zip(specs, bufs, alone)):
        mixed = b.cpu().numpy()
        assert np.array_equal(mixed, a), "job %d differs between alone and mix" % i
        ref = oracle.predict(o, s)
        if k == vp.VP_JOB_SUBTRACT:
            ref = x.astype(np.complex128) - ref
        err = oracle.error_metric(mixed.astype(np.complex128), ref, o, s) if s.nominal_components() else 0.0
        assert err <= 1e-6, (i, err)
        r = res[tickets[i]]
        assert r["t_submit"] <= r["t_admit"] <= r["t_start"] <= r["t_done"]
    _log("%d uneven jobs: mix == alone bitwise, all within 1e-6 of the oracle" % len(specs))
    launches, resident_ms = vp.vp_serve_stats(ctx)
    _log("  persistent kernels: %d launches, %.2f ms resident" % (launches, resident_ms))
    assert launches >= 2 and resident_ms > 0  # both passes ran at least once
    pairs = _overlapping_pairs([res[t] for t in tickets])
    _log("  %d pairs of jobs had tiles on the device at the same time" % pairs)
    assert pairs > 0
    for oh, sh in handles:
        vp.vp_destroy_sky(sh)
        vp.vp_destroy_obs(oh)


def _overlapping_pairs(results):
    """Pairs of jobs whose device intervals [first tile start, last tile end]
    intersect (device wall clock, one clock per device)."""
    iv = [(r["dev_first_tile"], r["dev_last_tile"]) for r in results if r["dev_last_tile"]]
    n = 0
    for i in range(len(iv)):
        for j in range(i + 1, len(iv)):
            if iv[i][0] < iv[j][1] and iv[j][0] < iv[i][1]:
                n += 1
    return n


def _bits_equal(a, b):
    import torch
    return bool(torch.equal(torch.view_as_real(a).contiguous().view(torch.int32),
                            torch.view_as_real(b).contiguous().view(torch.int32)))


def _stream_jobs():
    """Requests of the serving stream (seeded), from its largest (256 tiles,
    330-384 channels, up to 14 times, shapelets of order up to 77) to small
    ones, plus a 256-tile x 384-channel subtract job with two N = 80
    shapelets drawn by the stream's recipe."""
    import math
    reqs = synth.make_requests()
    pick = [130, 184, 172, 252, 0, 1, 2, 3]
    jobs = [(reqs[i].kind, reqs[i].obs, reqs[i].sky, reqs[i].noise_seed, "request %d" % i) for i in pick]
    rng = np.random.default_rng(31337)
    obs = synth.make_obs(rng, 256, 2, synth.channels(182e6, 80e3, 384))
    sky = synth.make_sky(rng, n_point=int(rng.poisson(2000)), n_gauss=int(rng.poisson(200)), shapelet_nmax=[80, 80],
                         cap_rad=math.radians(10.0), point_flux=synth._pl(0.05, 50.0),
                         shapelet_sref=synth._lu(1.0, 100.0), tau=20.0)
    jobs.append(("subtract", obs, sky, 4242, "256 tiles x 384 channels, N = 80"))
    return jobs


def test_stream_requests_mix_alone_oracle():
    """Serving-stream-sized jobs submitted together to fresh sky and
    observation handles, so that the persistent kernel builds every pair's
    tables itself; each result must equal vp_predict / vp_subtract on separate
    handles bit for bit and the oracle on sampled rows within 1e-6 of the
    total flux; some jobs' tiles must run on the device at the same time."""
    import torch
    jobs = _stream_jobs()
    ctx = vp.vp_create_ctx(0, 0)
    s = torch.cuda.current_stream()
    try:
        alone, mixed, handles = [], [], []
        for kind, obs, sky, seed, name in jobs:
            shape = (obs.n_time, obs.n_bl, obs.n_chan)
            g = torch.Generator(device="cuda").manual_seed(seed)
            data = torch.randn(shape, dtype=torch.complex64, device="cuda", generator=g)
            a = data.clone() if kind == "subtract" else torch.full_like(data, float("nan"))
            m = data.clone() if kind == "subtract" else torch.full_like(data, float("nan"))
            oa, sa = vp.vp_create_obs(ctx, obs), vp.vp_create_sky(ctx, sky)
            fn = vp.vp_subtract if kind == "subtract" else vp.vp_predict
            fn(ctx, sa, oa, vp.VP_PREC_MIXED, vp.VP_C64, a.data_ptr(), s.cuda_stream)
            s.synchronize()
            vp.vp_destroy_sky(sa)
            vp.vp_destroy_obs(oa)
            alone.append(a)
            mixed.append(m)
            handles.append((vp.vp_create_obs(ctx, obs), vp.vp_create_sky(ctx, sky)))
            _log("%s: %s, %d vis, %d points, %d Gaussians, shapelets %s"
                 % (name, kind, obs.n_vis, sky.n_point, sky.n_gauss, list(np.asarray(sky.s_nmax))))
            del data
        torch.cuda.synchronize()
        tickets = []
        for (kind, obs, sky, seed, name), (oh, sh), m in zip(jobs, handles, mixed):
            k = vp.VP_JOB_SUBTRACT if kind == "subtract" else vp.VP_JOB_PREDICT
            tickets.append(vp.vp_submit(ctx, k, sh, oh, vp.VP_PREC_MIXED, vp.VP_C64, m.data_ptr()))
        res = _wait(ctx, tickets, timeout=100.0)
        assert all(res[t]["status"] == vp.VP_OK for t in tickets)
        for i, ((kind, obs, sky, seed, name), a, m) in enumerate(zip(jobs, alone, mixed)):
            assert _bits_equal(m, a), "%s differs between serving (tables built in the kernel) and alone" % name
            nrows = obs.n_time * obs.n_bl
            rows = np.sort(np.random.default_rng(700 + i).choice(nrows, min(8, nrows), replace=False))
            got = m.reshape(nrows, obs.n_chan)[torch.as_tensor(rows, device="cuda")].cpu().numpy()
            ref = oracle.predict(obs, sky, rows=rows)
            if kind == "subtract":
                g = torch.Generator(device="cuda").manual_seed(seed)
                d0 = torch.randn((obs.n_time, obs.n_bl, obs.n_chan), dtype=torch.complex64, device="cuda",
                                 generator=g).reshape(nrows, obs.n_chan)
                ref = d0[torch.as_tensor(rows, device="cuda")].cpu().numpy().astype(np.complex128) - ref
                del d0
            err = oracle.error_metric(got.astype(np.complex128), ref, obs, sky)
            _log("  %s: serving == alone bitwise; sampled error / total flux = %.3e" % (name, err))
            assert err <= 1e-6, (name, err)
        pairs = _overlapping_pairs([res[t] for t in tickets])
        _log("  %d pairs of jobs had tiles on the device at the same time" % pairs)
        assert pairs > 0
        for oh, sh in handles:
            vp.vp_destroy_sky(sh)
            vp.vp_destroy_obs(oh)
    finally:
        vp.vp_destroy_ctx(ctx)


def test_budget_admission_fifo():
    import torch
    obs, sky = synth.make_config(1, seed=77, n_tiles=40, n_time=2, n_chan=16, n_point=400, n_gauss=20,
                                 shapelet_nmax=[30])
    probe = vp.vp_create_ctx(0, 0)
    oh0, sh0 = vp.vp_create_obs(probe, obs), vp.vp_create_sky(probe, sky)
    fp = vp.vp_job_footprint(probe, vp.VP_JOB_PREDICT, sh0, oh0, vp.VP_PREC_MIXED, vp.VP_C64)
    vp.vp_destroy_ctx(probe)
    # room for one job at a time
    ctx = vp.vp_create_ctx(0, int(fp * 1.5))
    try:
        oh, sh = vp.vp_create_obs(ctx, obs), vp.vp_create_sky(ctx, sky)
        bufs = [vis_tensor(obs, vp.VP_C64) for _ in range(5)]
        torch.cuda.synchronize()
        tickets = [vp.vp_submit(ctx, vp.VP_JOB_PREDICT, sh, oh, vp.VP_PREC_MIXED, vp.VP_C64, b.data_ptr())
                   for b in bufs]
        with pytest.raises(vp.VPError) as e:
            vp.vp_destroy_obs(oh)
        assert e.value.code == vp.VP_EBUSY
        res = _wait(ctx, tickets)
        order = [res[t] for t in tickets]
        for prev, cur in zip(order, order[1:]):
            assert cur["t_admit"] >= prev["t_admit"]          # FIFO
            assert cur["t_admit"] >= prev["t_done"]           # the budget holds one job
        first = bufs[0].cpu().numpy()
        for b in bufs[1:]:
            assert np.array_equal(b.cpu().numpy(), first)
        # a job larger than the whole budget is refused outright
        big, _ = synth.make_config(1, seed=78, n_tiles=80, n_time=3, n_chan=64, n_point=1, n_gauss=0,
                                   shapelet_nmax=[])
        ohb = vp.vp_create_obs(ctx, big)
        with pytest.raises(vp.VPError) as e:
            vp.vp_submit(ctx, vp.VP_JOB_PREDICT, sh, ohb, vp.VP_PREC_MIXED, vp.VP_C128, bufs[0].data_ptr())
        assert e.value.code == vp.VP_ECAPACITY
        vp.vp_destroy_obs(ohb)
    finally:
        vp.vp_destroy_ctx(ctx)


def test_error_paths(ctx):
    import torch
    obs, sky = synth.make_config(0, n_tiles=8)
    oh, sh = vp.vp_create_obs(ctx, obs), vp.vp_create_sky(ctx, sky)
    b = vis_tensor(obs, vp.VP_C64)
    with pytest.raises(vp.VPError) as e:
        vp.vp_submit(ctx, vp.VP_JOB_PREDICT, sh, oh, vp.VP_PREC_FP64, vp.VP_C64, b.data_ptr())
    assert e.value.code == vp.VP_EINVAL
    with pytest.raises(vp.VPError) as e:
        vp.vp_submit(ctx, 7, sh, oh, vp.VP_PREC_MIXED, vp.VP_C64, b.data_ptr())
    assert e.value.code == vp.VP_EINVAL
    with pytest.raises(vp.VPError) as e:
        vp.vp_poll(ctx, 987654321)
    assert e.value.code == vp.VP_ENOTFOUND
    t = vp.vp_submit(ctx, vp.VP_JOB_PREDICT, sh, oh, vp.VP_PREC_MIXED, vp.VP_C64, b.data_ptr())
    r = _wait(ctx, [t])[t]
    assert r["status"] == vp.VP_OK
    with pytest.raises(vp.VPError) as e:   # a collected ticket is released
        vp.vp_poll(ctx, t)
    assert e.value.code == vp.VP_ENOTFOUND
    vp.vp_destroy_sky(sh)
    vp.vp_destroy_obs(oh)


def test_destroy_busy_context():
    """A context with pending jobs refuses to go (VP_EBUSY) and goes once they
    are collected.  16 jobs of ~1 ms of device work each are pending when
    destroy is attempted microseconds after the last submission."""
    import torch
    obs, sky = synth.make_config(1, seed=79, n_tiles=64, n_time=4, n_chan=32, n_point=3000, n_gauss=100,
                                 shapelet_nmax=[40])
    ctx = vp.vp_create_ctx(0, 0)
    oh, sh = vp.vp_create_obs(ctx, obs), vp.vp_create_sky(ctx, sky)
    bufs = [vis_tensor(obs, vp.VP_C64) for _ in range(16)]
    torch.cuda.synchronize()
    tickets = [vp.vp_submit(ctx, vp.VP_JOB_PREDICT, sh, oh, vp.VP_PREC_MIXED, vp.VP_C64, b.data_ptr())
               for b in bufs]
    with pytest.raises(vp.VPError) as e:
        vp.vp_destroy_ctx(ctx)
    assert e.value.code == vp.VP_EBUSY
    with pytest.raises(vp.VPError) as e:
        vp.vp_destroy_sky(sh)
    assert e.value.code == vp.VP_EBUSY
    res = _wait(ctx, tickets)
    assert all(r["status"] == vp.VP_OK for r in res.values())
    vp.vp_destroy_sky(sh)
    vp.vp_destroy_obs(oh)
    vp.vp_destroy_ctx(ctx)
