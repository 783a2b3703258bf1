"""vp_predict_noalloc (the entry point for callers that cannot allocate device
memory) against vp_predict through the C ABI: the same kernels read the
per-(sky, observation) tables from the library's fixed scratch array instead
of a cached allocation, so the outputs must be bitwise equal; both are also
checked against the FP64 oracle at the path's bar.  Two calls in a row, the
second with a smaller workload, show that the scratch keeps no state that a
later call depends on."""
import sys

import numpy as np
import pytest

import oracle
import synth
from paper_2005_09316_amd import vp
from tests.helpers import Handles, vis_tensor

pytestmark = pytest.mark.gpu

TOL = {vp.VP_PREC_FP64: 1e-11, vp.VP_PREC_MIXED: 1e-6}


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = vp.vp_create_ctx(0, 0)
    yield c
    vp.vp_destroy_ctx(c)


def _predict(fn, ctx, h, obs, prec, dtype):
    import torch
    t = vis_tensor(obs, dtype)
    s = torch.cuda.current_stream()
    fn(ctx, h.sky, h.obs, prec, dtype, t.data_ptr(), s.cuda_stream)
    s.synchronize()
    return t.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("prec,dtype", [(vp.VP_PREC_MIXED, vp.VP_C64), (vp.VP_PREC_FP64, vp.VP_C128)])
def test_noalloc_matches_predict_twice(ctx, prec, dtype):
    # first a mid-size workload with points, Gaussians, two shapelets and the
    # beam (several row tiles, ragged channel blocks), then a smaller one
    cases = [synth.make_config(1, n_tiles=24, n_time=3, n_chan=13, n_point=300, n_gauss=60, shapelet_nmax=[54, 33]),
             synth.make_config(0)]
    for i, (obs, sky) in enumerate(cases):
        _log("call %d: precision %d dtype %d, %d visibilities, %d components" %
             (i, prec, dtype, obs.n_vis, sky.n_point + sky.n_gauss + sky.n_shp))
        ref = oracle.predict(obs, sky)
        with Handles(ctx, obs, sky) as h:
            got = _predict(vp.vp_predict_noalloc, ctx, h, obs, prec, dtype)
            base = _predict(vp.vp_predict, ctx, h, obs, prec, dtype)
        err = oracle.error_metric(got, ref, obs, sky)
        _log("  no-alloc vs vp_predict: max |diff| = %.3e; error vs oracle / total flux = %.3e"
             % (np.abs(got - base).max(), err))
        assert np.array_equal(got, base)
        assert err <= TOL[prec]


def test_noalloc_refuses_beyond_scratch(ctx):
    # 2000 points x 4096 channels need 98 MB of flux tables: over the 64 MiB scratch
    obs, sky = synth.make_config(0, n_tiles=2, n_chan=4096)
    sky = synth.select_components(sky, points=list(range(100)) * 20, gauss=[], shapelets=[])
    import torch
    t = torch.empty((obs.n_time, obs.n_bl, obs.n_chan), dtype=torch.complex64, device="cuda")
    with Handles(ctx, obs, sky) as h:
        with pytest.raises(vp.VPError) as e:
            vp.vp_predict_noalloc(ctx, h.sky, h.obs, vp.VP_PREC_MIXED, vp.VP_C64, t.data_ptr(), 0)
        assert e.value.code == vp.VP_EINVAL
        assert "scratch" in vp.vp_last_error()
        with pytest.raises(vp.VPError) as e:
            vp.vp_predict_noalloc(ctx, h.sky, h.obs, vp.VP_PREC_LUT, vp.VP_C64, t.data_ptr(), 0)
        assert e.value.code == vp.VP_EINVAL
