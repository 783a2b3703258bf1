"""Shared helpers for the GPU tests: run libvp on synthetic inputs and bring
the result back as numpy complex128."""
import numpy as np

from paper_2005_09316_amd import vp


def torch_cuda():
    import torch
    return torch


def vis_tensor(obs, dtype, data=None):
    torch = torch_cuda()
    tdt = torch.complex64 if dtype == vp.VP_C64 else torch.complex128
    shape = (int(obs.n_time), int(obs.n_bl), int(obs.n_chan))
    if data is None:
        return torch.full(shape, complex(float("nan"), float("nan")), dtype=tdt, device="cuda")
    return torch.from_numpy(np.ascontiguousarray(np.asarray(data).reshape(shape))).to(tdt).to("cuda")


def run(ctx, obs_h, sky_h, obs, precision, dtype, data=None, stream=None):
    """predict (data is None) or subtract (data given); returns complex128 numpy [T,B,K]."""
    torch = torch_cuda()
    t = vis_tensor(obs, dtype, data)
    s = stream if stream is not None else torch.cuda.current_stream()
    if data is None:
        vp.vp_predict(ctx, sky_h, obs_h, precision, dtype, t.data_ptr(), s.cuda_stream)
    else:
        vp.vp_subtract(ctx, sky_h, obs_h, precision, dtype, t.data_ptr(), s.cuda_stream)
    s.synchronize()
    return t.cpu().numpy().astype(np.complex128)


class Handles:
    """obs + sky handles on a context, destroyed together."""

    def __init__(self, ctx, obs, sky):
        self.ctx = ctx
        self.obs = vp.vp_create_obs(ctx, obs)
        self.sky = vp.vp_create_sky(ctx, sky)

    def close(self):
        vp.vp_destroy_sky(self.sky)
        vp.vp_destroy_obs(self.obs)

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
