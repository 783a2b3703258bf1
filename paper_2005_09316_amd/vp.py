"""ctypes binding of libvp (include/vp.h).

Argument marshalling only: every step of the computation runs in libvp's HIP
kernels.  PyTorch supplies device memory (tensor.data_ptr()) and streams
(torch.cuda.Stream.cuda_stream); nothing here falls back to the CPU.  Loading
fails loudly if libvp.so has not been built.

The functions mirror the C entry points one to one (same names, same
argument order, handles as opaque integers); each raises VPError with the
library's message when the C call returns a non-zero code (except vp_poll,
which returns None while a job is pending).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvp.so")

VP_OK, VP_EINVAL, VP_ENOMEM, VP_EDEVICE, VP_EAGAIN, VP_ECAPACITY, VP_ENOTFOUND, VP_EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
VP_PREC_FP64, VP_PREC_MIXED, VP_PREC_MIXED_BF16, VP_PREC_FP32, VP_PREC_MIXED_BF16X2 = 0, 1, 2, 3, 4
VP_PREC_MIXED_F32MMA = 5  # retired: refused with VP_EINVAL
VP_PREC_LUT = 6
VP_C128, VP_C64 = 0, 1
VP_JOB_PREDICT, VP_JOB_SUBTRACT = 0, 1
VP_NMAX_LIMIT = 96
VP_NTERM_LIMIT = 8
VP_PEEL_MAX_ANT, VP_PEEL_MAX_ITER, VP_PEEL_MAX_CG = 256, 1000, 200

PRECISIONS = {"fp64": VP_PREC_FP64, "mixed": VP_PREC_MIXED, "mixed_bf16": VP_PREC_MIXED_BF16,
              "fp32": VP_PREC_FP32, "mixed_bf16x2": VP_PREC_MIXED_BF16X2, "lut": VP_PREC_LUT}

# every symbol declared in include/vp.h
EXPORTS = ["vp_create_ctx", "vp_destroy_ctx", "vp_create_obs", "vp_destroy_obs", "vp_create_sky",
           "vp_destroy_sky", "vp_predict", "vp_predict_noalloc", "vp_subtract", "vp_peel", "vp_submit", "vp_poll", "vp_serve_stats", "vp_job_footprint",
           "vp_profile", "vp_profile_read", "vp_last_error", "vp_version"]

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


class VPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libvp error %d: %s" % (code, msg))
        self.code = code


class vp_obs_desc(ctypes.Structure):
    _fields_ = [("n_time", ctypes.c_int32), ("n_bl", ctypes.c_int32), ("n_chan", ctypes.c_int32),
                ("uvw_m", _dp), ("freq_hz", _dp), ("ra0", ctypes.c_double), ("dec0", ctypes.c_double),
                ("sign", ctypes.c_int32), ("beam_fwhm_rad", ctypes.c_double), ("beam_nu_ref_hz", ctypes.c_double)]


class vp_sky_desc(ctypes.Structure):
    _fields_ = [("nu_ref_hz", ctypes.c_double),
                ("n_point", ctypes.c_int32), ("p_ra", _dp), ("p_dec", _dp), ("p_sref", _dp), ("p_alpha", _dp),
                ("n_gauss", ctypes.c_int32), ("g_ra", _dp), ("g_dec", _dp), ("g_sref", _dp), ("g_alpha", _dp),
                ("g_maj", _dp), ("g_min", _dp), ("g_pa", _dp),
                ("n_shp", ctypes.c_int32), ("s_ra", _dp), ("s_dec", _dp), ("s_sref", _dp), ("s_alpha", _dp),
                ("s_beta1", _dp), ("s_beta2", _dp), ("s_pa", _dp),
                ("s_nmax", _i32p), ("s_coeff_off", _i64p), ("coeffs", _dp), ("s_nterm", _i32p)]


class vp_job(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("sky", ctypes.c_void_p), ("obs", ctypes.c_void_p),
                ("precision", ctypes.c_int32), ("dtype", ctypes.c_int32), ("vis_dev", ctypes.c_void_p),
                ("t_arrival_ns", ctypes.c_uint64)]


class vp_job_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("t_submit", ctypes.c_uint64), ("t_admit", ctypes.c_uint64),
                ("t_start", ctypes.c_uint64), ("t_done", ctypes.c_uint64),
                ("dev_first_tile", ctypes.c_uint64), ("dev_last_tile", ctypes.c_uint64)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libvp.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libvp.so not found at %s: build it with paper_2005_09316_amd/build.py" % path)
    # PyTorch ships its own HIP runtime with the same soname as the system one;
    # importing it first makes libvp bind to that copy, so that one HIP runtime
    # serves both (two runtimes in one process cannot share the device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    sig = {
        "vp_create_ctx": ([ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(vp)], ctypes.c_int),
        "vp_destroy_ctx": ([vp], ctypes.c_int),
        "vp_create_obs": ([vp, ctypes.POINTER(vp_obs_desc), ctypes.POINTER(vp)], ctypes.c_int),
        "vp_destroy_obs": ([vp], ctypes.c_int),
        "vp_create_sky": ([vp, ctypes.POINTER(vp_sky_desc), ctypes.POINTER(vp)], ctypes.c_int),
        "vp_destroy_sky": ([vp], ctypes.c_int),
        "vp_predict": ([vp, vp, vp, ctypes.c_int, ctypes.c_int, vp, vp], ctypes.c_int),
        "vp_predict_noalloc": ([vp, vp, vp, ctypes.c_int, ctypes.c_int, vp, vp], ctypes.c_int),
        "vp_subtract": ([vp, vp, vp, ctypes.c_int, ctypes.c_int, vp, vp], ctypes.c_int),
        "vp_peel": ([vp, vp, vp, _i32p, _i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.c_int, vp, vp,
                     vp], ctypes.c_int),
        "vp_submit": ([vp, ctypes.POINTER(vp_job), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "vp_poll": ([vp, ctypes.c_uint64, ctypes.POINTER(vp_job_result)], ctypes.c_int),
        "vp_job_footprint": ([vp, ctypes.POINTER(vp_job), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "vp_serve_stats": ([vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "vp_profile": ([vp, ctypes.c_int], ctypes.c_int),
        "vp_profile_read": ([vp, _i64p, _dp], ctypes.c_int),
        "vp_last_error": ([], ctypes.c_char_p),
        "vp_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != VP_OK:
        raise VPError(rc, vp_last_error())


def vp_last_error() -> str:
    return load().vp_last_error().decode()


def vp_version() -> str:
    return load().vp_version().decode()


def vp_create_ctx(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    out = ctypes.c_void_p()
    _check(load().vp_create_ctx(int(device), int(hbm_budget_bytes), ctypes.byref(out)))
    return out.value


def vp_destroy_ctx(ctx: int):
    _check(load().vp_destroy_ctx(ctx))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a, t=_dp):
    return a.ctypes.data_as(t) if a is not None and a.size else ctypes.cast(None, t)


def vp_create_obs(ctx: int, obs) -> int:
    """``obs`` carries n_time, n_bl, n_chan, uvw_m [T,B,3] (m), freq_hz [K],
    ra0, dec0, sign, beam_fwhm_rad, beam_nu_ref_hz."""
    uvw, fr = _f64(obs.uvw_m), _f64(obs.freq_hz)
    d = vp_obs_desc(int(obs.n_time), int(obs.n_bl), int(obs.n_chan), _p(uvw), _p(fr), float(obs.ra0),
                    float(obs.dec0), int(obs.sign), float(obs.beam_fwhm_rad), float(obs.beam_nu_ref_hz))
    out = ctypes.c_void_p()
    _check(load().vp_create_obs(ctx, ctypes.byref(d), ctypes.byref(out)))
    return out.value


def vp_destroy_obs(obs: int):
    _check(load().vp_destroy_obs(obs))


def vp_create_sky(ctx: int, sky) -> int:
    """``sky`` carries the component arrays named as in vp_sky_desc."""
    keep = []

    def f(name):
        a = _f64(getattr(sky, name))
        keep.append(a)
        return _p(a)

    nmax = np.ascontiguousarray(np.asarray(sky.s_nmax, np.int32))
    off = np.ascontiguousarray(np.asarray(sky.s_coeff_off, np.int64))
    d = vp_sky_desc(float(sky.nu_ref_hz),
                    int(np.size(sky.p_ra)), f("p_ra"), f("p_dec"), f("p_sref"), f("p_alpha"),
                    int(np.size(sky.g_ra)), f("g_ra"), f("g_dec"), f("g_sref"), f("g_alpha"),
                    f("g_maj"), f("g_min"), f("g_pa"),
                    int(np.size(sky.s_ra)), f("s_ra"), f("s_dec"), f("s_sref"), f("s_alpha"),
                    f("s_beta1"), f("s_beta2"), f("s_pa"),
                    _p(nmax, _i32p), _p(off, _i64p), f("coeffs"), None)
    nterm = getattr(sky, "s_nterm", None)
    if nterm is not None:
        nt = np.ascontiguousarray(np.asarray(nterm, np.int32))
        keep.append(nt)
        d.s_nterm = _p(nt, _i32p)
    out = ctypes.c_void_p()
    _check(load().vp_create_sky(ctx, ctypes.byref(d), ctypes.byref(out)))
    return out.value


def vp_destroy_sky(sky: int):
    _check(load().vp_destroy_sky(sky))


def vp_predict(ctx: int, sky: int, obs: int, precision: int, dtype: int, vis_dev: int, hip_stream: int = 0):
    _check(load().vp_predict(ctx, sky, obs, int(precision), int(dtype), vis_dev, hip_stream or None))


def vp_predict_noalloc(ctx: int, sky: int, obs: int, precision: int, dtype: int, vis_dev: int, hip_stream: int = 0):
    _check(load().vp_predict_noalloc(ctx, sky, obs, int(precision), int(dtype), vis_dev, hip_stream or None))


def vp_subtract(ctx: int, sky: int, obs: int, precision: int, dtype: int, data_dev: int, hip_stream: int = 0):
    _check(load().vp_subtract(ctx, sky, obs, int(precision), int(dtype), data_dev, hip_stream or None))


def vp_peel(ctx: int, sky: int, obs: int, ant1, ant2, n_ant: int, n_iter: int, precision: int, dtype: int,
            data_dev: int, gains_dev: int = 0, hip_stream: int = 0):
    """Calibrated peel of `sky` from the data (Sec. 5.1); ant1/ant2: int32 [n_bl] tile of each baseline."""
    a1 = np.ascontiguousarray(ant1, dtype=np.int32)
    a2 = np.ascontiguousarray(ant2, dtype=np.int32)
    if a1.shape != a2.shape or a1.ndim != 1:
        raise ValueError("ant1 and ant2 must be 1-D arrays of one length")
    _check(load().vp_peel(ctx, sky, obs, _p(a1, _i32p), _p(a2, _i32p), int(n_ant), int(n_iter), int(precision),
                          int(dtype), data_dev, gains_dev or None, hip_stream or None))


def vp_submit(ctx: int, kind: int, sky: int, obs: int, precision: int, dtype: int, vis_dev: int,
              t_arrival_ns: int = 0) -> int:
    j = vp_job(int(kind), sky, obs, int(precision), int(dtype), vis_dev, int(t_arrival_ns))
    t = ctypes.c_uint64()
    _check(load().vp_submit(ctx, ctypes.byref(j), ctypes.byref(t)))
    return t.value


def vp_serve_stats(ctx: int):
    """(launches, resident_ms) of the persistent serving kernel."""
    n, ms = ctypes.c_uint64(), ctypes.c_double()
    _check(load().vp_serve_stats(ctx, ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def vp_poll(ctx: int, ticket: int) -> Optional[dict]:
    """dict(status, t_submit, t_admit, t_start, t_done, dev_first_tile, dev_last_tile) when done, None if
    pending."""
    r = vp_job_result()
    rc = load().vp_poll(ctx, int(ticket), ctypes.byref(r))
    if rc == VP_EAGAIN:
        return None
    _check(rc)
    return {"status": r.status, "t_submit": r.t_submit, "t_admit": r.t_admit, "t_start": r.t_start,
            "t_done": r.t_done, "dev_first_tile": r.dev_first_tile, "dev_last_tile": r.dev_last_tile}


def vp_job_footprint(ctx: int, kind: int, sky: int, obs: int, precision: int, dtype: int, vis_dev: int = 0) -> int:
    j = vp_job(int(kind), sky, obs, int(precision), int(dtype), vis_dev, 0)
    b = ctypes.c_uint64()
    _check(load().vp_job_footprint(ctx, ctypes.byref(j), ctypes.byref(b)))
    return b.value


def vp_profile(ctx: int, enable: bool):
    _check(load().vp_profile(ctx, 1 if enable else 0))


def vp_profile_read(ctx: int):
    """(counts[4], total_ms[4]) for kernel classes 0 = tables, 1 = point/Gaussian, 2 = shapelet,
    3 = peel calibration."""
    c = np.zeros(4, np.int64)
    t = np.zeros(4, np.float64)
    _check(load().vp_profile_read(ctx, _p(c, _i64p), _p(t)))
    return c, t
