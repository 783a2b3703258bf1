"""FP64 CPU oracle for direct-Fourier visibility prediction (TEST INFRASTRUCTURE).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.  The arithmetic lives in ``vp_oracle.c`` (plain C,
double precision, Neumaier sums, libm); this wrapper only marshals arrays.

Functions and the paper passages they follow:

* :func:`predict` -- Sec. 3.1 Eq. (measure_eq_discrete) with the envelopes of
  Sec. 3.2 Eqs. (env_visi_def), (gauss-env), (shape-env): every visibility as
  an explicit sum over components, points first, then Gaussians, then
  shapelets.
* :func:`subtract` -- the peel residual R = V - M of Sec. 5.1 with unit gains.
* :func:`hermite` -- orthonormal Hermite functions, Sec. 2 Eq. (basis_1D).
* :func:`shapelet_envelope_ab`, :func:`gauss_envelope`, :func:`lmn`,
  :func:`rotation`, :func:`flux_table` -- the pieces above, exposed so that
  tests can pin each against closed forms.
* :func:`error_metric` -- max over channels of max |V - V_ref| / F_k with
  F_k = sum_j |S_j(nu_k)| |xi_j(0)|, the total flux per channel.
* :func:`calibrate_cell`, :func:`peel` -- the calibration and subtraction of
  Sec. 5.1: model M_ij = g_i g_j^* I_ij, residual R = V - M, the linearised
  least-squares step for the real and imaginary parts of the gain errors
  (Eq. peeling-iter) with an explicit design matrix, iterated from unit
  gains; the step is the minimum-norm least-squares solution (the global
  phase of the gains is not determined by the data).  Plain numpy.

Every function here is pinned by a test in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "vp_oracle.c")

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


class _Obs(ctypes.Structure):
    _fields_ = [
        ("n_time", ctypes.c_int32), ("n_bl", ctypes.c_int32), ("n_chan", ctypes.c_int32),
        ("uvw_m", _dp), ("freq_hz", _dp),
        ("ra0", ctypes.c_double), ("dec0", ctypes.c_double),
        ("sign", ctypes.c_int32),
        ("beam_fwhm_rad", ctypes.c_double), ("beam_nu_ref_hz", ctypes.c_double),
    ]


class _Sky(ctypes.Structure):
    _fields_ = [
        ("nu_ref_hz", ctypes.c_double),
        ("n_point", ctypes.c_int32), ("p_ra", _dp), ("p_dec", _dp), ("p_sref", _dp), ("p_alpha", _dp),
        ("n_gauss", ctypes.c_int32), ("g_ra", _dp), ("g_dec", _dp), ("g_sref", _dp), ("g_alpha", _dp),
        ("g_maj", _dp), ("g_min", _dp), ("g_pa", _dp),
        ("n_shp", ctypes.c_int32), ("s_ra", _dp), ("s_dec", _dp), ("s_sref", _dp), ("s_alpha", _dp),
        ("s_beta1", _dp), ("s_beta2", _dp), ("s_pa", _dp),
        ("s_nmax", _i32p), ("s_coeff_off", _i64p), ("coeffs", _dp),
        ("s_nterm", _i32p),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, OpenMP over rows)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-fopenmp", "-shared", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_hermite.argtypes = [ctypes.c_int32, ctypes.c_double, _dp]
        lib.oracle_hermite.restype = None
        lib.oracle_lmn.argtypes = [ctypes.c_double] * 4 + [_dp]
        lib.oracle_lmn.restype = None
        lib.oracle_rotation.argtypes = [ctypes.c_double] * 4 + [_dp]
        lib.oracle_rotation.restype = None
        lib.oracle_gauss_envelope.argtypes = [ctypes.c_double] * 5
        lib.oracle_gauss_envelope.restype = ctypes.c_double
        lib.oracle_shapelet_envelope_ab.argtypes = [ctypes.c_int32, _dp, ctypes.c_double, ctypes.c_double,
                                                    ctypes.c_int32, _dp, _dp]
        lib.oracle_shapelet_envelope_ab.restype = ctypes.c_int
        lib.oracle_shapelet_args.argtypes = [ctypes.c_double] * 5 + [_dp, _dp]
        lib.oracle_shapelet_args.restype = None
        lib.oracle_predict.argtypes = [ctypes.POINTER(_Obs), ctypes.POINTER(_Sky), _i64p, ctypes.c_int64,
                                       _dp, ctypes.c_int32]
        lib.oracle_predict.restype = ctypes.c_int
        lib.oracle_flux_table.argtypes = [ctypes.POINTER(_Obs), ctypes.POINTER(_Sky), _dp]
        lib.oracle_flux_table.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int32
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


def _marshal(obs, sky, sign: Optional[int] = None):
    keep = []

    def f(a):
        a = _f64(a)
        keep.append(a)
        return _ptr(a)

    o = _Obs(int(obs.n_time), int(obs.n_bl), int(obs.n_chan), f(obs.uvw_m), f(obs.freq_hz),
             float(obs.ra0), float(obs.dec0), int(obs.sign if sign is None else sign),
             float(obs.beam_fwhm_rad), float(obs.beam_nu_ref_hz))
    nmax = np.ascontiguousarray(np.asarray(sky.s_nmax, np.int32))
    off = np.ascontiguousarray(np.asarray(sky.s_coeff_off, np.int64))
    keep += [nmax, off]
    s = _Sky(float(sky.nu_ref_hz),
             int(np.size(sky.p_ra)), f(sky.p_ra), f(sky.p_dec), f(sky.p_sref), f(sky.p_alpha),
             int(np.size(sky.g_ra)), f(sky.g_ra), f(sky.g_dec), f(sky.g_sref), f(sky.g_alpha),
             f(sky.g_maj), f(sky.g_min), f(sky.g_pa),
             int(np.size(sky.s_ra)), f(sky.s_ra), f(sky.s_dec), f(sky.s_sref), f(sky.s_alpha),
             f(sky.s_beta1), f(sky.s_beta2), f(sky.s_pa),
             _ptr(nmax, _i32p), _ptr(off, _i64p), f(sky.coeffs), None)
    nterm = getattr(sky, "s_nterm", None)
    if nterm is not None:
        nt = np.ascontiguousarray(np.asarray(nterm, np.int32))
        keep.append(nt)
        s.s_nterm = _ptr(nt, _i32p)
    return o, s, keep


def predict(obs, sky, sign: Optional[int] = None, rows=None, nthreads: int = 0) -> np.ndarray:
    """Visibilities, complex128.  Full output has shape [T, B, K]; with
    ``rows`` (flat (time*B + baseline) indices) the shape is [len(rows), K]."""
    lib = _load()
    o, s, keep = _marshal(obs, sky, sign)
    K = int(obs.n_chan)
    if rows is None:
        nrows = int(obs.n_time) * int(obs.n_bl)
        rp = None
    else:
        r = np.ascontiguousarray(np.asarray(rows, np.int64))
        keep.append(r)
        nrows = r.size
        rp = _ptr(r, _i64p)
    out = np.zeros((nrows, K, 2), np.float64)
    if nrows:
        rc = lib.oracle_predict(ctypes.byref(o), ctypes.byref(s), rp, nrows, _ptr(out), int(nthreads))
        if rc != 0:
            raise ValueError("oracle_predict rejected its inputs (code %d)" % rc)
    v = out[..., 0] + 1j * out[..., 1]
    if rows is None:
        v = v.reshape(int(obs.n_time), int(obs.n_bl), K)
    return v


def subtract(data: np.ndarray, obs, sky, sign: Optional[int] = None, rows=None, nthreads: int = 0):
    """Peel residual R = D - V (unit gains)."""
    return np.asarray(data, np.complex128) - predict(obs, sky, sign, rows, nthreads)


def hermite(nmax: int, x: float) -> np.ndarray:
    lib = _load()
    out = np.zeros(nmax + 1)
    lib.oracle_hermite(int(nmax), float(x), _ptr(out))
    return out


def lmn(ra0, dec0, ra, dec) -> np.ndarray:
    """(l, m, n - 1)."""
    out = np.zeros(3)
    _load().oracle_lmn(float(ra0), float(dec0), float(ra), float(dec), _ptr(out))
    return out


def rotation(ra0, dec0, ra, dec) -> np.ndarray:
    out = np.zeros(9)
    _load().oracle_rotation(float(ra0), float(dec0), float(ra), float(dec), _ptr(out))
    return out.reshape(3, 3)


def gauss_envelope(u, v, maj, mn, pa) -> float:
    return float(_load().oracle_gauss_envelope(float(u), float(v), float(maj), float(mn), float(pa)))


def shapelet_args(up, vp, beta1, beta2, pa):
    a, b = ctypes.c_double(), ctypes.c_double()
    _load().oracle_shapelet_args(float(up), float(vp), float(beta1), float(beta2), float(pa),
                                 ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def shapelet_envelope_ab(nmax: int, coeffs, a: float, b: float, sign: int = -1) -> complex:
    c = _f64(coeffs)
    if c.size != (nmax + 2) * (nmax + 1) // 2:
        raise ValueError("coefficient count does not match nmax")
    re, im = ctypes.c_double(), ctypes.c_double()
    rc = _load().oracle_shapelet_envelope_ab(int(nmax), _ptr(c), float(a), float(b), int(sign),
                                             ctypes.byref(re), ctypes.byref(im))
    if rc:
        raise ValueError("nmax out of range")
    return complex(re.value, im.value)


def flux_table(obs, sky) -> np.ndarray:
    """S_j(nu_k) for every component (points, Gaussians, shapelets) x channel."""
    lib = _load()
    o, s, keep = _marshal(obs, sky)
    J = int(np.size(sky.p_ra) + np.size(sky.g_ra) + np.size(sky.s_ra))
    out = np.zeros((max(J, 1), int(obs.n_chan)))
    if J:
        rc = lib.oracle_flux_table(ctypes.byref(o), ctypes.byref(s), _ptr(out))
        if rc:
            raise ValueError("oracle_flux_table rejected its inputs")
    return out[:J]


def xi_origin(sky, nu_hz=None) -> np.ndarray:
    """|xi_j(0)| per component: 1 for points and Gaussians, the shapelet
    envelope at the uv origin otherwise (with spectral terms, of the
    coefficients at frequency nu_hz, default the reference frequency)."""
    vals = [1.0] * int(np.size(sky.p_ra) + np.size(sky.g_ra))
    nterm = getattr(sky, "s_nterm", None)
    x = 0.0 if nu_hz is None else math.log(nu_hz / sky.nu_ref_hz)
    for s in range(int(np.size(sky.s_ra))):
        n = int(sky.s_nmax[s])
        o = int(sky.s_coeff_off[s])
        cnt = (n + 2) * (n + 1) // 2
        q_n = 1 if nterm is None else int(nterm[s])
        c = sum(np.asarray(sky.coeffs[o + q * cnt:o + (q + 1) * cnt]) * x ** q for q in range(q_n))
        vals.append(abs(shapelet_envelope_ab(n, c, 0.0, 0.0)))
    return np.asarray(vals, np.float64)


def total_flux(obs, sky) -> np.ndarray:
    """F_k = sum_j |S_j(nu_k)| |xi_j(0)|, shape [K] (xi_j(0) at nu_k when a
    shapelet has spectral terms)."""
    ft = flux_table(obs, sky)
    if ft.shape[0] == 0:
        return np.zeros(int(obs.n_chan))
    if getattr(sky, "s_nterm", None) is None:
        return np.abs(ft).T @ xi_origin(sky)
    return np.array([np.abs(ft[:, k]) @ xi_origin(sky, float(obs.freq_hz[k])) for k in range(int(obs.n_chan))])


def error_metric(v, v_ref, obs, sky) -> float:
    """max_k max_rows |v - v_ref| / F_k; arrays shaped [..., K]."""
    F = total_flux(obs, sky)
    d = np.abs(np.asarray(v, np.complex128) - np.asarray(v_ref, np.complex128))
    d = d.reshape(-1, int(obs.n_chan)).max(axis=0) if d.size else np.zeros(int(obs.n_chan))
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(F > 0, d / np.where(F > 0, F, 1.0), np.where(d > 0, np.inf, 0.0))
    return float(r.max()) if r.size else 0.0


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def calibrate_cell(v, model, ant1, ant2, n_ant: int, n_iter: int = 10, g0=None) -> np.ndarray:
    """Per-tile complex gains for one (time, frequency) cell (Sec. 5.1).

    v, model: [n_bl] complex visibilities of the data and of the ideal model
    I_ij; ant1, ant2: the tiles of each baseline.  Each iteration linearises
    V_ij = (g_i + e_i)(g_j + e_j)^* I_ij around the current g: the residual
    R_ij = V_ij - g_i g_j^* I_ij is matched by e_i g_j^* I_ij + e_j^* g_i I_ij,
    whose real and imaginary parts are linear in Re e and Im e (the rows of
    the design matrix A below), and x = (A^T A)^+ A^T b is taken as the
    minimum-norm least-squares solution.  Then g <- g + e."""
    v = np.asarray(v, np.complex128)
    m = np.asarray(model, np.complex128)
    a1 = np.asarray(ant1, np.int64)
    a2 = np.asarray(ant2, np.int64)
    nb = v.size
    g = np.ones(n_ant, np.complex128) if g0 is None else np.array(g0, np.complex128)
    rows = np.arange(nb)
    for _ in range(n_iter):
        w = np.conj(g[a2]) * m   # coefficient of e_i
        z = g[a1] * m            # coefficient of e_j^*
        r = v - g[a1] * np.conj(g[a2]) * m
        A = np.zeros((2 * nb, 2 * n_ant))
        # Re R = Re(e_i w) + Re(e_j^* z);  Im R = Im(e_i w) + Im(e_j^* z)
        np.add.at(A, (rows, a1), w.real)
        np.add.at(A, (rows, n_ant + a1), -w.imag)
        np.add.at(A, (rows, a2), z.real)
        np.add.at(A, (rows, n_ant + a2), z.imag)
        np.add.at(A, (nb + rows, a1), w.imag)
        np.add.at(A, (nb + rows, n_ant + a1), w.real)
        np.add.at(A, (nb + rows, a2), z.imag)
        np.add.at(A, (nb + rows, n_ant + a2), -z.real)
        b = np.concatenate([r.real, r.imag])
        x = np.linalg.lstsq(A, b, rcond=None)[0]
        g = g + x[:n_ant] + 1j * x[n_ant:]
    return g


def peel(data, model, ant1, ant2, n_ant: int, n_iter: int = 10):
    """Calibrate every (time, channel) cell of data [T, B, K] against model
    [T, B, K] and subtract the gain-corrupted model.  Returns (gains [T, K,
    n_ant], residual [T, B, K])."""
    data = np.asarray(data, np.complex128)
    model = np.asarray(model, np.complex128)
    T, B, K = data.shape
    gains = np.empty((T, K, n_ant), np.complex128)
    res = np.empty_like(data)
    a1 = np.asarray(ant1, np.int64)
    a2 = np.asarray(ant2, np.int64)
    for t in range(T):
        for k in range(K):
            g = calibrate_cell(data[t, :, k], model[t, :, k], a1, a2, n_ant, n_iter)
            gains[t, k] = g
            res[t, :, k] = data[t, :, k] - g[a1] * np.conj(g[a2]) * model[t, :, k]
    return gains, res

