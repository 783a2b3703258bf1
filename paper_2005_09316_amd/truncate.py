"""Sky-model truncation (Sec. 5.3, "Model truncation").

The paper ranks the components of a model by their absolute integrated flux
density |I_j| and keeps the largest while their cumulative sum stays within a
fraction f_comp of the total over all components.  For a point or Gaussian
component I_j is its flux density.  For a shapelet basis function (p1, p2)
the paper images the restoring-beam-convolved basis function and sums the
absolute pixel values; with no image here, the image-plane L1 norm of the
basis function itself is used.  A shapelet of flux density S whose uv
envelope is sum C i^(p1+p2) phi_p1(a) phi_p2(b) has the image-plane term
(p1, p2) with absolute integral |S C| L1(p1) L1(p2) / (2 pi), L1(n) being the
integral of |phi_n| over the real line (the basis scales cancel), so points,
Gaussians and basis functions share one scale: a shapelet that is a single
(0, 0) term normalised to unit envelope at the uv origin counts as S, like
a Gaussian of the same flux.

Truncation by order (keep n1 + n2 <= N') is provided beside it: on matrix
cores the shapelet work follows the highest order kept, not the number of
basis functions.  Dropped points and Gaussians are removed; dropped shapelet
coefficients are set to zero, and a shapelet left with none is removed.
This is host-side model preparation, not part of the prediction path.
"""
from __future__ import annotations

import dataclasses

import numpy as np


def hermite_l1(nmax: int, h: float = 2e-3) -> np.ndarray:
    """Integral of |phi_n(x)| for n = 0..nmax (orthonormal Hermite functions),
    trapezoid rule with step h over |x| <= sqrt(2 nmax + 1) + 12."""
    xm = np.sqrt(2.0 * nmax + 1.0) + 12.0
    x = np.arange(-xm, xm + 0.5 * h, h)
    prev = np.zeros_like(x)
    cur = np.pi ** -0.25 * np.exp(-0.5 * x * x)
    out = np.empty(nmax + 1)
    for n in range(nmax + 1):
        out[n] = np.trapezoid(np.abs(cur), x)
        prev, cur = cur, np.sqrt(2.0 / (n + 1)) * x * cur - np.sqrt(n / (n + 1.0)) * prev
    return out


def _orders(nmax: int):
    n1 = np.concatenate([np.full(nmax + 1 - a, a) for a in range(nmax + 1)])
    n2 = np.concatenate([np.arange(nmax + 1 - a) for a in range(nmax + 1)])
    return n1, n2


def _single_term(sky):
    nterm = getattr(sky, "s_nterm", None)
    if nterm is not None and np.any(np.asarray(nterm) != 1):
        raise ValueError("truncation of shapelets with spectral terms is not defined")


def component_flux(sky):
    """|I_j| of every point, Gaussian and shapelet basis function (at the
    reference frequency), and a matching list of (kind, component, packed
    coefficient index) with kind 0 = point, 1 = Gaussian, 2 = shapelet."""
    _single_term(sky)
    flux = [np.abs(np.asarray(sky.p_sref, float)), np.abs(np.asarray(sky.g_sref, float))]
    kind = [np.zeros(len(sky.p_sref), int), np.ones(len(sky.g_sref), int)]
    comp = [np.arange(len(sky.p_sref)), np.arange(len(sky.g_sref))]
    coef = [np.full(len(sky.p_sref), -1), np.full(len(sky.g_sref), -1)]
    nmax = int(max(sky.s_nmax)) if len(sky.s_nmax) else 0
    l1 = hermite_l1(nmax) if len(sky.s_nmax) else None
    for s in range(len(sky.s_nmax)):
        N = int(sky.s_nmax[s])
        n1, n2 = _orders(N)
        c = np.asarray(sky.coeffs[int(sky.s_coeff_off[s]):int(sky.s_coeff_off[s]) + n1.size], float)
        flux.append(np.abs(sky.s_sref[s] * c) * l1[n1] * l1[n2] / (2.0 * np.pi))
        kind.append(np.full(n1.size, 2))
        comp.append(np.full(n1.size, s))
        coef.append(np.arange(n1.size))
    return (np.concatenate(flux), np.concatenate(kind), np.concatenate(comp), np.concatenate(coef))


def keep_count(flux: np.ndarray, f: float) -> int:
    """Number of components kept: the largest N_comp with the N_comp largest
    |I| summing to at most f times the total (at least one for f > 0)."""
    if not 0.0 < f <= 1.0:
        raise ValueError("f must lie in (0, 1]")
    order = np.sort(np.abs(flux))[::-1]
    cum = np.cumsum(order)
    n = int(np.searchsorted(cum, f * cum[-1], side="right"))
    return max(1, min(n, flux.size))


def _rebuild(sky, keep_p, keep_g, coeffs, keep_s):
    offs, packed = [], []
    base = 0
    for s in np.flatnonzero(keep_s):
        c = coeffs[s]
        offs.append(base)
        packed.append(c)
        base += c.size
    sel = np.flatnonzero(keep_s)
    return dataclasses.replace(
        sky,
        p_ra=np.asarray(sky.p_ra)[keep_p], p_dec=np.asarray(sky.p_dec)[keep_p],
        p_sref=np.asarray(sky.p_sref)[keep_p], p_alpha=np.asarray(sky.p_alpha)[keep_p],
        g_ra=np.asarray(sky.g_ra)[keep_g], g_dec=np.asarray(sky.g_dec)[keep_g],
        g_sref=np.asarray(sky.g_sref)[keep_g], g_alpha=np.asarray(sky.g_alpha)[keep_g],
        g_maj=np.asarray(sky.g_maj)[keep_g], g_min=np.asarray(sky.g_min)[keep_g],
        g_pa=np.asarray(sky.g_pa)[keep_g],
        s_ra=np.asarray(sky.s_ra)[sel], s_dec=np.asarray(sky.s_dec)[sel], s_sref=np.asarray(sky.s_sref)[sel],
        s_alpha=np.asarray(sky.s_alpha)[sel], s_beta1=np.asarray(sky.s_beta1)[sel],
        s_beta2=np.asarray(sky.s_beta2)[sel], s_pa=np.asarray(sky.s_pa)[sel],
        s_nmax=np.asarray(sky.s_nmax, np.int32)[sel],
        s_coeff_off=np.asarray(offs, np.int64),
        coeffs=np.concatenate(packed) if packed else np.zeros(0))


def _shapelet_coeffs(sky):
    out = []
    for s in range(len(sky.s_nmax)):
        N = int(sky.s_nmax[s])
        o = int(sky.s_coeff_off[s])
        out.append(np.array(sky.coeffs[o:o + (N + 1) * (N + 2) // 2], float))
    return out


def truncate_by_flux(sky, f: float):
    """The paper's truncation: keep the components (points, Gaussians and
    shapelet basis functions together) with the largest |I| whose cumulative
    |I| is at most f of the total.  Returns (truncated sky, number kept,
    number in the model, fraction of the total |I| kept)."""
    flux, kind, comp, coef = component_flux(sky)
    n = keep_count(flux, f)
    idx = np.argsort(-flux, kind="stable")[:n]
    keep = np.zeros(flux.size, bool)
    keep[idx] = True
    keep_p = np.sort(comp[keep & (kind == 0)])
    keep_g = np.sort(comp[keep & (kind == 1)])
    coeffs = _shapelet_coeffs(sky)
    kept_s = np.zeros(len(coeffs), bool)
    for s in range(len(coeffs)):
        sel = keep & (kind == 2) & (comp == s)
        mask = np.zeros(coeffs[s].size, bool)
        mask[coef[sel]] = True
        coeffs[s][~mask] = 0.0
        kept_s[s] = mask.any()
    return _rebuild(sky, keep_p, keep_g, coeffs, kept_s), n, flux.size, float(flux[keep].sum() / flux.sum())


def truncate_by_order(sky, nmax: int):
    """Set every shapelet coefficient with n1 + n2 > nmax to zero."""
    _single_term(sky)
    coeffs = _shapelet_coeffs(sky)
    for s, c in enumerate(coeffs):
        n1, n2 = _orders(int(sky.s_nmax[s]))
        c[n1 + n2 > nmax] = 0.0
    return _rebuild(sky, np.arange(len(sky.p_sref)), np.arange(len(sky.g_sref)), coeffs,
                    np.ones(len(coeffs), bool))
