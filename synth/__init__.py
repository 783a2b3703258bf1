"""Seeded synthetic inputs for direct-Fourier visibility prediction.

This module only builds inputs: an MWA-like array and its baseline uvw (in
metres), channel frequencies, and sky-component lists (points, Gaussians,
shapelets).  It holds none of the prediction arithmetic; both the GPU library
and the CPU oracle take its arrays as they are.

Recipe (shapes follow the paper's workloads; the data themselves are
synthetic stand-ins for the VLA Fornax A image, the real MWA observations
and the GLEAM-based sky, none of which are used):

* array: tiles uniform in a disk of radius 1.5 km in (east, north), zero
  height, latitude -26.7 deg (an MWA phase-I-like layout, maximum baseline
  about 3 km; paper Sec. 4.1);
* baselines: every tile pair i < j, baseline vector = tile_j - tile_i;
* uvw: textbook local (east, north, up) -> equatorial XYZ -> (u, v, w) at
  hour angle H towards the phase centre (RA 0, Dec -37 deg); time steps of
  8 s about H = 0 (the paper's peel cadence, Sec. 5);
* channels: centres of equal-width bins (80 kHz at 182 MHz, or 78.125 kHz
  over 150-180 MHz, or four 2.5 MHz bins over 170-180 MHz);
* positions: uniform in solid angle on a cap about the phase centre;
* fluxes: log-uniform, or a power-law source count dN/dS ~ S^-1.6 drawn by
  inverse CDF; spectral index N(-0.8, 0.2); reference frequency 180 MHz;
* Gaussians: major FWHM U(1', 20'), minor = U(0.3, 1) * major, PA U[0, pi);
* shapelets: beta1, beta2 U(5', 30') unless fixed, PA U[0, pi), coefficients
  N(0,1) exp(-(n1+n2)/tau) packed n1-major (n1 = 0..N, n2 = 0..N-n1) and
  rescaled so that the envelope at the uv origin equals one (the paper's
  C <- C / I convention, Sec. 3.2), with a guard that redraws a set whose
  raw value at the origin is too close to zero.

Seeds: ``numpy.random.default_rng(200509316 + config_index)``; draw order
array -> times -> points -> Gaussians -> shapelets -> noise.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

C_LIGHT = 299792458.0
SIDEREAL_DAY_S = 86164.0905
LAT_RAD = math.radians(-26.7)
RA0_RAD = 0.0
DEC0_RAD = math.radians(-37.0)
NU_REF_HZ = 180e6
ARCMIN = math.radians(1.0 / 60.0)
SEED_BASE = 200509316


@dataclasses.dataclass
class Obs:
    """One observation: uvw per (time, baseline) in metres and channel list."""

    n_time: int
    n_bl: int
    n_chan: int
    uvw_m: np.ndarray  # float64 [n_time, n_bl, 3]
    freq_hz: np.ndarray  # float64 [n_chan]
    ra0: float = RA0_RAD
    dec0: float = DEC0_RAD
    sign: int = -1
    beam_fwhm_rad: float = 0.0
    beam_nu_ref_hz: float = 0.0
    n_tiles: int = 0

    @property
    def n_vis(self) -> int:
        return self.n_time * self.n_bl * self.n_chan


@dataclasses.dataclass
class Sky:
    """Component lists.  Angles in radians, fluxes in Jy at ``nu_ref_hz``."""

    nu_ref_hz: float
    p_ra: np.ndarray
    p_dec: np.ndarray
    p_sref: np.ndarray
    p_alpha: np.ndarray
    g_ra: np.ndarray
    g_dec: np.ndarray
    g_sref: np.ndarray
    g_alpha: np.ndarray
    g_maj: np.ndarray
    g_min: np.ndarray
    g_pa: np.ndarray
    s_ra: np.ndarray
    s_dec: np.ndarray
    s_sref: np.ndarray
    s_alpha: np.ndarray
    s_beta1: np.ndarray
    s_beta2: np.ndarray
    s_pa: np.ndarray
    s_nmax: np.ndarray  # int32
    s_coeff_off: np.ndarray  # int64
    coeffs: np.ndarray  # float64, packed per shapelet
    dc_redraws: int = 0
    # None, or int32 [n_shp] spectral terms per shapelet: coefficient blocks
    # C_0 .. C_{Q-1} following each other, C(nu) = sum_q C_q ln(nu/nu_ref)^q
    s_nterm: Optional[np.ndarray] = None

    @property
    def n_point(self) -> int:
        return int(self.p_ra.size)

    @property
    def n_gauss(self) -> int:
        return int(self.g_ra.size)

    @property
    def n_shp(self) -> int:
        return int(self.s_ra.size)

    def n_basis(self) -> int:
        """Number of shapelet basis functions, (N+2)(N+1)/2 per shapelet."""
        return int(sum((int(n) + 2) * (int(n) + 1) // 2 for n in self.s_nmax))

    def nominal_components(self) -> int:
        """Points + Gaussians + shapelet basis functions."""
        return self.n_point + self.n_gauss + self.n_basis()


def empty_sky(nu_ref_hz: float = NU_REF_HZ) -> Sky:
    z = np.zeros(0, np.float64)
    return Sky(nu_ref_hz, z, z, z, z, z, z, z, z, z, z, z, z, z, z, z, z, z, z,
               np.zeros(0, np.int32), np.zeros(0, np.int64), z)


def shapelet_terms(sky: Sky) -> np.ndarray:
    """Spectral terms per shapelet (1 each when the sky has none)."""
    if sky.s_nterm is None:
        return np.ones(sky.n_shp, np.int32)
    return np.asarray(sky.s_nterm, np.int32)


def concat_skies(*skies: Sky) -> Sky:
    """Component-wise concatenation (order preserved)."""
    out = {}
    for f in dataclasses.fields(Sky):
        if f.name in ("nu_ref_hz", "dc_redraws", "s_coeff_off", "coeffs", "s_nterm"):
            continue
        out[f.name] = np.concatenate([getattr(s, f.name) for s in skies])
    if any(s.s_nterm is not None for s in skies):
        out["s_nterm"] = np.concatenate([shapelet_terms(s) for s in skies]).astype(np.int32)
    coeffs, offs, base = [], [], 0
    for s in skies:
        coeffs.append(s.coeffs)
        offs.append(s.s_coeff_off.astype(np.int64) + base)
        base += s.coeffs.size
    return Sky(nu_ref_hz=skies[0].nu_ref_hz, s_coeff_off=np.concatenate(offs).astype(np.int64),
               coeffs=np.concatenate(coeffs), dc_redraws=sum(s.dc_redraws for s in skies), **out)


def select_components(sky: Sky, points=None, gauss=None, shapelets=None) -> Sky:
    """Sub-sky holding the listed component indices of each kind."""
    def idx(sel, n):
        return np.arange(n) if sel is None else np.asarray(sel, dtype=np.int64)
    pi, gi, si = idx(points, sky.n_point), idx(gauss, sky.n_gauss), idx(shapelets, sky.n_shp)
    terms = shapelet_terms(sky)
    coeffs, offs, base = [], [], 0
    for s in si:
        n = int(sky.s_nmax[s])
        cnt = (n + 2) * (n + 1) // 2 * int(terms[s])
        o = int(sky.s_coeff_off[s])
        coeffs.append(sky.coeffs[o:o + cnt])
        offs.append(base)
        base += cnt
    return Sky(
        nu_ref_hz=sky.nu_ref_hz,
        p_ra=sky.p_ra[pi], p_dec=sky.p_dec[pi], p_sref=sky.p_sref[pi], p_alpha=sky.p_alpha[pi],
        g_ra=sky.g_ra[gi], g_dec=sky.g_dec[gi], g_sref=sky.g_sref[gi], g_alpha=sky.g_alpha[gi],
        g_maj=sky.g_maj[gi], g_min=sky.g_min[gi], g_pa=sky.g_pa[gi],
        s_ra=sky.s_ra[si], s_dec=sky.s_dec[si], s_sref=sky.s_sref[si], s_alpha=sky.s_alpha[si],
        s_beta1=sky.s_beta1[si], s_beta2=sky.s_beta2[si], s_pa=sky.s_pa[si],
        s_nmax=sky.s_nmax[si].astype(np.int32),
        s_coeff_off=np.asarray(offs, np.int64),
        coeffs=np.concatenate(coeffs) if coeffs else np.zeros(0, np.float64),
        s_nterm=None if sky.s_nterm is None else terms[si].astype(np.int32),
    )


def with_spectral_terms(sky: Sky, rng: np.random.Generator, n_terms: int, scale: float = 0.3) -> Sky:
    """The sky with every shapelet given n_terms spectral terms: C_0 is the
    shapelet's coefficient set and C_q = (scale / q!) d_q * C_0 with d_q
    drawn N(0, 1) per coefficient -- a spectral index that varies across the
    source by about `scale` (ln(nu/nu_ref) is ~0.1 over a 30 MHz band at
    165 MHz)."""
    coeffs, offs, base = [], [], 0
    for s in range(sky.n_shp):
        n = int(sky.s_nmax[s])
        cnt = (n + 2) * (n + 1) // 2
        o = int(sky.s_coeff_off[s])
        c0 = np.asarray(sky.coeffs[o:o + cnt], np.float64)
        offs.append(base)
        coeffs.append(c0)
        for q in range(1, n_terms):
            coeffs.append(scale / math.factorial(q) * rng.standard_normal(cnt) * c0)
        base += cnt * n_terms
    return dataclasses.replace(sky, s_coeff_off=np.asarray(offs, np.int64),
                               coeffs=np.concatenate(coeffs) if coeffs else np.zeros(0, np.float64),
                               s_nterm=np.full(sky.n_shp, n_terms, np.int32))


# --------------------------------------------------------------------------
# array and observation
# --------------------------------------------------------------------------

def tile_layout(rng: np.random.Generator, n_tiles: int, radius_m: float = 1500.0):
    """Tiles uniform in a disk: returns east, north in metres."""
    r = radius_m * np.sqrt(rng.random(n_tiles))
    th = 2.0 * math.pi * rng.random(n_tiles)
    return r * np.cos(th), r * np.sin(th)


def baselines_enu(east: np.ndarray, north: np.ndarray) -> np.ndarray:
    """All pairs i < j; returns [B, 3] (east, north, up) baseline vectors."""
    i, j = np.triu_indices(east.size, k=1)
    return np.stack([east[j] - east[i], north[j] - north[i], np.zeros(i.size)], axis=1)


def uvw_from_enu(bl_enu: np.ndarray, hour_angle: float, dec0: float = DEC0_RAD,
                 lat: float = LAT_RAD) -> np.ndarray:
    """Textbook (east, north, up) -> equatorial (X, Y, Z) -> (u, v, w) at hour
    angle H towards declination dec0.  Metres."""
    e, n, up = bl_enu[:, 0], bl_enu[:, 1], bl_enu[:, 2]
    X = -math.sin(lat) * n + math.cos(lat) * up
    Y = e
    Z = math.cos(lat) * n + math.sin(lat) * up
    sh, ch = math.sin(hour_angle), math.cos(hour_angle)
    sd, cd = math.sin(dec0), math.cos(dec0)
    u = sh * X + ch * Y
    v = -sd * ch * X + sd * sh * Y + cd * Z
    w = cd * ch * X - cd * sh * Y + sd * Z
    return np.stack([u, v, w], axis=1)


def hour_angles(n_time: int, dt_s: float = 8.0) -> np.ndarray:
    t = np.arange(n_time, dtype=np.float64) - 0.5 * (n_time - 1)
    return t * dt_s * 2.0 * math.pi / SIDEREAL_DAY_S


def make_obs(rng: np.random.Generator, n_tiles: int, n_time: int, freq_hz: np.ndarray,
             dt_s: float = 8.0, sign: int = -1, beam_fwhm_rad: float = 0.0,
             beam_nu_ref_hz: float = 0.0, radius_m: float = 1500.0) -> Obs:
    east, north = tile_layout(rng, n_tiles, radius_m)
    bl = baselines_enu(east, north)
    has = hour_angles(n_time, dt_s)
    uvw = np.stack([uvw_from_enu(bl, h) for h in has], axis=0)
    freq_hz = np.asarray(freq_hz, np.float64)
    return Obs(n_time=n_time, n_bl=bl.shape[0], n_chan=freq_hz.size, uvw_m=np.ascontiguousarray(uvw),
               freq_hz=freq_hz, sign=sign, beam_fwhm_rad=beam_fwhm_rad,
               beam_nu_ref_hz=beam_nu_ref_hz, n_tiles=n_tiles)


def antenna_pairs(n_tiles: int):
    """Tiles (ant1, ant2) of each baseline, in the order of baselines_enu."""
    i, j = np.triu_indices(n_tiles, k=1)
    return i.astype(np.int32), j.astype(np.int32)


def random_gains(rng: np.random.Generator, n_time: int, n_chan: int, n_ant: int, amp_sigma: float = 0.1,
                 phase_sigma: float = 0.5) -> np.ndarray:
    """Synthetic complex tile gains [n_time, n_chan, n_ant]: per tile a random
    amplitude and phase, a linear slope of each across the band and a small
    drift in time."""
    amp0 = 1.0 + amp_sigma * rng.standard_normal(n_ant)
    ph0 = phase_sigma * rng.standard_normal(n_ant)
    amp_slope = 0.2 * amp_sigma * rng.standard_normal(n_ant)
    ph_slope = 0.5 * phase_sigma * rng.standard_normal(n_ant)
    drift = 0.05 * phase_sigma * rng.standard_normal(n_ant)
    x = np.linspace(-0.5, 0.5, n_chan) if n_chan > 1 else np.zeros(1)
    t = np.linspace(-0.5, 0.5, n_time) if n_time > 1 else np.zeros(1)
    amp = amp0[None, None, :] + amp_slope[None, None, :] * x[None, :, None]
    ph = ph0[None, None, :] + ph_slope[None, None, :] * x[None, :, None] + drift[None, None, :] * t[:, None, None]
    return amp * np.exp(1j * ph)


def channels(centre_hz: float, width_hz: float, n: int) -> np.ndarray:
    """Centres of n equal bins of width width_hz, centred on centre_hz."""
    return centre_hz + (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * width_hz


def band(lo_hz: float, hi_hz: float, n: int) -> np.ndarray:
    """Centres of n equal bins spanning [lo_hz, hi_hz]."""
    w = (hi_hz - lo_hz) / n
    return lo_hz + (np.arange(n, dtype=np.float64) + 0.5) * w


# --------------------------------------------------------------------------
# sky
# --------------------------------------------------------------------------

def offset_to_radec(rho: np.ndarray, psi: np.ndarray, ra0: float = RA0_RAD, dec0: float = DEC0_RAD):
    """Position at angular distance rho and position angle psi (north through
    east) from (ra0, dec0)."""
    sd = np.sin(dec0) * np.cos(rho) + np.cos(dec0) * np.sin(rho) * np.cos(psi)
    dec = np.arcsin(np.clip(sd, -1.0, 1.0))
    ra = ra0 + np.arctan2(np.sin(psi) * np.sin(rho) * np.cos(dec0),
                          np.cos(rho) - np.sin(dec0) * sd)
    return ra, dec


def cap_positions(rng: np.random.Generator, n: int, radius_rad: float):
    """Uniform in solid angle on a cap of the given radius."""
    cosr = 1.0 - rng.random(n) * (1.0 - math.cos(radius_rad))
    rho = np.arccos(np.clip(cosr, -1.0, 1.0))
    psi = 2.0 * math.pi * rng.random(n)
    return offset_to_radec(rho, psi)


def loguniform(rng: np.random.Generator, n: int, lo: float, hi: float) -> np.ndarray:
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n))


def powerlaw_counts(rng: np.random.Generator, n: int, smin: float, smax: float,
                    slope: float = -1.6) -> np.ndarray:
    """dN/dS ~ S^slope on [smin, smax] by inverse CDF."""
    q = slope + 1.0
    u = rng.random(n)
    return (smin ** q + u * (smax ** q - smin ** q)) ** (1.0 / q)


def _basis_at_origin(nmax: int) -> np.ndarray:
    """Value at zero of the orthonormal Hermite functions, n = 0..nmax:
    zero for odd n; for even n the textbook ratio
    phi_n(0) = -sqrt((n-1)/n) phi_{n-2}(0), phi_0(0) = pi^(-1/4)."""
    out = np.zeros(nmax + 1)
    out[0] = math.pi ** -0.25
    for n in range(2, nmax + 1, 2):
        out[n] = -math.sqrt((n - 1.0) / n) * out[n - 2]
    return out


def shapelet_orders(nmax: int):
    """(n1, n2) in packed n1-major order."""
    n1 = np.concatenate([np.full(nmax + 1 - a, a) for a in range(nmax + 1)])
    n2 = np.concatenate([np.arange(nmax + 1 - a) for a in range(nmax + 1)])
    return n1, n2


def shapelet_coeffs(rng: np.random.Generator, nmax: int, tau: float):
    """Coefficients N(0,1) exp(-(n1+n2)/tau), rescaled so that the envelope is
    one at the uv origin.  A draw whose raw origin value is below 0.1 of its
    standard deviation is redrawn.  Returns (coeffs, redraws)."""
    n1, n2 = shapelet_orders(nmax)
    damp = np.exp(-(n1 + n2) / tau)
    p0 = _basis_at_origin(nmax)
    w0 = p0[n1] * p0[n2] * np.where((n1 + n2) % 4 == 0, 1.0, -1.0)  # (s i)^n at even n
    sigma_dc = math.sqrt(float(np.sum((damp * w0) ** 2)))
    redraws = 0
    while True:
        c = rng.standard_normal(n1.size) * damp
        x0 = float(np.dot(c, w0))
        if abs(x0) >= 0.1 * sigma_dc:
            return c / x0, redraws
        redraws += 1


def make_sky(rng: np.random.Generator, *, n_point: int, n_gauss: int, shapelet_nmax: List[int],
             cap_rad: float, point_flux, gauss_flux=None, shapelet_sref=None,
             tau: float = 20.0, beta=None, alpha_mean: float = -0.8, alpha_sd: float = 0.2,
             shapelet_positions=None, nu_ref_hz: float = NU_REF_HZ) -> Sky:
    """Draw points, then Gaussians, then shapelets (in that order)."""
    gauss_flux = gauss_flux or point_flux
    p_ra, p_dec = cap_positions(rng, n_point, cap_rad)
    p_s = point_flux(rng, n_point)
    p_a = rng.normal(alpha_mean, alpha_sd, n_point)
    g_ra, g_dec = cap_positions(rng, n_gauss, cap_rad)
    g_s = gauss_flux(rng, n_gauss)
    g_a = rng.normal(alpha_mean, alpha_sd, n_gauss)
    g_maj = rng.uniform(1.0, 20.0, n_gauss) * ARCMIN
    g_min = g_maj * rng.uniform(0.3, 1.0, n_gauss)
    g_pa = rng.uniform(0.0, math.pi, n_gauss)
    ns = len(shapelet_nmax)
    if shapelet_positions is None:
        s_ra, s_dec = cap_positions(rng, ns, cap_rad)
    else:
        s_ra, s_dec = (np.asarray(v, np.float64) for v in shapelet_positions)
    if shapelet_sref is None:
        s_s = np.full(ns, 10.0)
    elif callable(shapelet_sref):
        s_s = shapelet_sref(rng, ns)
    else:
        s_s = np.asarray(shapelet_sref, np.float64)
    s_a = rng.normal(alpha_mean, alpha_sd, ns)
    if beta is None:
        b1 = rng.uniform(5.0, 30.0, ns) * ARCMIN
        b2 = rng.uniform(5.0, 30.0, ns) * ARCMIN
    else:
        b1 = np.asarray(beta[0], np.float64)
        b2 = np.asarray(beta[1], np.float64)
    s_pa = rng.uniform(0.0, math.pi, ns)
    coeffs, offs, base, redraws = [], [], 0, 0
    for n in shapelet_nmax:
        c, r = shapelet_coeffs(rng, int(n), tau)
        coeffs.append(c)
        offs.append(base)
        base += c.size
        redraws += r
    return Sky(
        nu_ref_hz=nu_ref_hz,
        p_ra=p_ra, p_dec=p_dec, p_sref=p_s, p_alpha=p_a,
        g_ra=g_ra, g_dec=g_dec, g_sref=g_s, g_alpha=g_a, g_maj=g_maj, g_min=g_min, g_pa=g_pa,
        s_ra=np.asarray(s_ra, np.float64), s_dec=np.asarray(s_dec, np.float64), s_sref=s_s,
        s_alpha=s_a, s_beta1=b1, s_beta2=b2, s_pa=s_pa,
        s_nmax=np.asarray(shapelet_nmax, np.int32), s_coeff_off=np.asarray(offs, np.int64),
        coeffs=np.concatenate(coeffs) if coeffs else np.zeros(0, np.float64),
        dc_redraws=redraws,
    )


def _lu(lo, hi):
    return lambda rng, n: loguniform(rng, n, lo, hi)


def _pl(lo, hi, slope=-1.6):
    return lambda rng, n: powerlaw_counts(rng, n, lo, hi, slope)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

CONFIG_NAMES = {
    0: "tiny-fp64: 32 tiles, 1 time, 4 ch, 100 pt + 10 gauss + 1 shapelet N=10",
    1: "mwa-like: 128 tiles, 14 x 8 s, 32 x 80 kHz @182 MHz, 20000 pt + 2000 gauss + 2 shapelets N=54, Gaussian beam",
    2: "fornax-like: 128 tiles, 14 x 8 s, 32 x 80 kHz, 2 shapelet lobes N=70 (750 Jy) + 10 Jy core",
    3: "serving stream: 256 requests, Poisson 20/s",
    4: "large peel: 256 tiles, 1 time, 384 ch 150-180 MHz, 100000 pt + 5000 gauss + 10 shapelets N=80",
}


def config_rng(index: int, seed: Optional[int] = None) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + index if seed is None else seed)


def make_config(index: int, seed: Optional[int] = None, **over):
    """(obs, sky) for workloads 0, 1, 2, 4.  Keyword overrides shrink a
    workload for tests: n_tiles, n_time, n_chan, n_point, n_gauss,
    shapelet_nmax."""
    rng = config_rng(index, seed)
    if index == 0:
        obs = make_obs(rng, over.get("n_tiles", 32), over.get("n_time", 1),
                       over.get("freq_hz", band(170e6, 180e6, over.get("n_chan", 4))))
        sky = make_sky(rng, n_point=over.get("n_point", 100), n_gauss=over.get("n_gauss", 10),
                       shapelet_nmax=over.get("shapelet_nmax", [10]), cap_rad=math.radians(5.0),
                       point_flux=_lu(0.1, 10.0), shapelet_sref=[5.0] * len(over.get("shapelet_nmax", [10])),
                       tau=5.0, beta=over.get("beta", ([10 * ARCMIN] * len(over.get("shapelet_nmax", [10])),
                                                        [10 * ARCMIN] * len(over.get("shapelet_nmax", [10])))))
        return obs, sky
    if index == 1:
        obs = make_obs(rng, over.get("n_tiles", 128), over.get("n_time", 14),
                       over.get("freq_hz", channels(182e6, 80e3, over.get("n_chan", 32))),
                       beam_fwhm_rad=math.radians(25.0), beam_nu_ref_hz=150e6)
        sky = make_sky(rng, n_point=over.get("n_point", 20000), n_gauss=over.get("n_gauss", 2000),
                       shapelet_nmax=over.get("shapelet_nmax", [54, 54]), cap_rad=math.radians(10.0),
                       point_flux=_pl(0.05, 50.0), tau=20.0)
        return obs, sky
    if index == 2:
        obs = make_obs(rng, over.get("n_tiles", 128), over.get("n_time", 14),
                       over.get("freq_hz", channels(182e6, 80e3, over.get("n_chan", 32))))
        nm = over.get("shapelet_nmax", [70, 70])
        off = math.radians(0.3)
        ra, dec = offset_to_radec(np.array([off, off]), np.array([math.pi / 2, -math.pi / 2]))
        lobes = make_sky(rng, n_point=0, n_gauss=0, shapelet_nmax=nm, cap_rad=math.radians(1.0),
                         point_flux=_lu(1, 2), shapelet_sref=[375.0, 375.0][:len(nm)], tau=20.0,
                         beta=([15 * ARCMIN, 25 * ARCMIN][:len(nm)], [15 * ARCMIN, 25 * ARCMIN][:len(nm)]),
                         alpha_mean=-0.8, alpha_sd=0.0,
                         shapelet_positions=(ra[:len(nm)], dec[:len(nm)]))
        core = empty_sky()
        core.p_ra = np.array([RA0_RAD])
        core.p_dec = np.array([DEC0_RAD])
        core.p_sref = np.array([10.0])
        core.p_alpha = np.array([-0.8])
        sky = concat_skies(core, lobes)
        return obs, sky
    if index == 4:
        obs = make_obs(rng, over.get("n_tiles", 256), over.get("n_time", 1),
                       over.get("freq_hz", band(150e6, 180e6, over.get("n_chan", 384))))
        sky = make_sky(rng, n_point=over.get("n_point", 100000), n_gauss=over.get("n_gauss", 5000),
                       shapelet_nmax=over.get("shapelet_nmax", [80] * 10), cap_rad=math.radians(10.0),
                       point_flux=_pl(0.05, 50.0), shapelet_sref=_lu(20.0, 200.0), tau=20.0)
        return obs, sky
    raise ValueError("workload %d has no single (obs, sky); use make_requests for the serving stream" % index)


def make_paper_cost_comparison(seed: Optional[int] = None):
    """The paper's model-cost comparison (Sec. 5.3): one peel observation
    (MWA phase I layout, 15 x 8 s = 2 min, 384 x 80 kHz), phase-centred on
    the source, predicted either from an MS CLEAN-like model of 4540 points
    and 1791 Gaussians or from two shapelet lobes with p_max = 86 (7656 basis
    functions).  Both models carry 500 Jy at 180 MHz, spectral index -0.8, and
    lie within 0.5 deg of the centre.  Returns (obs, clean_sky, shapelet_sky)."""
    rng = np.random.default_rng(SEED_BASE + 10 if seed is None else seed)
    obs = make_obs(rng, 128, 15, channels(182e6, 80e3, 384))
    half = math.radians(0.5)
    clean = make_sky(rng, n_point=4540, n_gauss=1791, shapelet_nmax=[], cap_rad=half,
                     point_flux=lambda r, n: r.exponential(1.0, n), alpha_mean=-0.8, alpha_sd=0.0)
    tot = clean.p_sref.sum() + clean.g_sref.sum()
    clean.p_sref = clean.p_sref * 500.0 / tot
    clean.g_sref = clean.g_sref * 500.0 / tot
    off = math.radians(0.3)
    ra, dec = offset_to_radec(np.array([off, off]), np.array([math.pi / 2, -math.pi / 2]))
    lobes = make_sky(rng, n_point=0, n_gauss=0, shapelet_nmax=[86, 86], cap_rad=half,
                     point_flux=_lu(1, 2), shapelet_sref=[250.0, 250.0], tau=20.0,
                     beta=([15 * ARCMIN, 25 * ARCMIN], [15 * ARCMIN, 25 * ARCMIN]),
                     alpha_mean=-0.8, alpha_sd=0.0, shapelet_positions=(ra, dec))
    return obs, clean, lobes


@dataclasses.dataclass
class Request:
    kind: str  # "predict" or "subtract"
    t_arrival_s: float
    obs: Obs
    sky: Sky
    noise_seed: int


def make_requests(n_requests: int = 256, rate_hz: float = 20.0, seed: Optional[int] = None,
                  scale: float = 1.0) -> List[Request]:
    """Serving stream: Poisson arrivals; each request draws its own array,
    times, channels and sky.  ``scale`` < 1 shrinks sizes for tests."""
    rng = config_rng(3, seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n_requests))
    reqs = []
    for r in range(n_requests):
        sub = np.random.default_rng([SEED_BASE + 3, r] if seed is None else [seed, r])
        tiles = int(sub.choice([64, 128, 256]))
        tiles = max(4, int(round(tiles * math.sqrt(scale))))
        n_chan = max(1, int(round(int(sub.integers(8, 385)) * scale)))
        n_time = int(sub.integers(1, 15))
        obs = make_obs(sub, tiles, n_time, channels(182e6, 80e3, n_chan))
        n_pt = int(sub.poisson(2000 * scale))
        n_g = int(sub.poisson(200 * scale))
        n_s = int(sub.integers(0, 5))
        nm = [int(max(1, round(x * (scale if scale < 1 else 1)))) for x in sub.integers(20, 81, n_s)]
        sky = make_sky(sub, n_point=n_pt, n_gauss=n_g, shapelet_nmax=nm, cap_rad=math.radians(10.0),
                       point_flux=_pl(0.05, 50.0), shapelet_sref=_lu(1.0, 100.0), tau=20.0)
        kind = "predict" if sub.random() < 0.5 else "subtract"
        reqs.append(Request(kind=kind, t_arrival_s=float(t[r]), obs=obs, sky=sky,
                            noise_seed=int(sub.integers(0, 2**31 - 1))))
    return reqs


def noise_c64(shape, seed: int) -> np.ndarray:
    """N(0, 1 Jy) in real and imaginary parts, complex64."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
