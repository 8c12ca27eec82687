"""Seeded synthetic inputs shared by the tests, the benchmark and smoke().

This module holds no arithmetic of the transform itself: it only draws
coefficients, point sets and input maps with numpy's PCG64 generator.  The
sky regions of the paper (Fig. 1: SPT-3G main field ~1500 deg^2, BICEP3
~800 deg^2, EDFS ~57 deg^2) are not available as footprints, so RA/Dec
rectangles and polar discs of matching extent stand in for them.

Conventions: theta is the colatitude in [0, pi], phi the longitude in
[0, 2 pi), both in the patch frame (patch centre at the north pole, as in
step 1 of the method of Sec. II).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ARCMIN = math.pi / (180.0 * 60.0)
DEG = math.pi / 180.0

# Seed offsets per input kind; the workload number is added to each.
SEED_ALM = 1000
SEED_ALM2 = 1500
SEED_POINTS = 2000
SEED_MAP = 3000
SEED_SUBSAMPLE = 4000


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def nalm(lmax: int) -> int:
    return (lmax + 1) * (lmax + 2) // 2


def alm_m_l(lmax: int):
    """(m, l) of every entry of the m-major coefficient layout."""
    m = np.concatenate([np.full(lmax + 1 - mm, mm, dtype=np.int64) for mm in range(lmax + 1)])
    l = np.concatenate([np.arange(mm, lmax + 1, dtype=np.int64) for mm in range(lmax + 1)])
    return m, l


def gaussian_alm(lmax: int, spin: int, seed: int) -> np.ndarray:
    """g_lm, c_lm with E|a_lm|^2 = (l+1)^-2: m = 0 real N(0,1)/(l+1), m > 0
    complex with variance (l+1)^-2 / 2 per real part; entries with l < spin
    are zero.  Returns complex128 of shape (2, nalm)."""
    r = rng(seed)
    m, l = alm_m_l(lmax)
    out = np.zeros((2, nalm(lmax)), dtype=np.complex128)
    amp = 1.0 / (l + 1.0)
    for c in range(2):
        re = r.standard_normal(l.shape[0])
        im = r.standard_normal(l.shape[0])
        z = np.where(m == 0, re + 0j, (re + 1j * im) / math.sqrt(2.0))
        out[c] = z * amp
    out[:, l < spin] = 0.0
    return out


def gaussian_map(n: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Complex white noise with unit variance per real part."""
    r = rng(seed)
    return (r.standard_normal(n) + 1j * r.standard_normal(n)).astype(dtype)


def complex_noise(n: int, sigma: float, seed: int) -> np.ndarray:
    """Complex white noise with E|n|^2 = sigma^2 (variance sigma^2 / 2 per real part)."""
    r = rng(seed)
    return (r.standard_normal(n) + 1j * r.standard_normal(n)) * (sigma / math.sqrt(2.0))


def uniform_cap(n: int, radius: float, seed: int):
    """n points uniform in the spherical cap theta <= radius around the pole."""
    r = rng(seed)
    cth = r.uniform(math.cos(radius), 1.0, n)
    theta = np.arccos(np.clip(cth, -1.0, 1.0))
    phi = r.uniform(0.0, 2.0 * math.pi, n)
    return theta, phi


def _unit(theta, phi):
    st = np.sin(theta)
    return np.stack([st * np.cos(phi), st * np.sin(phi), np.cos(theta)], axis=-1)


def _angles(v):
    theta = np.arccos(np.clip(v[..., 2], -1.0, 1.0))
    phi = np.mod(np.arctan2(v[..., 1], v[..., 0]), 2.0 * math.pi)
    return theta, phi


def jitter(theta, phi, rms: float, r: np.random.Generator):
    """Displace every point by a Gaussian deflection of total RMS `rms`
    (per-component sigma rms/sqrt(2)) along the geodesic in the local
    (e_theta, e_phi) frame (exponential map)."""
    sig = rms / math.sqrt(2.0)
    dt = r.standard_normal(theta.shape[0]) * sig
    dp = r.standard_normal(theta.shape[0]) * sig
    v = _unit(theta, phi)
    ct, st, cp, sp = np.cos(theta), np.sin(theta), np.cos(phi), np.sin(phi)
    et = np.stack([ct * cp, ct * sp, -st], axis=-1)
    ep = np.stack([-sp, cp, np.zeros_like(sp)], axis=-1)
    a = np.hypot(dt, dp)
    safe = np.where(a > 0, a, 1.0)
    dirv = (dt[:, None] * et + dp[:, None] * ep) / safe[:, None]
    w = np.cos(a)[:, None] * v + np.sin(a)[:, None] * dirv
    return _angles(w)


def _rotate_to_pole(theta, phi, dec_c):
    """Rotate about the y axis so that (RA 0, Dec dec_c) lands on the pole."""
    v = _unit(theta, phi)
    psi = 0.5 * math.pi - dec_c
    c, s = math.cos(psi), math.sin(psi)
    x = v[:, 0] * c - v[:, 2] * s
    z = v[:, 0] * s + v[:, 2] * c
    return _angles(np.stack([x, v[:, 1], z], axis=-1))


def rect_raster(ra0, ra1, dec0, dec1, res):
    """RA/Dec rectangle (radians) sampled by rows every `res` in Dec with
    points every res / cos(Dec) in RA.  Returns equatorial (theta, phi)."""
    decs = np.arange(dec0, dec1 + 0.5 * res, res)
    th_list, ph_list = [], []
    for d in decs:
        step = res / max(math.cos(d), 1e-12)
        ras = np.arange(ra0, ra1 + 0.5 * step, step)
        th_list.append(np.full(ras.shape[0], 0.5 * math.pi - d))
        ph_list.append(np.mod(ras, 2.0 * math.pi))
    return np.concatenate(th_list), np.concatenate(ph_list)


def best_centre_dec(ra0, ra1, dec0, dec1):
    """Declination of the centre (at RA (ra0+ra1)/2 = 0) that minimises the
    largest angular distance to the rectangle's boundary (golden section)."""
    ts = np.linspace(0.0, 1.0, 401)
    bra = np.concatenate([ra0 + (ra1 - ra0) * ts, ra0 + (ra1 - ra0) * ts, np.full_like(ts, ra0), np.full_like(ts, ra1)])
    bde = np.concatenate([np.full_like(ts, dec0), np.full_like(ts, dec1), dec0 + (dec1 - dec0) * ts, dec0 + (dec1 - dec0) * ts])

    def radius(dc):
        cosd = np.sin(bde) * math.sin(dc) + np.cos(bde) * math.cos(dc) * np.cos(bra)
        return float(np.max(np.arccos(np.clip(cosd, -1.0, 1.0))))

    lo, hi = dec0, dec1
    g = (math.sqrt(5.0) - 1.0) / 2.0
    for _ in range(100):
        a = hi - g * (hi - lo)
        b = lo + g * (hi - lo)
        if radius(a) < radius(b):
            hi = b
        else:
            lo = a
    return 0.5 * (lo + hi)


def rect_patch(ra_half_deg, dec0_deg, dec1_deg, res_arcmin, jitter_arcmin, seed):
    """Jittered raster of an RA/Dec rectangle, rotated to the patch frame."""
    ra0, ra1 = -ra_half_deg * DEG, ra_half_deg * DEG
    dec0, dec1 = dec0_deg * DEG, dec1_deg * DEG
    th, ph = rect_raster(ra0, ra1, dec0, dec1, res_arcmin * ARCMIN)
    r = rng(seed)
    if jitter_arcmin > 0:
        th, ph = jitter(th, ph, jitter_arcmin * ARCMIN, r)
    dc = best_centre_dec(ra0, ra1, dec0, dec1)
    return _rotate_to_pole(th, ph, dc)


def disc_patch(radius_deg, res_arcmin, jitter_arcmin, seed):
    """Polar disc of the given radius: rings every `res` in theta with points
    every res / sin(theta) in phi, then jittered."""
    res = res_arcmin * ARCMIN
    rad = radius_deg * DEG
    ths = np.arange(0.5 * res, rad, res)
    th_list, ph_list = [], []
    for t in ths:
        n = max(1, int(round(2.0 * math.pi * math.sin(t) / res)))
        ph_list.append(np.arange(n) * (2.0 * math.pi / n))
        th_list.append(np.full(n, t))
    th, ph = np.concatenate(th_list), np.concatenate(ph_list)
    if jitter_arcmin > 0:
        th, ph = jitter(th, ph, jitter_arcmin * ARCMIN, rng(seed))
    return th, ph


@dataclasses.dataclass
class Workload:
    name: str
    lmax: int
    spin: int
    epsilon: float
    precision: str           # "fp64" or "fp32"
    theta: np.ndarray
    phi: np.ndarray
    seed_base: int

    @property
    def npoints(self) -> int:
        return int(self.theta.shape[0])

    def alm(self, which: int = 0) -> np.ndarray:
        return gaussian_alm(self.lmax, self.spin, (SEED_ALM if which == 0 else SEED_ALM2) + self.seed_base)

    def adjoint_map(self, dtype=np.complex128) -> np.ndarray:
        return gaussian_map(self.npoints, SEED_MAP + self.seed_base, dtype)

    def subsample(self, n: int) -> np.ndarray:
        """Seeded sorted subset of point indices (for oracle checks)."""
        n = min(n, self.npoints)
        return np.sort(rng(SEED_SUBSAMPLE + self.seed_base).choice(self.npoints, size=n, replace=False))

    def shuffled(self) -> "Workload":
        p = rng(SEED_POINTS + 100 + self.seed_base).permutation(self.npoints)
        return dataclasses.replace(self, name=self.name + "-shuffled", theta=self.theta[p], phi=self.phi[p])


def cap_small(n: int = 20000) -> Workload:
    """Spin-0, lmax 128, FP64, eps 1e-10: n points uniform in a 10 deg polar cap."""
    th, ph = uniform_cap(n, 10.0 * DEG, SEED_POINTS + 1)
    return Workload("cap10-l128-s0-fp64", 128, 0, 1e-10, "fp64", th, ph, 1)


def spt_like(lmax: int = 2048) -> Workload:
    """Spin-2, lmax 2048, FP64, eps 1e-10: RA [-50,50] x Dec [-71,-41] deg
    (~1658 deg^2, ~4% of the sky) at 1', 2.5' RMS jitter (~5.97M points)."""
    th, ph = rect_patch(50.0, -71.0, -41.0, 1.0, 2.5, SEED_POINTS + 2)
    return Workload("spt1658-l%d-s2-fp64" % lmax, lmax, 2, 1e-10, "fp64", th, ph, 2)


_POINTS: dict = {}  # point sets shared by workloads that differ only in precision


def spt_fine(precision: str = "fp32") -> Workload:
    """Spin-2, lmax 4096: RA [-48.4,48.4] x Dec [-70,-42] deg (~1501 deg^2)
    at 0.5', 2.5' RMS jitter (~21.6M points); eps 1e-5 FP32 or 1e-10 FP64."""
    if "spt_fine" not in _POINTS:
        _POINTS["spt_fine"] = rect_patch(48.4, -70.0, -42.0, 0.5, 2.5, SEED_POINTS + 3)
    th, ph = _POINTS["spt_fine"]
    eps = 1e-5 if precision == "fp32" else 1e-10
    return Workload("spt1501-l4096-s2-%s" % precision, 4096, 2, eps, precision, th, ph, 3)


SERVED_RADII = (2.0, 5.0, 10.0, 20.0)
SERVED_LMAX = (512, 1024, 2048, 4096)
SERVED_SPINS = (0, 2)


def served_patch(radius_deg: float, res_arcmin: float = 1.0):
    """Point set of one served disc: polar disc at `res` (1') with 2.5' jitter."""
    return disc_patch(radius_deg, res_arcmin, 2.5, SEED_POINTS + 4 + int(round(radius_deg * 100)))


def served_mix(n: int, seed: int = SEED_MAP + 4, radii=SERVED_RADII, lmaxes=SERVED_LMAX, spins=SERVED_SPINS):
    """n requests of the served mix: (radius, lmax, spin, op, data seed), uniform
    over the radius x lmax x spin combinations, 50/50 synthesis / adjoint."""
    r = rng(seed)
    out = []
    for i in range(n):
        out.append((float(radii[r.integers(len(radii))]), int(lmaxes[r.integers(len(lmaxes))]),
                    int(spins[r.integers(len(spins))]), "synth" if r.integers(2) == 0 else "adjoint",
                    int(seed * 7919 + i)))
    return out


def served_disc(radius_deg: float, lmax: int, spin: int) -> Workload:
    """One member of the served mix as a stand-alone workload (FP32, eps 1e-5)."""
    th, ph = served_patch(radius_deg)
    return Workload("disc%g-l%d-s%d-fp32" % (radius_deg, lmax, spin), lmax, spin, 1e-5, "fp32", th, ph, 4)


def autograd_patch() -> Workload:
    """Spin-2, lmax 3000, FP64: RA [-37.5,37.5] x Dec [-70,-45] deg (~999 deg^2)
    at 1', 2.5' RMS jitter (~3.6M points)."""
    th, ph = rect_patch(37.5, -70.0, -45.0, 1.0, 2.5, SEED_POINTS + 5)
    return Workload("rect999-l3000-s2-fp64", 3000, 2, 1e-10, "fp64", th, ph, 5)
