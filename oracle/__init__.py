"""Oracle for the partial-sky spin-weighted SHT -- TEST INFRASTRUCTURE ONLY.

A plain CPU direct sum of the spin-s synthesis (Sec. I, eq. syn), of its
adjoint (Sec. I, "Adjoint synthesis general") and of the per-ring azimuthal
Fourier coefficients of the same map, with sYlm from the Wigner-d definition
of Appendix A (eq. Ylm).  The arithmetic lives in ``oracle.c`` (long double
internally, double outputs); this module only builds and loads it and
marshals numpy arrays.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library.

Layouts: alm is complex128 of shape (2, nalm) (g then c), with
nalm = (lmax+1)(lmax+2)/2 and index(l, m) = m(2 lmax + 1 - m)/2 + l for m >= 0;
maps are complex128 of shape (npts,).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc + OpenMP."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_wigner_d.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
        lib.oracle_synth.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int64, dp, dp, dp, ctypes.c_int]
        lib.oracle_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int64, dp, dp, dp, ctypes.c_int]
        lib.oracle_ring_coeffs.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int]
        for f in (lib.oracle_wigner_d, lib.oracle_synth, lib.oracle_adjoint, lib.oracle_ring_coeffs):
            f.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def nalm(lmax: int) -> int:
    return (lmax + 1) * (lmax + 2) // 2


def alm_index(lmax: int, l, m):
    return m * (2 * lmax + 1 - m) // 2 + l


def wigner_d(lmax: int, a: int, b: int, theta: float) -> np.ndarray:
    """d^l_{a b}(theta) for l = 0..lmax (zero below max(|a|,|b|))."""
    out = np.zeros(lmax + 1, dtype=np.float64)
    _load().oracle_wigner_d(lmax, a, b, float(theta), _ptr(out))
    return out


def synth(alm: np.ndarray, theta: np.ndarray, phi: np.ndarray, lmax: int, spin: int, nthreads: int = 0) -> np.ndarray:
    """Direct-sum synthesis, eq. syn.  Returns complex128 (npts,)."""
    alm = np.ascontiguousarray(alm, dtype=np.complex128)
    assert alm.shape == (2, nalm(lmax))
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    out = np.zeros(th.shape[0], dtype=np.complex128)
    _load().oracle_synth(lmax, spin, _ptr(alm.view(np.float64)), th.shape[0], _ptr(th), _ptr(ph),
                         _ptr(out.view(np.float64)), nthreads)
    return out


def adjoint(fmap: np.ndarray, theta: np.ndarray, phi: np.ndarray, lmax: int, spin: int, nthreads: int = 0) -> np.ndarray:
    """Direct-sum adjoint synthesis (Sec. I).  Returns complex128 (2, nalm)."""
    fm = np.ascontiguousarray(fmap, dtype=np.complex128)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    out = np.zeros((2, nalm(lmax)), dtype=np.complex128)
    _load().oracle_adjoint(lmax, spin, _ptr(fm.view(np.float64)), th.shape[0], _ptr(th), _ptr(ph),
                           _ptr(out.view(np.float64)), nthreads)
    return out


def ring_coeffs(alm: np.ndarray, theta_rings: np.ndarray, lmax: int, spin: int, mmax: int, nthreads: int = 0) -> np.ndarray:
    """F_m(theta_j) for m = -mmax..mmax; complex128 of shape (2 mmax + 1, nring)."""
    alm = np.ascontiguousarray(alm, dtype=np.complex128)
    th = np.ascontiguousarray(theta_rings, dtype=np.float64)
    out = np.zeros((2 * mmax + 1, th.shape[0]), dtype=np.complex128)
    _load().oracle_ring_coeffs(lmax, spin, _ptr(alm.view(np.float64)), th.shape[0], _ptr(th), mmax,
                               _ptr(out.view(np.float64)), nthreads)
    return out


def alm_dot(a: np.ndarray, b: np.ndarray, lmax: int) -> float:
    """Real inner product on coefficient sets that obey the reality condition:
    sum over all -l <= m <= l of Re(conj(a) b), i.e. the m = 0 real parts once
    and the m > 0 terms twice."""
    m_of = np.concatenate([np.full(lmax + 1 - m, m) for m in range(lmax + 1)])
    w = np.where(m_of == 0, 1.0, 2.0)
    a0 = np.where(m_of == 0, a.real + 0j, a)
    b0 = np.where(m_of == 0, b.real + 0j, b)
    return float(np.sum(w * (np.conj(a0) * b0).real))


def map_dot(f: np.ndarray, g: np.ndarray) -> float:
    """Real inner product on maps: sum_p Re(conj(f_p) g_p)."""
    return float(np.sum((np.conj(f) * g).real))


# ---------------------------------------------------------------- rotations
#
# Patch frame (Sec. II, step 1: coordinates in which the patch centre is the
# north pole).  A rotation R = Rz(alpha) Ry(beta) Rz(gamma) (active, z-y-z
# Euler angles) acts on points as n -> R n and on a field as f -> f o R^-1.
# With the Wigner functions D^l_{m m'}(alpha, beta, gamma) =
# exp(-i m alpha) d^l_{m m'}(beta) exp(-i m' gamma) (d from wigner_d above) the
# coefficients of the rotated field are a'_lm = sum_{m'} D^l_{m m'} a_lm',
# a_{l,-m'} = (-1)^m' conj(a_lm') for fields that obey the reality condition;
# g and c of a spin field each rotate this way.


def rotation_matrix(alpha: float, beta: float, gamma: float) -> np.ndarray:
    """3x3 matrix of Rz(alpha) Ry(beta) Rz(gamma)."""
    def rz(a):
        c, s = np.cos(a), np.sin(a)
        return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])

    def ry(b):
        c, s = np.cos(b), np.sin(b)
        return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])

    return rz(alpha) @ ry(beta) @ rz(gamma)


def rotate_alm(alm: np.ndarray, lmax: int, alpha: float, beta: float, gamma: float) -> np.ndarray:
    """a'_lm = sum_{m'=-l..l} exp(-i m alpha) d^l_{m m'}(beta) exp(-i m' gamma) a_lm'
    for each row of alm (shape (ncomp, nalm), m >= 0 stored); O(lmax^3)."""
    alm = np.atleast_2d(np.asarray(alm, dtype=np.complex128))
    out = np.zeros_like(alm)
    l = np.arange(lmax + 1)
    for m in range(lmax + 1):
        acc = np.zeros((alm.shape[0], lmax + 1), dtype=np.complex128)
        for mp in range(-lmax, lmax + 1):
            d = wigner_d(lmax, m, mp, beta)
            k = abs(mp)
            lsel = l[max(m, k):]
            a = alm[:, alm_index(lmax, lsel, k)]
            if mp < 0:
                a = (-1) ** k * np.conj(a)
            if k == 0:
                a = a.real + 0j
            acc[:, lsel] += d[lsel] * np.exp(-1j * mp * gamma) * a
        lsel = l[m:]
        out[:, alm_index(lmax, lsel, m)] = np.exp(-1j * m * alpha) * acc[:, lsel]
    return out


def rotate_points(theta: np.ndarray, phi: np.ndarray, alpha: float, beta: float, gamma: float):
    """(theta', phi', psi) of the points R n, phi' in [0, 2 pi).  psi is the
    angle from the rotated local basis vector R e_theta(n) to e_theta(R n),
    measured towards e_phi(R n)."""
    R = rotation_matrix(alpha, beta, gamma)
    th = np.asarray(theta, dtype=np.float64)
    ph = np.asarray(phi, dtype=np.float64)
    n = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    et = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)])
    n2 = R @ n
    et_rot = R @ et
    th2 = np.arctan2(np.hypot(n2[0], n2[1]), n2[2])
    ph2 = np.mod(np.arctan2(n2[1], n2[0]), 2 * np.pi)
    et2 = np.stack([np.cos(th2) * np.cos(ph2), np.cos(th2) * np.sin(ph2), -np.sin(th2)])
    ep2 = np.stack([-np.sin(ph2), np.cos(ph2), np.zeros_like(ph2)])
    psi = np.arctan2(np.sum(et_rot * ep2, axis=0), np.sum(et_rot * et2, axis=0))
    return th2, ph2, psi
