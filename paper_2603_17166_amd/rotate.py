"""Patch frame (Sec. II, step 1): rotation of coefficients, points and spin
bases into coordinates in which the patch centre is the north pole.

R = Rz(alpha) Ry(beta) Rz(gamma) (active, z-y-z Euler angles).  With
``a2 = rotate_alm(a, lmax, *angles)`` and ``th2, ph2, psi = rotate_points(th, ph, *angles)``
the spin-s synthesis of a2 at (th2, ph2) equals exp(i s psi) times the
synthesis of a at (th, ph); ``spin_phase`` applies or removes that factor.
Every step runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .plan import _stream


def patch_angles(theta_c: float, phi_c: float, psi0: float = 0.0):
    """Euler angles that take the point (theta_c, phi_c) to the north pole
    (psi0 turns the patch about its centre afterwards)."""
    return (float(psi0), -float(theta_c), -float(phi_c))


def inverse_angles(alpha: float, beta: float, gamma: float):
    """Angles of R^-1 (also the adjoint of the coefficient rotation)."""
    return (-gamma, -beta, -alpha)


def rotate_alm(alm: torch.Tensor, lmax: int, alpha: float, beta: float, gamma: float, stream=None) -> torch.Tensor:
    """Rotated copy of alm: complex128 CUDA tensor (ncomp, nalm), ncomp 1 or 2."""
    if alm.dtype != torch.complex128 or not alm.is_cuda:
        raise TypeError("alm must be a complex128 CUDA tensor")
    a = alm.contiguous()
    flat = a.dim() == 1
    if flat:
        a = a.unsqueeze(0)
    nc = a.shape[0]
    if a.shape[1] != (lmax + 1) * (lmax + 2) // 2:
        raise ValueError("alm has %d entries per component, lmax %d needs %d" % (a.shape[1], lmax,
                                                                             (lmax + 1) * (lmax + 2) // 2))
    lib = _lib.load()
    need = ctypes.c_size_t()
    _lib.check(lib.psht_rotate_alm_workspace(int(lmax), int(nc), ctypes.byref(need)))
    out = torch.empty_like(a)
    with torch.cuda.device(a.device):
        ws = torch.empty(max(1, need.value), dtype=torch.uint8, device=a.device)
        _lib.check(lib.psht_rotate_alm(int(lmax), int(nc), float(alpha), float(beta), float(gamma), a.data_ptr(),
                                       out.data_ptr(), ws.data_ptr(), need.value, _stream(stream)))
    return out[0] if flat else out


def rotate_points(theta: torch.Tensor, phi: torch.Tensor, alpha: float, beta: float, gamma: float, stream=None):
    """(theta', phi', psi) of the points R n; float64 CUDA tensors."""
    th = theta.to(torch.float64).contiguous()
    ph = phi.to(device=th.device, dtype=torch.float64).contiguous()
    if not th.is_cuda or th.shape != ph.shape or th.dim() != 1:
        raise ValueError("theta and phi must be 1-D CUDA tensors of equal length")
    t2, p2, psi = torch.empty_like(th), torch.empty_like(th), torch.empty_like(th)
    with torch.cuda.device(th.device):
        _lib.check(_lib.load().psht_rotate_points(th.shape[0], float(alpha), float(beta), float(gamma),
                                                  th.data_ptr() or None, ph.data_ptr() or None,
                                                  t2.data_ptr() or None, p2.data_ptr() or None,
                                                  psi.data_ptr() or None, _stream(stream)))
    return t2, p2, psi


def spin_phase(fmap: torch.Tensor, psi: torch.Tensor, spin: int, sign: int = 1, stream=None) -> torch.Tensor:
    """fmap *= exp(i sign spin psi) in place (complex64 or complex128 CUDA tensor)."""
    if fmap.dtype not in (torch.complex64, torch.complex128) or not fmap.is_contiguous():
        raise TypeError("fmap must be a contiguous complex CUDA tensor")
    if psi.dtype != torch.float64 or psi.shape != fmap.shape:
        raise ValueError("psi must be float64 with the map's shape")
    with torch.cuda.device(fmap.device):
        _lib.check(_lib.load().psht_spin_phase(fmap.numel(), int(spin), int(sign),
                                               1 if fmap.dtype == torch.complex64 else 0,
                                               psi.contiguous().data_ptr() or None, fmap.data_ptr() or None,
                                               _stream(stream)))
    return fmap


__all__ = ["patch_angles", "inverse_angles", "rotate_alm", "rotate_points", "spin_phase"]
