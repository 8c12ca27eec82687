"""Python binding of the partial-sky SHT: plans, synthesis and adjoint.

Thin marshalling over the C ABI (include/psht.h): torch provides device
memory and the current HIP stream; every step of the transform runs in the
library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib


def nalm(lmax: int) -> int:
    return (lmax + 1) * (lmax + 2) // 2


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _device_f64(x, device) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        t = x.to(device=device, dtype=torch.float64)
    else:
        t = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device=device)
    return t.contiguous()


def _options(full_sky: bool, window: str, cl, lmax_rule: str = "band"):
    """psht_plan_options (and the array it points to, kept alive by the caller)."""
    opts = _lib.PlanOptions()
    opts.full_sky = 1 if full_sky else 0
    opts.window = _lib.WINDOWS[window]
    opts.lmax_rule = _lib.LMAX_RULES[lmax_rule]
    arr = None
    if cl is not None:
        arr = np.ascontiguousarray(cl, dtype=np.float64)
        opts.cl = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        opts.cl_lmax = int(arr.shape[0]) - 1
    return opts, arr


class Plan:
    """Plan for spin-`spin` synthesis / adjoint at the points (theta, phi)
    (patch frame: patch centre at the north pole), band limit `lmax`, target
    accuracy `epsilon`; precision "auto" (FP32 grid when epsilon >= 1e-6),
    "fp32" or "fp64".  Options: `full_sky` (Fourier-sphere transform over the
    whole sphere), `window` ("es", "kb" or "pswf" apodization bell), `cl` (power
    spectrum C_l, l = 0..lmax or more, to tune Lmax by the predicted error),
    `lmax_rule` ("band": eq. Lmax2; "cost": least Legendre work)."""

    def __init__(self, theta, phi, lmax: int, spin: int, epsilon: float, precision: str = "auto", device=None,
                 stream=None, full_sky: bool = False, window: str = "es", cl=None, lmax_rule: str = "band"):
        lib = _lib.load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        th = _device_f64(theta, self.device)
        ph = _device_f64(phi, self.device)
        if th.shape != ph.shape or th.dim() != 1:
            raise ValueError("theta and phi must be 1-D arrays of equal length")
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = _stream(stream)
            opts, _keep = _options(full_sky, window, cl, lmax_rule)
            _lib.check(lib.psht_plan_create_ex(ctypes.byref(handle), int(lmax), int(spin), int(th.shape[0]),
                                               th.data_ptr() or None, ph.data_ptr() or None, float(epsilon),
                                               _lib.PREC[precision], ctypes.byref(opts), st))
        self._h = handle
        info = _lib.PlanInfo()
        _lib.check(lib.psht_plan_query(self._h, ctypes.byref(info)))
        self.info = info.as_dict()
        self.lmax, self.spin, self.npoints = int(lmax), int(spin), int(th.shape[0])
        self.map_dtype = torch.complex64 if info.map_is_fp32 else torch.complex128
        self._ws = None

    # -- resources ---------------------------------------------------------
    def workspace(self, nmaps: int = 1) -> torch.Tensor:
        need = max(1, nmaps * self.info["workspace_bytes_per_map"])
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def close(self, sync: bool = True) -> None:
        """Free the plan's device memory.  sync=False skips the device
        synchronisation: only for a plan with no work in flight."""
        if getattr(self, "_h", None) is not None and self._h.value:
            if sync:
                torch.cuda.synchronize(self.device)
            _lib.load().psht_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- transforms --------------------------------------------------------
    def _alm_in(self, alm: torch.Tensor):
        if alm.dtype != torch.complex128:
            raise TypeError("alm must be complex128")
        if alm.device != self.device:
            raise ValueError("alm is on %s, plan on %s" % (alm.device, self.device))
        single = alm.dim() == 2
        a = alm.unsqueeze(0) if single else alm
        if a.dim() != 3 or a.shape[1:] != (2, nalm(self.lmax)):
            raise ValueError("alm must have shape (2, nalm) or (nmaps, 2, nalm)")
        return a.contiguous(), single

    # `workspace`: optional caller-owned uint8 device tensor of at least
    # nmaps * workspace_bytes_per_map bytes (calls that overlap on different
    # streams need distinct workspaces); by default the plan's own one.
    def synth(self, alm: torch.Tensor, out: torch.Tensor | None = None, stream=None, workspace=None) -> torch.Tensor:
        """Synthesis general (eq. syn): alm (2, nalm) or (nmaps, 2, nalm) complex128 -> map."""
        return self._synth("psht_synth", alm, out, stream, workspace)

    def synth_grad(self, alm_grad: torch.Tensor, out: torch.Tensor | None = None, stream=None,
                   workspace=None) -> torch.Tensor:
        """Gradient w.r.t. the map of a real loss of adjoint(map), from its gradient w.r.t. the adjoint's output."""
        return self._synth("psht_synth_grad", alm_grad, out, stream, workspace)

    def adjoint(self, fmap: torch.Tensor, out: torch.Tensor | None = None, stream=None, workspace=None) -> torch.Tensor:
        """Adjoint synthesis general: map (npts,) or (nmaps, npts) -> alm (.., 2, nalm) complex128."""
        return self._adjoint("psht_adjoint", fmap, out, stream, workspace)

    def adjoint_grad(self, map_grad: torch.Tensor, out: torch.Tensor | None = None, stream=None,
                     workspace=None) -> torch.Tensor:
        """Gradient w.r.t. alm of a real loss of synth(alm), from its gradient w.r.t. the synthesized map."""
        return self._adjoint("psht_adjoint_grad", map_grad, out, stream, workspace)

    def _workspace_for(self, nm: int, workspace):
        if workspace is None:
            return self.workspace(nm)
        if workspace.dtype != torch.uint8 or workspace.device != self.device or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 tensor on %s" % self.device)
        return workspace

    def _synth(self, fn: str, alm: torch.Tensor, out, stream, workspace) -> torch.Tensor:
        a, single = self._alm_in(alm)
        nm = a.shape[0]
        if out is None:
            out = torch.empty((nm, self.npoints), dtype=self.map_dtype, device=self.device)
        else:
            out = out.view(nm, self.npoints)
            if out.dtype != self.map_dtype or not out.is_contiguous():
                raise ValueError("out must be a contiguous %s tensor" % self.map_dtype)
        ws = self._workspace_for(nm, workspace)
        with torch.cuda.device(self.device):
            _lib.check(getattr(_lib.load(), fn)(self._h, nm, a.data_ptr(), out.data_ptr() or None, ws.data_ptr(),
                                                ws.numel(), _stream(stream)))
        return out[0] if single else out

    def _adjoint(self, fn: str, fmap: torch.Tensor, out, stream, workspace) -> torch.Tensor:
        if fmap.dtype != self.map_dtype:
            raise TypeError("map must be %s for this plan" % self.map_dtype)
        if fmap.device != self.device:
            raise ValueError("map is on %s, plan on %s" % (fmap.device, self.device))
        single = fmap.dim() == 1
        f = (fmap.unsqueeze(0) if single else fmap).contiguous()
        if f.shape[1] != self.npoints:
            raise ValueError("map has %d points, plan %d" % (f.shape[1], self.npoints))
        nm = f.shape[0]
        if out is None:
            out = torch.empty((nm, 2, nalm(self.lmax)), dtype=torch.complex128, device=self.device)
        else:
            if out.dtype != torch.complex128 or not out.is_contiguous() or out.numel() != nm * 2 * nalm(self.lmax):
                raise ValueError("out must be a contiguous complex128 tensor of %d elements" % (nm * 2 * nalm(self.lmax)))
            out = out.view(nm, 2, nalm(self.lmax))
        ws = self._workspace_for(nm, workspace)
        with torch.cuda.device(self.device):
            _lib.check(getattr(_lib.load(), fn)(self._h, nm, f.data_ptr() or None, out.data_ptr(), ws.data_ptr(),
                                                ws.numel(), _stream(stream)))
        return out[0] if single else out

    def dropped_points(self, stream=None) -> int:
        """Points the NUFFT kernels skipped because their stencil left their tile (0 unless broken)."""
        v = ctypes.c_int64()
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().psht_plan_check(self._h, ctypes.byref(v), _stream(stream)))
        return int(v.value)

    def set_timing(self, enable: bool = True, stages=None) -> None:
        """Record HIP events around the stage launches of later calls (every stage,
        or only those named in `stages`) and reset the totals."""
        mask = 0
        if enable:
            mask = (1 << len(_lib.STAGE_NAMES)) - 1 if stages is None else \
                sum(1 << _lib.STAGE_NAMES.index(s) for s in stages)
        _lib.check(_lib.load().psht_plan_set_timing(self._h, mask))

    def timing(self) -> dict:
        """{stage: (total ms, launches)} since timing was enabled (synchronises the events)."""
        ms = (ctypes.c_double * 10)()
        n = (ctypes.c_int64 * 10)()
        _lib.check(_lib.load().psht_plan_timing(self._h, ms, n))
        return {name: (ms[i], n[i]) for i, name in enumerate(_lib.STAGE_NAMES)}

    def stage(self, stage: int, inp: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().psht_stage(self._h, stage, inp.data_ptr(), out.data_ptr(), _stream(stream)))
        return out

    def legendre_synth(self, alm: torch.Tensor, workspace: bool = False) -> torch.Tensor:
        """Per-ring Fourier coefficients F_m(theta_j), shape (2 mmax + 1, Lmax + 1).  With workspace=True
        through the work decomposition of synth (degree segments when info["syn_segment"] is non-zero)."""
        out = torch.empty((2 * self.info["mmax"] + 1, self.info["Lmax"] + 1), dtype=torch.complex128,
                          device=self.device)
        if workspace:
            return self._stage_ws(_lib.STAGE_LEGENDRE_SYNTH, alm.contiguous(), out)
        return self.stage(_lib.STAGE_LEGENDRE_SYNTH, alm.contiguous(), out)

    def legendre_adjoint(self, F: torch.Tensor) -> torch.Tensor:
        out = torch.empty((2, nalm(self.lmax)), dtype=torch.complex128, device=self.device)
        return self.stage(_lib.STAGE_LEGENDRE_ADJOINT, F.contiguous(), out)

    def _stage_ws(self, stage: int, inp: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
        ws = self.workspace(1)
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().psht_stage_ex(self._h, stage, inp.data_ptr(), out.data_ptr(), ws.data_ptr(),
                                                 ws.numel(), _stream(stream)))
        return out

    def fourier_synth(self, F: torch.Tensor) -> torch.Tensor:
        """Map from per-ring Fourier coefficients F (2 mmax + 1, Lmax + 1): Theta and phi stages and interpolation."""
        out = torch.empty(self.npoints, dtype=self.map_dtype, device=self.device)
        return self._stage_ws(_lib.STAGE_FOURIER_SYNTH, F.to(torch.complex128).contiguous(), out)

    def fourier_adjoint(self, fmap: torch.Tensor) -> torch.Tensor:
        """Transpose of fourier_synth: (2 mmax + 1, Lmax + 1) complex128 from a map."""
        out = torch.empty((2 * self.info["mmax"] + 1, self.info["Lmax"] + 1), dtype=torch.complex128,
                          device=self.device)
        return self._stage_ws(_lib.STAGE_FOURIER_ADJOINT, fmap.to(self.map_dtype).contiguous(), out)


def synth(alm, theta, phi, lmax, spin, epsilon, precision="auto"):
    """One-shot synthesis (builds and drops a plan)."""
    p = Plan(theta, phi, lmax, spin, epsilon, precision)
    try:
        return p.synth(alm)
    finally:
        p.close()


def adjoint(fmap, theta, phi, lmax, spin, epsilon, precision="auto"):
    """One-shot adjoint synthesis (builds and drops a plan)."""
    p = Plan(theta, phi, lmax, spin, epsilon, precision)
    try:
        return p.adjoint(fmap)
    finally:
        p.close()


def plan_geometry(lmax: int, spin: int, theta_star: float, epsilon: float, precision: str = "auto",
                  full_sky: bool = False, window: str = "es", cl=None, lmax_rule: str = "band", rings: bool = True):
    """Host-only plan parameters for a cap of radius theta_star: (info, ring_theta, ring_w, ring_mmax);
    with rings=False only info (no per-ring polar cut-offs, which take the longest)."""
    lib = _lib.load()
    info = _lib.PlanInfo()
    opts, _keep = _options(full_sky, window, cl, lmax_rule)
    _lib.check(lib.psht_plan_geometry_ex(lmax, spin, theta_star, epsilon, _lib.PREC[precision], ctypes.byref(opts),
                                         ctypes.byref(info), None, None, None, 0))
    if not rings:
        return info.as_dict(), None, None, None
    n = info.Lmax + 1
    th = np.zeros(n)
    w = np.zeros(n)
    mm = np.zeros(n, dtype=np.int32)
    dp = ctypes.POINTER(ctypes.c_double)
    _lib.check(lib.psht_plan_geometry_ex(lmax, spin, theta_star, epsilon, _lib.PREC[precision], ctypes.byref(opts),
                                         ctypes.byref(info), th.ctypes.data_as(dp), w.ctypes.data_as(dp),
                                         mm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n))
    return info.as_dict(), th, w, mm


def legendre_column(lmax: int, spin: int, m: int, theta: float):
    """lambda+_l and lambda-_l (l = 0..lmax) by the kernels' own seeds/tables, on the host."""
    lp = np.zeros(lmax + 1)
    lm = np.zeros(lmax + 1)
    dp = ctypes.POINTER(ctypes.c_double)
    _lib.check(_lib.load().psht_legendre_column(lmax, spin, m, theta, lp.ctypes.data_as(dp), lm.ctypes.data_as(dp)))
    return lp, lm


def fft(x: torch.Tensor, sign: int) -> torch.Tensor:
    """Batched unnormalized FFT along the last axis with the library's LDS FFT kernel."""
    fp32 = x.dtype == torch.complex64
    x = x.contiguous()
    out = torch.empty_like(x)
    n = x.shape[-1]
    batch = x.numel() // n if n else 0
    _lib.check(_lib.load().psht_fft(n, batch, sign, 1 if fp32 else 0, x.data_ptr(), out.data_ptr(),
                                    _stream()))
    return out


def great_circle_spectrum(lmax: int, spin: int, cl) -> np.ndarray:
    """c_m, m = -lmax..lmax (index m + lmax), of an isotropic spin-`spin` field with power spectrum cl[0..lmax]."""
    c = np.ascontiguousarray(cl, dtype=np.float64)
    if c.ndim != 1 or c.shape[0] < lmax + 1:
        raise ValueError("cl must hold C_l for l = 0..lmax")
    out = np.zeros(2 * lmax + 1)
    dp = ctypes.POINTER(ctypes.c_double)
    _lib.check(_lib.load().psht_great_circle_spectrum(lmax, spin, c.ctypes.data_as(dp), out.ctypes.data_as(dp)))
    return out
