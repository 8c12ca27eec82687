"""ctypes loader for libpsht.so (the C ABI of include/psht.h).

Argument marshalling only.  Loading fails loudly when the library has not
been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsht.so")

PSHT_OK = 0
PSHT_ERR_ARG = 1
PSHT_ERR_NOMEM = 2
PSHT_ERR_DEVICE = 3
PSHT_ERR_UNSUPPORTED = 4
PSHT_ERR_WORKSPACE = 5

PREC = {"auto": 0, "fp32": 1, "fp64": 2}

NOALLOC_SCRATCH_BYTES = 64 << 20  # PSHT_NOALLOC_SCRATCH_BYTES

STAGE_LEGENDRE_SYNTH = 1
STAGE_LEGENDRE_ADJOINT = 2
STAGE_FOURIER_SYNTH = 3
STAGE_FOURIER_ADJOINT = 4

# Every function the header declares; tests check that all are exported.
EXPORTS = (
    "psht_plan_create", "psht_plan_query", "psht_synth", "psht_adjoint", "psht_plan_destroy",
    "psht_last_error", "psht_plan_geometry", "psht_stage", "psht_fft", "psht_legendre_column",
    "psht_plan_set_timing", "psht_plan_timing", "psht_adjoint_grad", "psht_synth_grad", "psht_synth_noalloc",
    "psht_plan_check", "psht_plan_create_ex", "psht_plan_geometry_ex", "psht_great_circle_spectrum",
    "psht_rotate_alm_workspace", "psht_rotate_alm", "psht_rotate_points", "psht_spin_phase", "psht_stage_ex",
)

STAGE_NAMES = ("leg_synth", "theta_synth", "phi_synth", "interp", "grid_zero", "spread", "phi_adj", "theta_adj",
               "alm_zero", "leg_adj")


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("lmax", ctypes.c_int32), ("spin", ctypes.c_int32), ("Lmax", ctypes.c_int32), ("n2", ctypes.c_int32),
        ("mmax", ctypes.c_int32), ("nufft_w", ctypes.c_int32), ("ntheta_grid", ctypes.c_int32),
        ("nphi_grid", ctypes.c_int32), ("row_lo", ctypes.c_int32), ("rows_used", ctypes.c_int32),
        ("map_is_fp32", ctypes.c_int32), ("full_sky", ctypes.c_int32),
        ("epsilon", ctypes.c_double), ("theta_star", ctypes.c_double), ("theta_min", ctypes.c_double),
        ("theta_max", ctypes.c_double), ("eps_apo", ctypes.c_double), ("alpha", ctypes.c_double),
        ("nufft_beta", ctypes.c_double), ("nufft_sigma", ctypes.c_double), ("predicted_speedup", ctypes.c_double),
        ("legendre_triples", ctypes.c_double),
        ("npoints", ctypes.c_int64), ("resident_bytes", ctypes.c_size_t), ("workspace_bytes_per_map", ctypes.c_size_t),
        ("kernel_poly_err", ctypes.c_double),
        ("adj_segment", ctypes.c_int32), ("adj_waves", ctypes.c_int32), ("adj_rings_per_lane", ctypes.c_int32),
        ("adj_states", ctypes.c_int64), ("Lmax_rule", ctypes.c_int32), ("predicted_error", ctypes.c_double),
        ("window", ctypes.c_int32), ("shared_bytes", ctypes.c_size_t),
        ("syn_segment", ctypes.c_int32), ("syn_parts", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


WINDOWS = {"es": 0, "kb": 1, "pswf": 2}
LMAX_RULES = {"band": 0, "cost": 1}


class PlanOptions(ctypes.Structure):
    _fields_ = [("full_sky", ctypes.c_int32), ("window", ctypes.c_int32), ("cl", ctypes.POINTER(ctypes.c_double)),
                ("cl_lmax", ctypes.c_int32), ("lmax_rule", ctypes.c_int32)]


class PshtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("psht error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpsht.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.psht_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int64, vp, vp,
                                     ctypes.c_double, ctypes.c_int, vp]
    lib.psht_plan_create_ex.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int64, vp, vp,
                                        ctypes.c_double, ctypes.c_int, ctypes.POINTER(PlanOptions), vp]
    lib.psht_plan_geometry_ex.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                          ctypes.POINTER(PlanOptions), ctypes.POINTER(PlanInfo), dp, dp, i32p,
                                          ctypes.c_int]
    lib.psht_great_circle_spectrum.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
    lib.psht_plan_query.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.psht_synth.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp]
    lib.psht_adjoint.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp]
    lib.psht_adjoint_grad.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp]
    lib.psht_synth_grad.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp]
    lib.psht_synth_noalloc.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.psht_plan_check.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), vp]
    lib.psht_plan_destroy.argtypes = [vp]
    lib.psht_plan_destroy.restype = None
    d = ctypes.c_double
    lib.psht_stage_ex.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp]
    lib.psht_rotate_alm_workspace.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    lib.psht_rotate_alm.argtypes = [ctypes.c_int, ctypes.c_int, d, d, d, vp, vp, vp, ctypes.c_size_t, vp]
    lib.psht_rotate_points.argtypes = [ctypes.c_int64, d, d, d, vp, vp, vp, vp, vp, vp]
    lib.psht_spin_phase.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    lib.psht_last_error.argtypes = []
    lib.psht_last_error.restype = ctypes.c_char_p
    lib.psht_plan_geometry.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                       ctypes.POINTER(PlanInfo), dp, dp, i32p, ctypes.c_int]
    lib.psht_stage.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.psht_fft.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    lib.psht_legendre_column.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp]
    lib.psht_plan_set_timing.argtypes = [vp, ctypes.c_int]
    lib.psht_plan_timing.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64)]
    for name in ("psht_plan_create", "psht_plan_query", "psht_synth", "psht_adjoint", "psht_plan_geometry",
                 "psht_stage", "psht_fft", "psht_legendre_column", "psht_plan_set_timing", "psht_plan_timing",
                 "psht_adjoint_grad", "psht_synth_grad", "psht_synth_noalloc", "psht_plan_check",
                 "psht_plan_create_ex", "psht_plan_geometry_ex", "psht_great_circle_spectrum",
                 "psht_rotate_alm_workspace", "psht_rotate_alm", "psht_rotate_points", "psht_spin_phase",
                 "psht_stage_ex"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(code: int) -> None:
    if code != PSHT_OK:
        raise PshtError(code, load().psht_last_error().decode())
