"""Partial-sky spin-weighted spherical harmonic transforms on MI355X (gfx950).

Synthesis of (g_lm, c_lm) at arbitrary points clustered in one sky patch and
its exact adjoint, through rings inside the stretched, apodized polar cap,
FFTs and an exponential-of-semicircle NUFFT (Carron & Reinecke, Sec. II).
The compute path is the HIP library ``libpsht.so`` behind the C ABI in
``include/psht.h``; this package is its thin Python binding.
"""
__all__ = ["Plan", "SynthFn", "AdjointFn", "synth", "adjoint"]


def __getattr__(name):
    if name in ("Plan", "synth", "adjoint"):
        from . import plan as _plan
        return getattr(_plan, name)
    if name in ("SynthFn", "AdjointFn"):
        from . import autograd as _ag
        return getattr(_ag, name)
    raise AttributeError(name)
