"""Autograd form of the partial-sky transforms.

`SynthFn.apply(alm, plan)` is synthesis general (eq. syn) as a differentiable
torch operation; its backward is the adjoint synthesis of Sec. I with the
outputs of every order m >= 1 doubled (`psht_adjoint_grad`), because the
map is a real-linear function of (Re, Im) of each coefficient and the
reality condition makes every m >= 1 coefficient stand for the pair (m, -m).
`AdjointFn.apply(map, plan)` is the adjoint synthesis; its backward is a
synthesis with the m >= 1 gradient entries halved (`psht_synth_grad`).

Gradients follow torch's convention for complex tensors of a real loss,
dL/dRe z + i dL/dIm z.  Both directions run the library's kernels; nothing
here does arithmetic on the data.
"""
from __future__ import annotations

import torch

from .plan import Plan


class SynthFn(torch.autograd.Function):
    """alm (2, nalm) or (nmaps, 2, nalm) complex128 -> map of the plan's dtype."""

    @staticmethod
    def forward(ctx, alm: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        return plan.synth(alm.detach())

    @staticmethod
    def backward(ctx, gmap: torch.Tensor):
        plan = ctx.plan
        g = gmap.to(plan.map_dtype).contiguous()
        return plan.adjoint_grad(g), None


class AdjointFn(torch.autograd.Function):
    """map (npoints,) or (nmaps, npoints) -> alm (.., 2, nalm) complex128."""

    @staticmethod
    def forward(ctx, fmap: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        return plan.adjoint(fmap.detach())

    @staticmethod
    def backward(ctx, galm: torch.Tensor):
        plan = ctx.plan
        return plan.synth_grad(galm.to(torch.complex128).contiguous()), None


def synth(alm: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable synthesis of `alm` on `plan`."""
    return SynthFn.apply(alm, plan)


def adjoint(fmap: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable adjoint synthesis of `fmap` on `plan`."""
    return AdjointFn.apply(fmap, plan)
