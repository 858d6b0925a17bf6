"""Differentiable focus intensities: phase (real tensor) -> I_n = |Theta_n|^2.

Forward runs E = A exp(i phi) and the forward matrix triple product (Eq. 2)
at the foci in the library's kernels.  Backward receives g = dL/dI and runs
the adjoint product with a gradient epilogue in the library:

    dL/dphi = 2 Im( conj(E) * P^H(g * Theta) ).

Intensities are real, so no complex-gradient convention crosses the boundary.
"""
from __future__ import annotations

import itertools

import torch

_tokens = itertools.count(1)


class MTPIntensity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi: torch.Tensor, plan) -> torch.Tensor:
        if not (phi.is_cuda and phi.dtype == torch.float32):
            raise TypeError("phi must be a float32 CUDA tensor")
        if phi.numel() != plan.ny * plan.nx:
            raise ValueError("phi has the wrong number of elements")
        plan.set_phase(phi)
        token = next(_tokens)
        plan._phase_token = token
        _, inten = plan.foci_field_device(intensity=True)
        ctx.plan = plan
        ctx.token = token
        ctx.save_for_backward(phi)
        return inten

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (phi,) = ctx.saved_tensors
        plan = ctx.plan
        if getattr(plan, "_phase_token", None) != ctx.token:
            plan.set_phase(phi)
            plan._phase_token = ctx.token
        grad = plan.phase_gradient_device(g.contiguous())
        return grad.view_as(phi), None


def foci_intensity(phi: torch.Tensor, plan) -> torch.Tensor:
    """I_n(phi) for the plan's pupil and foci, differentiable in phi."""
    return MTPIntensity.apply(phi, plan)
