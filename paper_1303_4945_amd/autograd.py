"""Differentiable synthesis: alm2map (and the first-derivative maps of
Sect. 4.3) as torch.autograd.Functions.

The backward pass is the library's adjoint synthesis Y^T (Sect. 4.5 of the
paper: analysis with unit weights), with the real-field factor fac_m
(1 for m = 0, 2 for m > 0) applied in the same kernel, so that for a real
loss L the gradient tensor holds dL/dRe(a_lm) and dL/dIm(a_lm) in the
(re, im) slots of the stored coefficients.  For a plan in real spherical
harmonics storage the backward is the plain transpose (dL/dr in every slot).
"""
from __future__ import annotations

import torch


class AlmToMap(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alm: torch.Tensor, plan) -> torch.Tensor:
        ctx.plan = plan
        return plan.alm2map(alm)

    @staticmethod
    def backward(ctx, grad_map: torch.Tensor):
        return ctx.plan.alm2map_grad(grad_map.contiguous()), None


def alm2map(alm: torch.Tensor, plan) -> torch.Tensor:
    """Differentiable synthesis of float64 coefficients [ntrans][ncomp][nalm][2]."""
    return AlmToMap.apply(alm, plan)


class AlmToDeriv1(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alm: torch.Tensor, plan) -> torch.Tensor:
        ctx.plan = plan
        return plan.alm2map_deriv1(alm)

    @staticmethod
    def backward(ctx, grad_map: torch.Tensor):
        return ctx.plan.alm2map_deriv1_grad(grad_map.contiguous()), None


def alm2map_deriv1(alm: torch.Tensor, plan) -> torch.Tensor:
    """Differentiable maps of df/dtheta and df/(sin theta dphi) from spin-0
    coefficients [ntrans][1][nalm][2] (plan of spin 1)."""
    return AlmToDeriv1.apply(alm, plan)
