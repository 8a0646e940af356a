"""Autograd over the transform.

Decomposition and recomposition are linear maps, so the backward pass of
each is its transpose: D^T for decompose, R^T for recompose.  Both run in the
library's adjoint kernels (level by level in reverse order).
"""
from __future__ import annotations

import torch


class DecomposeFn(torch.autograd.Function):
    """coeff = D(x); backward: grad_x = D^T(grad_coeff)."""

    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return plan.decompose(x.contiguous())

    @staticmethod
    def backward(ctx, gcoeff):
        return ctx.plan.decompose_adjoint(gcoeff.contiguous()), None


class RecomposeFn(torch.autograd.Function):
    """x = R(coeff); backward: grad_coeff = R^T(grad_x)."""

    @staticmethod
    def forward(ctx, coeff, plan):
        ctx.plan = plan
        return plan.recompose(coeff.contiguous())

    @staticmethod
    def backward(ctx, gx):
        return ctx.plan.recompose_adjoint(gx.contiguous()), None


def decompose(x: torch.Tensor, plan) -> torch.Tensor:
    return DecomposeFn.apply(x, plan)


def recompose(coeff: torch.Tensor, plan) -> torch.Tensor:
    return RecomposeFn.apply(coeff, plan)
