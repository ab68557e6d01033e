"""torch.autograd.Function wrappers of the library's operators.

The gradient of a loss through g = A f is A^T (dL/dg), where A^T is the
Euclidean transpose of the discrete forward operator.  The library computes
the weighted adjoint A* = s A^T of the L2 inner products of the paper's
eq. eqn:innerProducts (Hauptmann, Kunyansky & Poimala, arXiv 2510.24687,
Sec. 2.1), so A^T = A*/s with s = Plan.adjoint_scale.  The data-fidelity
gradient of eq. E:operators, grad ||A f - g||^2 = 2 A^T (A f - g), follows by
autograd.  Every application runs the HIP kernels; nothing here computes.
"""
from __future__ import annotations

import torch

from .pat import Plan


# Each backward applies the opposite operator through its own Function, so the
# backward pass is itself differentiable: under create_graph=True the second
# derivative of a loss through A is built from A and A^T again (the operators
# are linear, so that is exact), not silently zero.
class _Forward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, plan):
        ctx.plan = plan
        return plan.forward(f.contiguous())

    @staticmethod
    def backward(ctx, grad_g):
        return _Transpose.apply(grad_g, ctx.plan), None


class _Transpose(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g, plan):
        ctx.plan = plan
        return plan.transpose(g.contiguous())

    @staticmethod
    def backward(ctx, grad_f):
        return _Forward.apply(grad_f, ctx.plan), None


class _ScaledForward(torch.autograd.Function):
    """s A f with s the plan's adjoint scale (the transpose of A* = s A^T)."""

    @staticmethod
    def forward(ctx, f, plan):
        ctx.plan = plan
        out = plan.forward(f.contiguous())
        return plan.scale_(out, plan.adjoint_scale)

    @staticmethod
    def backward(ctx, grad_g):
        return _Adjoint.apply(grad_g, ctx.plan), None


class _Adjoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g, plan):
        ctx.plan = plan
        return plan.adjoint(g.contiguous())

    @staticmethod
    def backward(ctx, grad_f):
        return _ScaledForward.apply(grad_f, ctx.plan), None


def forward(f: torch.Tensor, plan: Plan) -> torch.Tensor:
    """g = A f, differentiable (backward A^T)."""
    return _Forward.apply(f, plan)


def transpose(g: torch.Tensor, plan: Plan) -> torch.Tensor:
    """f = A^T g, differentiable (backward A)."""
    return _Transpose.apply(g, plan)


def adjoint(g: torch.Tensor, plan: Plan) -> torch.Tensor:
    """f = A* g (weighted adjoint), differentiable (backward s A)."""
    return _Adjoint.apply(g, plan)


class PATOperator(torch.nn.Module):
    """The forward operator as a module: ``op(f)`` = A f, ``op.T(g)`` = A^T g,
    ``op.adjoint(g)`` = A* g; all differentiable."""

    def __init__(self, geom: dict, dtype=torch.float32, max_batch: int = 1, device=None):
        super().__init__()
        self.plan = Plan(geom, dtype, max_batch=max_batch, device=device)

    def forward(self, f):
        return forward(f, self.plan)

    def T(self, g):
        return transpose(g, self.plan)

    def adjoint(self, g):
        return adjoint(g, self.plan)
