"""torch.autograd wrappers of the ISAM operator (Sec. 2.1, eq. (2)-(3), (7)).

For a real loss L of a complex image x, PyTorch's gradient is
dL/dRe(x) + j dL/dIm(x); since Phi is real-linear, that gradient through
y = Phi x is Phi^H (dL/dy) with the adjoint taken under <a,b> = Re(a^H b) --
exactly what oct_adjoint computes.  Both functions run entirely in liboct.
"""
from __future__ import annotations

import torch

from . import Plan


class OCTPhi(torch.autograd.Function):
    """y = Phi x; backward: grad_x = Phi^H grad_y (the hand-written adjoint)."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        return plan.forward(x.contiguous())

    @staticmethod
    def backward(ctx, gy: torch.Tensor):
        gx = ctx.plan.adjoint(gy.contiguous().to(torch.float32))
        return gx, None


class OCTDataLoss(torch.autograd.Function):
    """D(x; y) = 1/2 ||diag(s)(Phi x - y)||^2 (eq. (2)) with its gradient
    Phi^H (Phi x - y) (eq. (3)) from one fused oct_grad call; the loss is
    accumulated in FP64 and returned as a float64 scalar."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, y: torch.Tensor, plan: Plan) -> torch.Tensor:
        g, half = plan.grad(x.contiguous(), y.contiguous())
        ctx.save_for_backward(g)
        return half

    @staticmethod
    def backward(ctx, gout: torch.Tensor):
        (g,) = ctx.saved_tensors
        return g * gout.to(torch.float32), None, None


def phi(x: torch.Tensor, plan: Plan) -> torch.Tensor:
    return OCTPhi.apply(x, plan)


def data_loss(x: torch.Tensor, y: torch.Tensor, plan: Plan) -> torch.Tensor:
    return OCTDataLoss.apply(x, y, plan)


__all__ = ["OCTPhi", "OCTDataLoss", "phi", "data_loss"]
