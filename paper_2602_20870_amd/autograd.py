"""Differentiable FGFRFT (Proposition 4): Y[a] = Q_L^{alpha_a} X[a] as a torch
autograd Function whose backward is the library's hand-written gradient.

Convention: for complex outputs torch passes grad_output = dl/dRe Y + j dl/dIm Y,
which is exactly the GY the C ABI expects; the order gradient is returned as
float64 on the device of alpha, the signal gradient in the dtype of X (its real
part when X is real).
"""
from __future__ import annotations

import torch

from .ops import Plan


class FGFRFTFunction(torch.autograd.Function):
    """Y = FGFRFTFunction.apply(X, alpha, plan).

    X: float32 or complex64 cuda tensor [n, N, B] (one block per order) or [N, B]
    (one block shared by every order); alpha: float64 tensor [n] (any device).
    """

    @staticmethod
    def forward(ctx, X: torch.Tensor, alpha: torch.Tensor, plan: Plan) -> torch.Tensor:
        a = alpha.detach().to("cpu", torch.float64).reshape(-1)
        Xc = X.detach().contiguous()
        Y = plan.apply(a.numpy(), Xc)
        ctx.plan = plan
        ctx.save_for_backward(Xc, alpha)
        return Y

    @staticmethod
    def backward(ctx, GY: torch.Tensor):
        X, alpha = ctx.saved_tensors
        plan: Plan = ctx.plan
        a = alpha.detach().to("cpu", torch.float64).reshape(-1).numpy()
        gy = GY.to(torch.complex64).contiguous()
        want_dx = ctx.needs_input_grad[0]
        dal, dX = plan.grad(a, X, gy, want_dX=want_dx)
        d_alpha = torch.from_numpy(dal).to(device=alpha.device, dtype=alpha.dtype).reshape(alpha.shape)
        return (dX if want_dx else None), (d_alpha if ctx.needs_input_grad[1] else None), None


def fgfrft(X: torch.Tensor, alpha: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable Y[a] = Q_L^{alpha_a} X[a]."""
    return FGFRFTFunction.apply(X, alpha, plan)
