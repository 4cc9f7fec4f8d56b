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


class FractionalFilterFunction(torch.autograd.Function):
    """Y = FractionalFilterFunction.apply(X, alpha, h, plan): per order a,
    Y[a] = Q^{-alpha_a} diag(h[a]) Q^{alpha_a} X[a], a filter h in the fractional domain.

    The operator Q^{a} is formed once in the forward pass and kept for the backward one; since
    Q^{-a} = (Q^{a})^H (Proposition 3) every product with Q^{-a} is an adjoint apply of Q^{a}, so no
    second operator is formed:
      Y = (Q^{a})^H M,  GM = Q^{a} GY,  dh = Re sum_b conj(GM) Z,  GZ = h GM,  dX = (Q^{a})^H GZ,
      dalpha = Re<GZ X^H, dQ/da (a)> - Re<GY M^H, dQ/da (-a)>   (Proposition 4), with Z = Q^{a} X
    and M = h Z.  Differentiating Q^{-a} = (Q^{a})^H gives dQ/da (-a) = -(dQ/da (a))^H, so the second
    term is Re<M GY^H, dQ/da (a)> and dalpha is one order gradient at a (the library's, without its
    signal part) of the outer product [GZ | M] [X | GY]^H over the two signal blocks side by side.
    X: float32 or complex64 [n, N, B] or shared [N, B]; h: float32, broadcastable to [n, N, B]
    (e.g. [n, N, 1] or [N, 1]); returns complex64 [n, N, B].
    """

    @staticmethod
    def forward(ctx, X: torch.Tensor, alpha: torch.Tensor, h: torch.Tensor, plan: Plan) -> torch.Tensor:
        from .ops import apply_operator
        a = alpha.detach().to("cpu", torch.float64).reshape(-1).numpy()
        Xc = X.detach().contiguous()
        Qp = plan.update(a)
        Z = apply_operator(Qp, Xc)
        M = (h.detach() * Z).contiguous()
        Y = apply_operator(Qp, M, adjoint=True)     # Q^{-a} M
        ctx.plan = plan
        ctx.save_for_backward(Xc, alpha, h, Qp, Z, M)
        return Y

    @staticmethod
    def backward(ctx, GY: torch.Tensor):
        from .ops import apply_operator
        X, alpha, h, Qp, Z, M = ctx.saved_tensors
        plan: Plan = ctx.plan
        a = alpha.detach().to("cpu", torch.float64).reshape(-1).numpy()
        gy = GY.to(torch.complex64).contiguous()
        GM = apply_operator(Qp, gy)
        GZ = (h.detach() * GM).contiguous()
        dX = dh = d_alpha = None
        if ctx.needs_input_grad[0]:
            gx = apply_operator(Qp, GZ, adjoint=True)   # Q^{-a} GZ
            if not X.is_complex():
                gx = gx.real
            dX = gx.sum(dim=0) if X.dim() == 2 else gx
        if ctx.needs_input_grad[2]:
            dh = (GM.conj() * Z).real.sum_to_size(h.shape)
        if ctx.needs_input_grad[1]:
            n = a.size
            Xb = X.to(torch.complex64)
            if Xb.dim() == 2:
                Xb = Xb.expand(n, *Xb.shape)
            Xcat = torch.cat([Xb, gy], dim=-1).contiguous()       # [X | GY]
            Gcat = torch.cat([GZ, M], dim=-1).contiguous()        # [GZ | M]
            g, _ = plan.grad(a, Xcat, Gcat, want_dX=False)
            d_alpha = torch.from_numpy(g).to(device=alpha.device, dtype=alpha.dtype).reshape(alpha.shape)
        return dX, d_alpha, dh, None


def fractional_filter(X: torch.Tensor, alpha: torch.Tensor, h: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable Y[a] = Q_L^{-alpha_a} diag(h[a]) Q_L^{alpha_a} X[a]."""
    return FractionalFilterFunction.apply(X, alpha, h, plan)
