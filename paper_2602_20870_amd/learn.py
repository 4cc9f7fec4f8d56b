"""Learnable-order pipelines on top of the differentiable FGFRFT (Proposition 4).

* ``OrderCascade``: K layers Q_L^{alpha_K} ... Q_L^{alpha_1} X with one learnable order per
  layer (the cascaded-network experiment of Sec. IV, learning setup).
* ``FractionalMaskDenoiser``: Q_L^{-alpha} diag(h) Q_L^{alpha} y with a learnable order and a
  learnable diagonal mask h in the fractional domain (the denoising model of Sec. IV).
* ``PointCloudDenoiser``: the same mask pipeline with one learnable order and mask per channel
  between a linear lift of the point coordinates to C channels and a projection back.

Every forward and backward step runs through the library (update + apply on the GPU, gradient
through ``fgfrft_grad``); torch only holds the parameters and the optimizer state.
"""
from __future__ import annotations

import torch

from .autograd import fgfrft, fractional_filter
from .ops import Plan


class OrderCascade(torch.nn.Module):
    """Y = Q^{alpha_K} ... Q^{alpha_1} X for X [N, B] (real or complex); returns complex64 [N, B]."""

    def __init__(self, plan: Plan, K: int, alpha_init: float = 0.1):
        super().__init__()
        self.plan = plan
        self.alpha = torch.nn.Parameter(torch.full((K,), float(alpha_init), dtype=torch.float64))

    def total_order(self) -> float:
        return float(self.alpha.detach().sum())

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        Y = X
        for l in range(self.alpha.numel()):
            Y = fgfrft(Y.contiguous(), self.alpha[l:l + 1], self.plan)[0]
        return Y


class FractionalMaskDenoiser(torch.nn.Module):
    """x_hat = Q^{-alpha} diag(h) Q^{alpha} y for real signals y [N, B]; returns complex64 [N, B]."""

    def __init__(self, plan: Plan, alpha_init: float = 0.5):
        super().__init__()
        self.plan = plan
        self.alpha = torch.nn.Parameter(torch.tensor([float(alpha_init)], dtype=torch.float64))
        self.h = torch.nn.Parameter(torch.ones(plan.N, 1, dtype=torch.float32, device=plan.device))

    def forward(self, y: torch.Tensor) -> torch.Tensor:
        return fractional_filter(y.contiguous(), self.alpha, self.h, self.plan)[0]


class PointCloudDenoiser(torch.nn.Module):
    """Y_hat = proj(Re Q^{-alpha_c} diag(h_c) Q^{alpha_c} lift(Y)_c) for noisy point coordinates
    Y [clouds, N, c_in] (float32, on the plan's device): a c_in -> C linear lift, per channel c a
    learnable order alpha_c and mask h_c in the fractional domain, and a C -> c_in projection of the
    real part.  Channel c takes the clouds as its signals, so each transform is one library call for
    all C orders with `clouds` signals per order, forward and backward."""

    def __init__(self, plan: Plan, channels: int = 64, c_in: int = 3, alpha_init: float = 0.5, seed: int = 0):
        super().__init__()
        g = torch.Generator().manual_seed(seed)
        dev = plan.device
        self.plan = plan
        self.W_in = torch.nn.Parameter((torch.randn(c_in, channels, generator=g) / c_in ** 0.5).to(dev))
        self.W_out = torch.nn.Parameter((torch.randn(channels, c_in, generator=g) / channels ** 0.5).to(dev))
        spread = torch.linspace(0.5, 1.5, channels, dtype=torch.float64)
        self.alpha = torch.nn.Parameter(float(alpha_init) * spread)
        self.h = torch.nn.Parameter(torch.ones(channels, plan.N, 1, dtype=torch.float32, device=dev))

    def forward(self, Y: torch.Tensor) -> torch.Tensor:
        # The lift and the projection contract over 3 or C values per (point, cloud); written as
        # broadcast multiply-adds in the filter's [C, N, clouds] layout their weight gradients are
        # plain reductions, not GEMMs with a contraction over all N x clouds positions and a 3 x C
        # result (which the BLAS library runs with little parallelism).
        Yt = Y.permute(2, 1, 0)                                            # [c_in, N, clouds]
        X = self.W_in[0][:, None, None] * Yt[0]
        for d in range(1, Yt.shape[0]):
            X = X + self.W_in[d][:, None, None] * Yt[d]
        Zi = fractional_filter(X.contiguous(), self.alpha, self.h, self.plan)   # [C, N, clouds]
        Zr = Zi.real
        out = torch.stack([(Zr * self.W_out[:, e][:, None, None]).sum(0) for e in range(self.W_out.shape[1])],
                          dim=-1)                                          # [N, clouds, c_in]
        return out.permute(1, 0, 2)                                        # [clouds, N, c_in]


def train(model: torch.nn.Module, loss_fn, steps: int, lr: float = 0.01, params=None) -> list[float]:
    """Adam on the model's parameters (orders live on the host, masks on the device)."""
    opt = torch.optim.Adam(model.parameters() if params is None else params, lr=lr)
    hist = []
    for _ in range(steps):
        opt.zero_grad()
        loss = loss_fn(model)
        loss.backward()
        opt.step()
        hist.append(float(loss.detach()))
    return hist
