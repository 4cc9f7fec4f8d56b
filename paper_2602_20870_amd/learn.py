"""Learnable-order pipelines on top of the differentiable FGFRFT (Proposition 4).

* ``OrderCascade``: K layers Q_L^{alpha_K} ... Q_L^{alpha_1} X with one learnable order per
  layer (the cascaded-network experiment of Sec. IV, learning setup).
* ``FractionalMaskDenoiser``: Q_L^{-alpha} diag(h) Q_L^{alpha} y with a learnable order and a
  learnable diagonal mask h in the fractional domain (the denoising model of Sec. IV).

Every forward and backward step runs through the library (update + apply on the GPU, gradient
through ``fgfrft_grad``); torch only holds the parameters and the optimizer state.
"""
from __future__ import annotations

import torch

from .autograd import fgfrft
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
        Z = fgfrft(y.contiguous(), self.alpha, self.plan)[0]
        W = (self.h * Z).contiguous()
        return fgfrft(W, -self.alpha, self.plan)[0]


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
