"""Fitting goals and rationality from observed tracks through the
differentiable trajectory log-likelihood (the product form of Eq. beta_update
over each track, with the hand-written adjoint behind capred.LogLik).

The objective is the marginal log-likelihood of the tracks under a uniform
prior over the candidate goals (and over the beta grid when log_beta is a
shared grid):

    J = sum_n log (1 / (G B)) sum_{b, g} exp(LL[n, b, g]),

maximised with Adam over the continuous goal positions and log beta.  With
per-track log beta ([N, 1]) each track gets its own rationality, jointly with
the G shared goals.  Everything but the optimiser's few elementwise updates
runs in the library's kernels (forward: the batched log-likelihood; backward:
its adjoint, with fixed-order FP64 reductions).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import torch

from . import capred


@dataclasses.dataclass
class FitResult:
    goals: torch.Tensor          # [G, 2] FP32, fitted
    log_beta: torch.Tensor       # like log_beta0, fitted
    objective: List[float]       # J / N before each step


def marginal_loglik(LL: torch.Tensor) -> torch.Tensor:
    """sum_n log mean_{b,g} exp(LL[n, b, g]) (FP64)."""
    N, B, G = LL.shape
    return (torch.logsumexp(LL.reshape(N, B * G), dim=1) - math.log(B * G)).sum()


def fit_goals_beta(K: int, speed: float, dt: float, tracks: torch.Tensor,
                   lengths: torch.Tensor, goals0: torch.Tensor, log_beta0: torch.Tensor,
                   iters: int = 300, lr: float = 0.02) -> FitResult:
    """Adam ascent of the marginal log-likelihood J / N from (goals0, log_beta0).
    tracks [N, T+1, 2] FP32 and lengths [N] int32 on the GPU; goals0 [G, 2]
    FP32; log_beta0 [B] (shared grid) or [N, B] (per track) FP32."""
    g = goals0.detach().clone().float().contiguous().requires_grad_(True)
    b = log_beta0.detach().clone().float().contiguous().requires_grad_(True)
    opt = torch.optim.Adam([g, b], lr=lr)
    n = tracks.shape[0]
    hist = []
    for _ in range(iters):
        opt.zero_grad()
        LL = capred.LogLik.apply(g, b, tracks, lengths, K, speed, dt)
        J = marginal_loglik(LL) / n
        (-J).backward()
        hist.append(J.detach())
        opt.step()
    return FitResult(g.detach(), b.detach(), [float(x) for x in torch.stack(hist).cpu()])
