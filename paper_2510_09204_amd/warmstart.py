"""Learned warm start of the SF, trained through the hand-written adjoint.

The paper ("Learned Initialization for Fixed-Point Iteration", eq. NN_loss)
trains a network that maps the flow sample xi and the context (start/goal
pairs, obstacles) to the warm start (xi_bar^0, lambda^0), by unrolling L
applications of T and minimising

    sum_{l<L} L_FP^l + ||xi_bar^L - xi||^2,

L_FP^l = ||z^{l+1} - z^l||^2, z = (xi_bar, lambda) (eq. fixed_point_residual
with the reading that the printed form compares z^{l+1} with T(z^l), which is
identically 0).  No ground-truth solution is needed.  The gradient of both
terms w.r.t. (xi_bar^0, lambda^0) comes from sf_project_backward (the first
through its fixed-point weight), so the SF's forward and reverse passes run
in the library's kernels; the network itself is ordinary torch.

The paper's network is a pair of CNN encoders and a small transformer; this
module is a lighter permutation-invariant stand-in with the same inputs and
outputs: a per-robot MLP over the robot's sample coefficients and its
start/goal, with mean-pooled robot and obstacle embeddings as context.  Its
outputs are a correction of the sample (xi_bar^0 = xi + delta) and lambda^0.
"""
from __future__ import annotations

from typing import Optional

import torch
from torch import nn

from .binding import SFPlan, SFProject


class WarmStartNet(nn.Module):
    """Per-robot warm start for problems of n robots and M obstacles with
    n_coef Bernstein coefficients per axis (one context shape per batch)."""

    def __init__(self, n_coef: int, hidden: int = 128):
        super().__init__()
        self.n_coef = n_coef
        d_in = 2 * n_coef + 4                      # sample (x, y) + start + goal
        self.robot = nn.Sequential(nn.Linear(d_in, hidden), nn.SiLU(),
                                   nn.Linear(hidden, hidden), nn.SiLU())
        self.obstacle = nn.Sequential(nn.Linear(3, hidden), nn.SiLU(),
                                      nn.Linear(hidden, hidden), nn.SiLU())
        self.head = nn.Sequential(nn.Linear(3 * hidden, hidden), nn.SiLU(),
                                  nn.Linear(hidden, 4 * n_coef))
        nn.init.zeros_(self.head[-1].weight)       # start from xi_bar^0 = xi, lambda^0 = 0
        nn.init.zeros_(self.head[-1].bias)

    def forward(self, xi: torch.Tensor, boundary: torch.Tensor,
                obstacles: Optional[torch.Tensor]):
        """xi [B][2][n][nc], boundary [B][n][2][2], obstacles [B][M][3] or None
        -> (xi_bar^0, lambda^0), both [B][2][n][nc]."""
        B, _, n, nc = xi.shape
        feats = torch.cat([xi.permute(0, 2, 1, 3).reshape(B, n, 2 * nc),
                           boundary.reshape(B, n, 4)], dim=-1)
        h = self.robot(feats)                                     # [B][n][H]
        ctx_r = h.mean(dim=1, keepdim=True).expand(-1, n, -1)
        if obstacles is not None and obstacles.shape[1] > 0:
            ctx_o = self.obstacle(obstacles).mean(dim=1, keepdim=True).expand(-1, n, -1)
        else:
            ctx_o = torch.zeros_like(h)
        out = self.head(torch.cat([h, ctx_r, ctx_o], dim=-1))     # [B][n][4 nc]
        out = out.reshape(B, n, 2, 2, nc).permute(2, 0, 3, 1, 4)  # [2][B][axis][n][nc]
        return xi + out[0], out[1]


def warm_start_loss(net: WarmStartNet, plan: SFPlan, xi: torch.Tensor,
                    boundary: torch.Tensor, obstacles: Optional[torch.Tensor], n_iters: int,
                    fp_weight: float = 1.0):
    """The training objective of eq. NN_loss for a batch of equal-shape
    problems (the plan's).  xi [B][2][n][nc]; boundary [B][n][2][2];
    obstacles [B][M][3] or None.  Returns (loss_without_fp, xi_bar^L,
    lambda^L, residual): the returned loss holds ||xi_bar^L - xi||^2 (summed
    over the batch); its backward also carries fp_weight * sum_l L_FP^l (the
    fixed-point terms enter through sf_project_backward)."""
    xi0, lam0 = net(xi, boundary, obstacles)
    flat = lambda t: t.reshape(-1).contiguous()
    obs = None if obstacles is None or obstacles.numel() == 0 else flat(obstacles)
    xo, lo, res = SFProject.apply(flat(xi), flat(xi0), flat(lam0), flat(boundary), obs, plan,
                                  n_iters, fp_weight)
    loss = ((xo - flat(xi)) ** 2).sum()
    return loss, xo, lo, res


__all__ = ["WarmStartNet", "warm_start_loss"]
