"""Differentiable cut-cell solve: u = A-bar(theta)^{-1} M_cut f.

Per-cell conductivity kappa_e = exp(theta_e).  The forward pass runs the
library's setup, factorisation and BDDC-PCG solve; the backward pass reuses
the same factorisation for the adjoint solve lambda = A-bar^{-1} (dJ/du)
(A-bar is symmetric) and contracts it per element in the library:
  dJ/dtheta_e = -kappa_e h lambda_e^T Khat_e u_e,   dJ/df = M_cut^T lambda.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np
import torch

from .cutbddc import Solver


class CutCellSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, f, problem, rtol, max_iter):
        kappa = np.exp(theta.detach().double().cpu().numpy())
        s = Solver(replace(problem, kappa=kappa))
        s.factor()
        u, it, rel = s.solve(f.detach(), rtol=rtol, max_iter=max_iter)
        ctx.solver = s
        ctx.rtol = rtol
        ctx.max_iter = max_iter
        ctx.iterations = it
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        (u,) = ctx.saved_tensors
        s = ctx.solver
        lam, it, rel = s.solve_rhs(grad_u.contiguous(), rtol=ctx.rtol, max_iter=ctx.max_iter)
        dtheta, df = s.grad(u, lam)
        ctx.solver = None
        return dtheta, df, None, None, None


def solve(theta, f, problem, rtol=1e-8, max_iter=1000):
    """u [n_dof] on the GPU for per-cell log-conductivity theta [N^3] and
    nodal source f [(N+1)^3] (both cuda float64 tensors)."""
    return CutCellSolve.apply(theta, f, problem, rtol, max_iter)
