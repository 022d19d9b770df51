"""Adjoint gradient of J = 0.5 |u - u_t|_2^2 where A-bar(theta) u = M_cut f.

With kappa_e = exp(theta_e), A-bar = sum_e kappa_e h Khat_e (Khat_e the
kept-point stiffness at kappa = 1, h = 1, Sect. 2.2), so
dA-bar/dtheta_e = kappa_e h Khat_e and, with lambda = A-bar^{-1}(u - u_t)
(A-bar is symmetric),
  dJ/dtheta_e = -kappa_e h lambda_e^T Khat_e u_e,    dJ/df = M_cut^T lambda.
"""
from __future__ import annotations

import numpy as np


def gradients(d, u, lam):
    """Per-cell dJ/dtheta (float64[n^3], zero on inactive cells) and per-node
    dJ/df (float64[(n+1)^3])."""
    ld = d.dof_of_node[d.nodes]
    ue = np.where(ld >= 0, u[np.maximum(ld, 0)], 0.0)
    le = np.where(ld >= 0, lam[np.maximum(ld, 0)], 0.0)
    Ku = np.einsum("cab,cb->ca", d.Kunit, ue)
    g_active = -d.kappa[d.active] * d.h * np.einsum("ca,ca->c", le, Ku)
    dtheta = np.zeros(d.n ** 3)
    dtheta[d.active] = g_active
    df = d.Mcut.T @ lam
    return dtheta, df
