"""Preconditioned conjugate gradients (paper Sect. 2.2: CG applies since
A-bar is SPD; Sect. 5.1: convergence when |r|_2 < tol |b|_2 with r = b - A x).

Reading taken: x_0 = 0, the recursively updated residual is tested after
each update, and the returned count is the number of operator applies.
b = 0 returns x = 0 after 0 iterations.
"""
from __future__ import annotations

import numpy as np


def pcg(apply_A, apply_M, b, rtol=1e-8, max_iter=1000):
    """Returns (x, iterations, relative residual |r|/|b|, alphas, betas)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = np.linalg.norm(b)
    alphas, betas = [], []
    if bnorm == 0.0:
        return x, 0, 0.0, alphas, betas
    r = b.copy()
    z = apply_M(r)
    p = z.copy()
    rho = r @ z
    k = 0
    relres = 1.0
    while k < max_iter:
        q = apply_A(p)
        alpha = rho / (p @ q)
        x += alpha * p
        r -= alpha * q
        k += 1
        alphas.append(alpha)
        relres = np.linalg.norm(r) / bnorm
        if relres < rtol:
            break
        z = apply_M(r)
        rho_new = r @ z
        beta = rho_new / rho
        betas.append(beta)
        rho = rho_new
        p = z + beta * p
    return x, k, relres, alphas, betas


def lanczos_condition(alphas, betas):
    """Extreme eigenvalue estimates of M A from the CG coefficients (the
    Lanczos tridiagonal matrix): returns (lambda_min, lambda_max)."""
    k = len(alphas)
    if k == 0:
        return 1.0, 1.0
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = 1.0 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i > 0 else 0.0)
        if i + 1 < k and i < len(betas):
            T[i, i + 1] = T[i + 1, i] = np.sqrt(betas[i]) / alphas[i]
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])
