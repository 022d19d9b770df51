"""Weak Dirichlet condition on the ball surfaces by Nitsche's method (paper
Sect. 2.2: the element form A_e with its surface terms, the coefficient
beta_e >= C_e, eq. local-eigenvals, and the choice beta_e = 2 lambda_max).

TEST INFRASTRUCTURE ONLY (part of the oracle package).

Readings taken (the paper omits its integration section):
  * Surface rule.  Each ball i carries a tensor rule on its sphere:
    n_t Gauss-Legendre nodes t_j in t = cos(theta) in [-1, 1] and n_phi =
    2 n_t midpoint nodes phi_k = 2 pi (k + 1/2) / n_phi, with
    n_t = max(8, ceil(4 pi r / h)) (spacing about h/4 on the sphere).  Point
    x = c + r d, d = (sqrt(1 - t^2) cos(phi), sqrt(1 - t^2) sin(phi), t),
    weight r^2 w_j 2 pi / n_phi.  Over a whole sphere the rule integrates
    polynomials of degree < 2 n_t in t and trigonometric ones of degree
    < n_phi in phi exactly.
  * Gamma_cut of ball i is the part of its sphere inside the open unit
    cube and outside every other ball: a point is kept iff 0 < x_d < 1 for
    every axis and (dx dx + dy dy) + dz dz > r_j^2 for every other ball j
    (the kept-point test of the volume rule).
  * A kept point belongs to the cell floor(x N) (clamped to N - 1) and
    counts only if that cell is cut by the volume rule (0 < kept points <
    512); points in other cells are dropped.
  * The outward normal of Omega on ball i's sphere points into the ball:
    n = -d.
  * In the unit frame of a cell (xi = x N - cell index, weights scaled by
    N^2) the surface matrices are
      S[a, b] = sum w N_a N_b,  T[a, b] = sum w (n . grad N_a) N_b,
      U[a, b] = sum w (n . grad N_a)(n . grad N_b),
    summed over the cell's points in the order (ball, j, k).  With
    D_e = h K_unit (the volume form), B_e = U (the surface form of eq.
    local-eigenvals in physical units), beta_e = 2 lambda_max / h where
    lambda_max is the largest eigenvalue of U x = lambda (K_unit + alpha
    K_ref) x on the complement of the constants (both forms vanish on
    constants), K_ref the unit stiffness of a whole cell and alpha =
    BETA_REG.  The kept-point rule leaves K_unit singular on that
    complement in cells with one or two kept points, where the paper's
    exactly integrated form is not; the shift counts the cell's void part
    with stiffness alpha, as the fictitious domain of the finite cell
    method, and bounds lambda_max there.  It is small enough that the
    coercivity bound x^T A_e x >= x^T K_e x / 2 - alpha x^T K_ref x / 2
    keeps every local matrix positive definite on our workloads (1e-4
    does not).
  * The Nitsche element form with homogeneous Dirichlet data, kappa_e
    times the paper's form, is then kappa_e h (K_unit + 2 lambda_max S - T
    - T^T): the stored unit stiffness of a cut cell becomes
    K_unit + 2 lambda_max S - T - T^T, and the load is unchanged.
"""
from __future__ import annotations

import math

import numpy as np

from .integrate import LOCAL_NODE_OFFSETS

# stiffness of a cut cell's void part in the eigenproblem (relative to a
# whole cell's)
BETA_REG = 1e-6


def sphere_rule(r: float, h: float):
    """(directions (n_t n_phi, 3) in (j, k) order with k fastest, weights
    (n_t n_phi,)) of the tensor rule on the sphere of radius r."""
    nt = max(8, int(math.ceil(4.0 * math.pi * r / h)))
    nphi = 2 * nt
    t, wt = np.polynomial.legendre.leggauss(nt)
    phi = 2.0 * np.pi * (np.arange(nphi) + 0.5) / nphi
    st = np.sqrt(1.0 - t * t)
    d = np.empty((nt, nphi, 3))
    d[:, :, 0] = st[:, None] * np.cos(phi)[None, :]
    d[:, :, 1] = st[:, None] * np.sin(phi)[None, :]
    d[:, :, 2] = t[:, None]
    w = (r * r) * wt[:, None] * (2.0 * np.pi / nphi) * np.ones((1, nphi))
    return d.reshape(-1, 3), w.reshape(-1)


def surface_points(problem):
    """Kept points of Gamma_cut: (cell, x, n, w) arrays over all balls, in
    the order (ball, j, k), before any cell filtering."""
    n = problem.n
    h = 1.0 / n
    C = np.asarray(problem.centres, dtype=np.float64).reshape(-1, 3)
    R = np.asarray(problem.radii, dtype=np.float64)
    cells, xs, ns, ws = [], [], [], []
    for i in range(R.size):
        d, w = sphere_rule(float(R[i]), h)
        x = C[i][None, :] + R[i] * d
        keep = np.all((x > 0.0) & (x < 1.0), axis=1)
        for j in range(R.size):
            if j == i:
                continue
            dx = x[:, 0] - C[j, 0]
            dy = x[:, 1] - C[j, 1]
            dz = x[:, 2] - C[j, 2]
            keep &= (dx * dx + dy * dy) + dz * dz > R[j] * R[j]
        x, d, w = x[keep], d[keep], w[keep]
        ijk = np.minimum(np.floor(x * n).astype(np.int64), n - 1)
        cells.append(ijk[:, 0] + n * (ijk[:, 1] + n * ijk[:, 2]))
        xs.append(x)
        ns.append(-d)
        ws.append(w)
    if not cells:
        z = np.zeros((0, 3))
        return np.zeros(0, np.int64), z, z, np.zeros(0)
    return np.concatenate(cells), np.concatenate(xs), np.concatenate(ns), np.concatenate(ws)


def _shape(xi):
    """N (m, 8) and reference gradients G (m, 8, 3) at unit-cell points."""
    m = xi.shape[0]
    N = np.empty((m, 8))
    G = np.empty((m, 8, 3))
    for a in range(8):
        o = LOCAL_NODE_OFFSETS[a]
        f = [xi[:, d] if o[d] else 1.0 - xi[:, d] for d in range(3)]
        s = [1.0 if o[d] else -1.0 for d in range(3)]
        N[:, a] = f[0] * f[1] * f[2]
        G[:, a, 0] = s[0] * f[1] * f[2]
        G[:, a, 1] = f[0] * s[1] * f[2]
        G[:, a, 2] = f[0] * f[1] * s[2]
    return N, G


def surface_matrices(problem, cut_cells):
    """Unit-frame S, T, U (len(cut_cells), 8, 8) of the given cut cells."""
    n = problem.n
    cells, x, nrm, w = surface_points(problem)
    pos = np.full(n ** 3, -1, dtype=np.int64)
    pos[np.asarray(cut_cells, dtype=np.int64)] = np.arange(len(cut_cells))
    p = pos[cells]
    sel = p >= 0
    p, x, nrm, w, cells = p[sel], x[sel], nrm[sel], w[sel], cells[sel]
    order = np.argsort(p, kind="stable")          # per cell, keep the (ball, j, k) order
    p, x, nrm, w, cells = p[order], x[order], nrm[order], w[order], cells[order]
    ci, cj, ck = cells % n, (cells // n) % n, cells // (n * n)
    xi = x * n - np.stack([ci, cj, ck], axis=1).astype(np.float64)
    N, G = _shape(xi)
    dn = np.einsum("mad,md->ma", G, nrm)           # n . grad N_a
    wu = w * (n * n)
    S = np.zeros((len(cut_cells), 8, 8))
    T = np.zeros((len(cut_cells), 8, 8))
    U = np.zeros((len(cut_cells), 8, 8))
    np.add.at(S, p, wu[:, None, None] * N[:, :, None] * N[:, None, :])
    np.add.at(T, p, wu[:, None, None] * dn[:, :, None] * N[:, None, :])
    np.add.at(U, p, wu[:, None, None] * dn[:, :, None] * dn[:, None, :])
    return S, T, U


def _complement_basis():
    """Orthonormal basis (8, 7) of the vectors with zero sum."""
    H = np.eye(8) - np.full((8, 8), 1.0 / 8.0)
    vals, vecs = np.linalg.eigh(H)
    return vecs[:, vals > 0.5]


def reference_stiffness():
    """Unit stiffness of a whole cell (every point of the volume rule kept)."""
    from .integrate import unit_stiffness
    return unit_stiffness(np.ones((1, 512), dtype=bool))[0]


def beta_unit(K, U):
    """2 lambda_max of U x = lambda (K + BETA_REG K_ref) x on the complement
    of the constants (eq. local-eigenvals, beta_e = 2 lambda_max; the
    physical beta_e is this value over h), per cell; 0 where U vanishes."""
    import scipy.linalg
    Q = _complement_basis()
    Kr = Q.T @ reference_stiffness() @ Q
    out = np.zeros(K.shape[0])
    for e in range(K.shape[0]):
        K7 = Q.T @ K[e] @ Q
        U7 = Q.T @ U[e] @ Q
        if not np.any(U7):
            continue
        lam = scipy.linalg.eigh(U7, K7 + BETA_REG * Kr, eigvals_only=True)
        out[e] = 2.0 * lam[-1]
    return out


def nitsche_unit_stiffness(problem, Kunit_cut, cut_cells):
    """K_unit + beta S - T - T^T for the cut cells (unit frame), and beta."""
    S, T, U = surface_matrices(problem, cut_cells)
    beta = beta_unit(Kunit_cut, U)
    return Kunit_cut + beta[:, None, None] * S - T - np.transpose(T, (0, 2, 1)), beta
