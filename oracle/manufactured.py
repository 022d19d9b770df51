"""Manufactured-solution accuracy (paper Sect. 5.1: the exact solution
u = sin(5 pi |x|), strong Dirichlet data on the mesh-aligned boundary,
Neumann or Nitsche-Dirichlet data on the unfitted one, and the H^1 / L^2
convergence of the discretisation error).

TEST INFRASTRUCTURE ONLY (part of the oracle package).

Readings taken:
  * u(x) = sin(k rho), rho = |x - x0|, k = 5 pi, x0 = the origin of the
    paper's formula, which is the corner (0, 0, 0) of our unit cube (the
    paper's domains are not given in its text).  f = -Lap u = k^2 sin(k rho)
    - (2 k / rho) cos(k rho) has an integrable 1/rho singularity there; it
    is evaluated only at the quadrature points of the volume rule, none of
    which is at rho = 0.
  * Cube faces: strong Dirichlet data, u_h = u at the face nodes (the
    discrete solution is the DOF vector plus that lift).
  * Ball surfaces: Neumann data g_N = grad u . n (n the outward normal of
    Omega, into the ball) or Dirichlet data u imposed by Nitsche's method
    (module `surface`), both integrated with the surface rule of `surface`.
  * Volume integrals (load and errors) use the kept-point rule of the
    discretisation with the exact f, u and grad u at the points:
      b_a  = sum_e sum_kept (h^3/512) N_a f,
      e_L2 = sqrt(sum (h^3/512) (u - u_h)^2),  e_H1 = sqrt(sum (h^3/512) |grad u - grad u_h|^2).
  * Surface load, per kept sphere point with weight w: Neumann w N_a g_N;
    Nitsche (element form of Sect. 2.2 with data g = u)
    w (beta_e N_a - n . grad N_a) u, beta_e = beta_unit / h.  Nitsche data
    go to the cut cells only, like the Nitsche terms of the matrix.  Neumann
    data go to the cell that contains the point whatever its class: a
    sphere point can lie in a cell that the volume rule classifies interior
    or inactive (a thin sliver of the cell on one side of the sphere holds
    none of its 512 points), and dropping those points loses a share of the
    flux that does not fall with h (about 0.4% of the sphere's area for the
    single ball at every mesh size) and stalls the L2 convergence.  The
    load of such a cell reaches the DOFs among its nodes.
  * The load and the errors are those of -Lap u = f (kappa = 1).

Every function takes the exact solution as `sol`, a callable x (m, 3) ->
(u (m,), grad u (m, 3), f (m,)); the default is the paper's radial sine
(`radial`).  Tests pass other solutions (linear ones, which Q1 reproduces).
"""
from __future__ import annotations

import numpy as np

from . import assemble, geometry, integrate, surface

K_WAVE = 5.0 * np.pi
X0 = np.zeros(3)


def exact(x, x0=X0, k=K_WAVE):
    """(u, grad u (m, 3), f = -Lap u) of sin(k |x - x0|) at points x (m, 3)."""
    d = np.asarray(x, dtype=np.float64) - np.asarray(x0, dtype=np.float64)[None, :]
    rho = np.sqrt((d * d).sum(axis=1))
    u = np.sin(k * rho)
    du = k * np.cos(k * rho)
    with np.errstate(divide="ignore", invalid="ignore"):
        grad = (du / rho)[:, None] * d
        f = k * k * np.sin(k * rho) - 2.0 * du / rho
    return u, grad, f


def radial(x0=X0, k=K_WAVE):
    """The exact solution sin(k |x - x0|) as a `sol` callable."""
    return lambda x: exact(x, x0, k)


def _sol(sol):
    return radial() if sol is None else sol


def _cell_points(problem, cells):
    """Physical points (len(cells), 512, 3) of the volume rule in each cell,
    the kept mask (len(cells), 512) and the shape values N (512, 8) and
    reference gradients G (512, 8, 3) at the rule's reference points (the
    same in every cell)."""
    n, h = problem.n, 1.0 / problem.n
    xi = geometry.axis_offsets()
    q = np.arange(512)
    ref = np.stack([xi[q % 8], xi[(q // 8) % 8], xi[q // 64]], axis=1)
    keep = assemble.keep_masks(problem, cells)
    ci, cj, ck = cells % n, (cells // n) % n, cells // (n * n)
    org = np.stack([ci, cj, ck], axis=1).astype(np.float64)
    x = (org[:, None, :] + ref[None, :, :]) * h
    N, G = surface._shape(ref)
    return x, keep, N, G


def _at_points(sol, x, keep):
    """(u, grad u, f) of sol at the points x (c, 512, 3), 0 where not kept."""
    u, g, f = _sol(sol)(x.reshape(-1, 3))
    k = keep.reshape(-1)
    u = np.where(k, u, 0.0).reshape(keep.shape)
    f = np.where(k, f, 0.0).reshape(keep.shape)
    g = np.where(k[:, None], g, 0.0).reshape(keep.shape + (3,))
    return u, g, f


def lift(problem, sol=None):
    """u at every grid node on the cube faces, 0 elsewhere."""
    n1 = problem.n + 1
    g = np.arange(n1 ** 3)
    I, J, K = g % n1, (g // n1) % n1, g // (n1 * n1)
    face = (I == 0) | (I == problem.n) | (J == 0) | (J == problem.n) | (K == 0) | (K == problem.n)
    x = np.stack([I, J, K], axis=1)[face] / problem.n
    ud = np.zeros(n1 ** 3)
    ud[face] = _sol(sol)(x)[0]
    return ud


def volume_load(problem, d, sol=None):
    """Volume load (n_active, 8): sum over the kept points of (h^3/512) N_a f."""
    h = 1.0 / problem.n
    x, keep, N, _ = _cell_points(problem, d.active)
    _, _, f = _at_points(sol, x, keep)
    return (h ** 3 / 512.0) * (f @ N)


def surface_load(problem, d, sol=None):
    """Surface load: (cells (m,), loads (m, 8)).  Neumann data grad u . n
    on every cell that holds a kept sphere point, or the Nitsche data terms
    on the cut cells (d.cut), by problem.cut_boundary."""
    n, h = problem.n, 1.0 / problem.n
    nitsche = getattr(problem, "cut_boundary", 0) == 1
    cells, x, nrm, w = surface.surface_points(problem)
    own = d.cut if nitsche else np.unique(cells)
    pos = np.full(n ** 3, -1, dtype=np.int64)
    pos[own] = np.arange(own.size)
    p = pos[cells]
    sel = p >= 0
    p, x, nrm, w, cells = p[sel], x[sel], nrm[sel], w[sel], cells[sel]
    order = np.argsort(p, kind="stable")
    p, x, nrm, w, cells = p[order], x[order], nrm[order], w[order], cells[order]
    ci, cj, ck = cells % n, (cells // n) % n, cells // (n * n)
    xi = x * n - np.stack([ci, cj, ck], axis=1).astype(np.float64)
    N, G = surface._shape(xi)
    u, grad, _ = _sol(sol)(x)
    out = np.zeros((own.size, 8))
    if not nitsche:
        gN = (grad * nrm).sum(axis=1)
        np.add.at(out, p, w[:, None] * N * gN[:, None])
    else:
        # beta of every cut cell from the volume form before the surface terms
        keep = assemble.keep_masks(problem, d.cut)
        _, _, U = surface.surface_matrices(problem, d.cut)
        beta = surface.beta_unit(integrate.unit_stiffness(keep), U)
        dn = np.einsum("mad,md->ma", G, nrm)
        wu = w * (n * n)
        np.add.at(out, p, h * wu[:, None] * (beta[p][:, None] * N - dn) * u[:, None])
    return own, out


def load(problem, d, sol=None):
    """Right-hand side on the DOFs: volume load, surface load and the
    Dirichlet lift moved to the right, b - A_{I,D} u_D."""
    h = 1.0 / problem.n
    cells = d.active
    be = volume_load(problem, d, sol)
    # assemble on the DOFs
    ld = d.dof_of_node[d.nodes]
    b = np.zeros(d.n_dof)
    m = ld >= 0
    np.add.at(b, ld[m], be[m])
    if not problem.full_elements:
        sc, sl = surface_load(problem, d, sol)
        sd = d.dof_of_node[integrate.cell_nodes(problem.n, sc)]
        ms = sd >= 0
        np.add.at(b, sd[ms], sl[ms])
    # strong Dirichlet lift: A_e over all nodes of each cell, restricted to DOF rows
    ud = lift(problem, sol)
    Ke = d.kappa[cells][:, None, None] * h * d.Kunit
    lv = Ke @ ud[d.nodes][:, :, None]
    np.add.at(b, ld[m], -lv[:, :, 0][m])
    return b


def errors(problem, d, u_dofs, sol=None):
    """(L2 error, H1-seminorm error) of u_h = u_dofs + lift."""
    h = 1.0 / problem.n
    ug = lift(problem, sol)
    ug[d.dof_node] = u_dofs
    x, keep, N, G = _cell_points(problem, d.active)
    u, grad, _ = _at_points(sol, x, keep)
    ue = ug[d.nodes]                                          # (c, 8)
    uh = np.where(keep, ue @ N.T, 0.0)                        # (c, 512)
    gh = np.where(keep[:, :, None], np.einsum("qad,ca->cqd", G, ue) / h, 0.0)
    w = h ** 3 / 512.0
    return float(np.sqrt(w * ((u - uh) ** 2).sum())), float(np.sqrt(w * ((grad - gh) ** 2).sum()))
