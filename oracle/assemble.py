"""Discrete problem: DOF numbering, global operator and load (paper Sect. 2.2,
global problem "find u in V-bar with A-bar u = b"; strong Dirichlet data on
the mesh-aligned boundary as in Sect. 5.1).

Readings taken:
  * DOFs are the grid nodes (I, J, K) with 1 <= I, J, K <= N-1 that belong to
    at least one active cell; nodes on the cube faces carry u = 0.  DOFs are
    numbered in ascending order of g = I + (N+1)(J + (N+1) K).
  * b = M_cut f: the source is the Q1 field with the given nodal values on
    all (N+1)^3 grid nodes, integrated with the kept-point rule.
  * With cut_boundary = 1 the ball surfaces carry homogeneous Dirichlet
    data imposed by Nitsche's method (module `surface`): the cut cells'
    unit stiffness gains the surface terms, the load is unchanged.
  * A connected set of active cells (joined through shared DOF nodes) that
    touches no Dirichlet node leaves A-bar singular; such meshes are rejected.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from . import geometry, integrate


@dataclass
class Discretisation:
    n: int
    h: float
    status: np.ndarray          # uint8[n^3]
    count: np.ndarray           # int32[n^3] kept points per cell
    active: np.ndarray          # int64 ids of active cells (ascending)
    cut: np.ndarray             # int64 ids of cut cells (ascending)
    kappa: np.ndarray           # float64[n^3]
    Kunit: np.ndarray           # (n_active, 8, 8) reference stiffness (kappa=1, h=1)
    Munit: np.ndarray           # (n_active, 8, 8) reference mass (h=1)
    nodes: np.ndarray           # (n_active, 8) global node ids
    dof_of_node: np.ndarray     # int64[(n+1)^3], -1 if not a DOF
    dof_node: np.ndarray        # int64[n_dof] node id of each DOF
    A: sp.csr_matrix            # global operator on DOFs
    Mcut: sp.csr_matrix         # (n_dof, (n+1)^3): b = Mcut f

    @property
    def n_dof(self) -> int:
        return int(self.dof_node.size)


class SingularProblem(ValueError):
    pass


def keep_masks(problem, cells):
    if problem.full_elements:
        return np.ones((len(cells), 512), dtype=bool)
    return geometry.kept_points(problem.n, problem.centres, problem.radii, cells)


def discretise(problem, check_floating: bool = True, count=None) -> Discretisation:
    """Discrete problem of `problem`.  `count` (optional, int[n^3]) replaces
    the classification by hand-made cell data for tests of the indexing
    rules: every entry must be 0 (inactive) or 512 (whole cell kept), and the
    problem must have no balls, so active cells integrate as whole cells."""
    n = problem.n
    h = 1.0 / n
    if count is None:
        status, count = geometry.classify(n, problem.centres, problem.radii)
    else:
        count = np.asarray(count, dtype=np.int32).reshape(-1)
        if count.size != n ** 3 or ((count != 0) & (count != 512)).any() or problem.n_balls:
            raise ValueError("hand-made cell data: n^3 counts of 0 or 512, no balls")
        status = np.where(count == 512, geometry.INTERIOR, geometry.INACTIVE).astype(np.uint8)
    active = np.flatnonzero(status != geometry.INACTIVE).astype(np.int64)
    cut = np.flatnonzero(status == geometry.CUT).astype(np.int64)
    kappa = (np.ones(n ** 3) if problem.kappa is None
             else np.asarray(problem.kappa, dtype=np.float64))
    Kunit = np.empty((active.size, 8, 8))
    Munit = np.empty((active.size, 8, 8))
    for start in range(0, active.size, 4096):
        sl = slice(start, min(active.size, start + 4096))
        keep = keep_masks(problem, active[sl])
        Kunit[sl] = integrate.unit_stiffness(keep)
        Munit[sl] = integrate.unit_mass(keep)
    if getattr(problem, "cut_boundary", 0) == 1 and not problem.full_elements and cut.size:
        # weak Dirichlet data on the ball surfaces (Nitsche, Sect. 2.2)
        from . import surface
        pos = np.searchsorted(active, cut)
        Kunit[pos], _ = surface.nitsche_unit_stiffness(problem, Kunit[pos], cut)
    nodes = integrate.cell_nodes(n, active)

    # DOFs: interior grid nodes touched by an active cell (Sect. 5.1: strong
    # Dirichlet on the mesh-aligned boundary).
    n1 = n + 1
    touched = np.zeros(n1 ** 3, dtype=bool)
    touched[nodes.ravel()] = True
    g = np.arange(n1 ** 3)
    I, J, K = g % n1, (g // n1) % n1, g // (n1 * n1)
    inner = (I >= 1) & (I <= n - 1) & (J >= 1) & (J <= n - 1) & (K >= 1) & (K <= n - 1)
    is_dof = touched & inner
    dof_node = np.flatnonzero(is_dof).astype(np.int64)
    dof_of_node = np.full(n1 ** 3, -1, dtype=np.int64)
    dof_of_node[dof_node] = np.arange(dof_node.size)

    # A-bar = sum_e A_e, restricted to the DOFs (Sect. 2.2).
    Ke = kappa[active][:, None, None] * h * Kunit
    Me = h ** 3 * Munit
    ld = dof_of_node[nodes]                         # (n_active, 8)
    rows = np.repeat(ld, 8, axis=1).ravel()
    cols = np.tile(ld, (1, 8)).ravel()
    keep = (rows >= 0) & (cols >= 0)
    nd = dof_node.size
    A = sp.coo_matrix((Ke.reshape(-1)[keep], (rows[keep], cols[keep])),
                      shape=(nd, nd)).tocsr()
    # b = sum_e M_e f_e over all grid nodes of the cell (f defined everywhere).
    mcols = np.tile(nodes, (1, 8)).ravel()
    mkeep = rows >= 0
    Mcut = sp.coo_matrix((Me.reshape(-1)[mkeep], (rows[mkeep], mcols[mkeep])),
                         shape=(nd, n1 ** 3)).tocsr()
    d = Discretisation(n=n, h=h, status=status, count=count, active=active,
                       cut=cut, kappa=kappa, Kunit=Kunit, Munit=Munit,
                       nodes=nodes, dof_of_node=dof_of_node, dof_node=dof_node,
                       A=A, Mcut=Mcut)
    if check_floating and floating_components(d):
        raise SingularProblem("an active component touches no Dirichlet node")
    return d


def floating_components(d: Discretisation) -> int:
    """Number of connected groups of active cells (joined through shared DOF
    nodes) none of whose cells has a Dirichlet (cube-face) node."""
    na = d.active.size
    if na == 0:
        return 0
    ld = d.dof_of_node[d.nodes]
    cell_idx = np.repeat(np.arange(na), 8)
    dof_idx = ld.ravel()
    m = dof_idx >= 0
    # bipartite cell-DOF graph
    G = sp.coo_matrix((np.ones(m.sum()), (cell_idx[m], na + dof_idx[m])),
                      shape=(na + d.n_dof, na + d.n_dof))
    ncomp, lab = connected_components(G, directed=False)
    n1 = d.n + 1
    nodes = d.nodes
    I, J, K = nodes % n1, (nodes // n1) % n1, nodes // (n1 * n1)
    on_face = ((I == 0) | (I == d.n) | (J == 0) | (J == d.n) | (K == 0) | (K == d.n)).any(axis=1)
    grounded = np.zeros(ncomp, dtype=bool)
    grounded[lab[:na][on_face]] = True
    comps = np.unique(lab[:na])
    return int((~grounded[comps]).sum())


def load(d: Discretisation, f_nodes) -> np.ndarray:
    """b = M_cut f (f = 1 everywhere when f_nodes is None)."""
    if f_nodes is None:
        f_nodes = np.ones(d.Mcut.shape[1])
    return d.Mcut @ np.asarray(f_nodes, dtype=np.float64)
