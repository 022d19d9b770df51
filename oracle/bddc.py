"""BDDC preconditioner M = I0 A0^{-1} I0^T + Q A~^{-1} Q^T (paper eq. bddc,
Sect. 3.4) with Q = E W (Sect. 3.3).

Pieces, in the paper's terms:
  * A_omega: sub-assembled Neumann matrix of subdomain omega (Sect. 3.1),
    dense over omega's DOFs (interior first is NOT assumed; local order is
    ascending global DOF id).
  * W: weighting; topological (eq. weighting): 1/|neigh(xi)|, or stiffness
    (eq. alge-weighting): A^omega_{xi xi} / sum_{omega'} A^{omega'}_{xi xi}.
  * E: harmonic extension, corrects interior DOFs with local Dirichlet solves.
  * A~: A restricted to the BDDC space (coarse DOFs continuous); applied as
    local constrained Neumann (KKT) solves plus a coarse correction on the
    coarse basis Phi (energy-minimising, C Phi = I).

Apply of M to a residual r, steps in order:
  (1) delta_I = A_II^{-1} r_I                          (I0 A0^{-1} I0^T r)
  (2) rhat_G  = r_G - sum_omega A^omega_GI delta_I      (E^T r on the interface)
  (3) g_omega = D_omega rhat_G|omega                   (W^T)
  (4) [z; mu] = KKT_omega^{-1} [g; 0];  c += R_c^T Phi^T g
  (5) u_c = A_c^{-1} c;  u~_omega = z + Phi R_c u_c     (A~^{-1})
  (6) u_G = sum_omega R^T D_omega u~_omega|G            (W)
  (7) u_I = -A_II^{-1} A_IG u_G;  M r = [delta_I + u_I; u_G]   (E)

The constrained Neumann problem is solved in its plain saddle-point (KKT)
form with a dense LU factorisation; the Dirichlet problems and the coarse
problem with dense Cholesky.  Everything is FP64.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.linalg as sla

from .topology import Topology


def local_matrix(d, topo: Topology, w: int) -> np.ndarray:
    """Dense A_omega over omega's DOFs (ascending), assembled from the active
    cells of omega only (Sect. 3.1)."""
    dofs = topo.sub_dofs[w]
    A = np.zeros((dofs.size, dofs.size))
    cells = topo.sub_cells[w]
    if cells.size == 0:
        return A
    ld = d.dof_of_node[d.nodes[cells]]                       # global DOF or -1
    loc = np.where(ld >= 0, np.searchsorted(dofs, np.maximum(ld, 0)), -1)
    Ke = d.kappa[d.active[cells]][:, None, None] * d.h * d.Kunit[cells]
    ra = np.repeat(loc, 8, axis=1).ravel()          # row local index of (c, a, b)
    cb = np.tile(loc, (1, 8)).ravel()               # column local index
    ok = (ra >= 0) & (cb >= 0)
    np.add.at(A, (ra[ok], cb[ok]), Ke.reshape(-1)[ok])
    return A


def weights(d, topo: Topology, locA: List[np.ndarray], stiffness: bool):
    """Per subdomain, the weight of each local DOF: 1 at interior DOFs,
    topological 1/|S(xi)| or stiffness A^w_xx / sum_{w' in S(xi)} A^{w'}_xx
    (summed over ascending w') at interface DOFs."""
    nd = d.n_dof
    card = topo.card()
    if not stiffness:
        return [1.0 / card[topo.sub_dofs[w]] for w in range(topo.n_sub)]
    diag = [np.diag(locA[w]).copy() for w in range(topo.n_sub)]
    total = np.zeros(nd)
    for w in range(topo.n_sub):           # ascending subdomain order
        total[topo.sub_dofs[w]] += diag[w]
    return [diag[w] / total[topo.sub_dofs[w]] for w in range(topo.n_sub)]


def constraint_matrix(topo: Topology, w: int):
    """C_omega (rows: selected objects of omega in coarse-id order) and the
    global coarse ids of those rows.  Row of object lambda = 1/|lambda| on
    lambda's DOFs (eq. coarse-dofs, equal-weight mean)."""
    dofs = topo.sub_dofs[w]
    rows, ids = [], []
    for o, od in enumerate(topo.objects()):
        cid = topo.coarse_of_obj[o]
        if cid < 0 or w not in topo.obj_S[o]:
            continue
        r = np.zeros(dofs.size)
        r[np.searchsorted(dofs, od)] = 1.0 / od.size
        rows.append(r)
        ids.append(int(cid))
    if not rows:
        return np.zeros((0, dofs.size)), np.zeros(0, dtype=np.int64)
    order = np.argsort(ids)
    return np.array(rows)[order], np.array(ids, dtype=np.int64)[order]


@dataclass
class SubdomainOps:
    dofs: np.ndarray        # local DOFs (global ids)
    I: np.ndarray           # positions of interior DOFs within dofs
    G: np.ndarray           # positions of interface DOFs within dofs
    A: np.ndarray           # dense A_omega
    D: np.ndarray           # weights per local DOF
    C: np.ndarray           # constraint rows
    cids: np.ndarray        # coarse ids of the constraint rows
    chol_II: tuple          # cho_factor of A_II (or None if no interior DOF)
    kkt: tuple              # lu_factor of [[A, C^T], [C, 0]]
    Phi: np.ndarray         # coarse basis (n_local x n_c_local)
    Ac: np.ndarray          # Phi^T A Phi


class BDDC:
    """Factors and applies M (eq. bddc)."""

    def __init__(self, d, topo: Topology, stiffness: bool = True):
        self.d, self.topo = d, topo
        card = topo.card()
        locA = [local_matrix(d, topo, w) for w in range(topo.n_sub)]
        D = weights(d, topo, locA, stiffness)
        self.subs: List[SubdomainOps] = []
        nc = topo.n_coarse
        Ac = np.zeros((nc, nc))
        for w in range(topo.n_sub):
            dofs = topo.sub_dofs[w]
            if dofs.size == 0:
                self.subs.append(None)
                continue
            A = locA[w]
            I = np.flatnonzero(card[dofs] == 1)
            G = np.flatnonzero(card[dofs] >= 2)
            C, cids = constraint_matrix(topo, w)
            chol = sla.cho_factor(A[np.ix_(I, I)], lower=True) if I.size else None
            k = C.shape[0]
            KKT = np.zeros((dofs.size + k, dofs.size + k))
            KKT[:dofs.size, :dofs.size] = A
            KKT[:dofs.size, dofs.size:] = C.T
            KKT[dofs.size:, :dofs.size] = C
            lu = sla.lu_factor(KKT)
            rhs = np.zeros((dofs.size + k, k))
            rhs[dofs.size:, :] = np.eye(k)
            Phi = sla.lu_solve(lu, rhs)[:dofs.size] if k else np.zeros((dofs.size, 0))
            Acw = Phi.T @ A @ Phi
            Ac[np.ix_(cids, cids)] += Acw
            self.subs.append(SubdomainOps(dofs=dofs, I=I, G=G, A=A, D=D[w], C=C,
                                          cids=cids, chol_II=chol, kkt=lu,
                                          Phi=Phi, Ac=Acw))
        self.Ac = Ac
        self.chol_c = sla.cho_factor(Ac, lower=True) if nc else None
        self.iface = card >= 2

    def apply(self, r: np.ndarray) -> np.ndarray:
        nd = self.d.n_dof
        # (1) interior Dirichlet solves
        delta = np.zeros(nd)
        for sw in self.subs:
            if sw is None or sw.I.size == 0:
                continue
            delta[sw.dofs[sw.I]] = sla.cho_solve(sw.chol_II, r[sw.dofs[sw.I]])
        # (2) rhat_G = r_G - sum_w A_GI delta_I
        rhat = r.copy()
        for sw in self.subs:
            if sw is None or sw.I.size == 0 or sw.G.size == 0:
                continue
            rhat[sw.dofs[sw.G]] -= sw.A[np.ix_(sw.G, sw.I)] @ delta[sw.dofs[sw.I]]
        # (3)-(4) weighted restriction, constrained Neumann solves, coarse rhs
        nc = self.topo.n_coarse
        c = np.zeros(nc)
        zs = []
        for sw in self.subs:
            if sw is None:
                zs.append(None)
                continue
            g = np.zeros(sw.dofs.size)
            g[sw.G] = sw.D[sw.G] * rhat[sw.dofs[sw.G]]
            k = sw.C.shape[0]
            z = sla.lu_solve(sw.kkt, np.concatenate([g, np.zeros(k)]))[:sw.dofs.size]
            zs.append(z)
            if k:
                c[sw.cids] += sw.Phi.T @ g
        # (5) coarse solve
        uc = sla.cho_solve(self.chol_c, c) if nc else c
        # (6) weighted average of u~ on the interface
        out = np.zeros(nd)
        for sw, z in zip(self.subs, zs):
            if sw is None:
                continue
            ut = z + (sw.Phi @ uc[sw.cids] if sw.cids.size else 0.0)
            np.add.at(out, sw.dofs[sw.G], sw.D[sw.G] * ut[sw.G])
        # (7) harmonic extension into the interiors
        for sw in self.subs:
            if sw is None or sw.I.size == 0:
                continue
            rhs = -(sw.A[np.ix_(sw.I, sw.G)] @ out[sw.dofs[sw.G]]) if sw.G.size else 0.0 * delta[sw.dofs[sw.I]]
            out[sw.dofs[sw.I]] = delta[sw.dofs[sw.I]] + sla.cho_solve(sw.chol_II, rhs)
        return out
