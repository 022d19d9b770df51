"""Subdomain partition, interface objects and coarse DOFs.

Sect. 2.1: subdomains are built by aggregating active cells; on the uniform
Cartesian mesh subdomain omega = block (Bx, By, Bz) of s^3 cells, numbered
Bx + m (By + m Bz) with m = N / s, holding the block's active cells.
Sect. 3.1: V_omega lives on the nodes of omega's active cells.
Sect. 3.2: interface nodes are classified into objects (corners, edges,
faces) by the set of subdomains containing them; coarse DOFs are mean
values on the selected objects (eq. coarse-dofs); BDDC(cef) selects all
objects, BDDC(ce) corners and edges.
Sect. 4.4 (variant 1): edges cut by the boundary are split: every DOF on a
cut FE edge becomes a corner and the remaining FE edges are aggregated into
connected sub-edges.

Readings taken (the paper gives no algorithm for these steps):
  * S(xi) = ascending ids of the subdomains having an active cell that
    contains node xi; a DOF is interior when |S| = 1, interface otherwise.
  * Two axis-adjacent interface DOFs a, b are linked when S(a) = S(b) and
    every subdomain of S(a) has an active cell containing the FE edge (a, b).
    Objects are the connected components of the links.
  * Object type: corner if it holds one DOF; face if it holds the 4 DOFs of a
    mesh face whose two cells are active and lie in the two subdomains of S;
    edge otherwise (so a two-subdomain contact along a line is an edge).
  * Objects are ordered by their smallest DOF id.
  * Variant 1 classifies each linking FE edge t of an edge object exactly
    against the balls: interior (t in Omega) if every ball is at distance
    > r from t, exterior (t misses Omega) if the closed chords of the balls
    cover t, cut otherwise.  Sub-edges of one DOF become corners.
  * Variant 2 (Sect. 4.5) applies with the stiffness weighting: the
    weighting coefficient of an interface DOF xi is the vector of its
    weights A^w_xixi / sum_{w' in S} A^w'_xixi over w in S (eq.
    alge-weighting), each A^w_xixi summed over the active cells of w that
    contain xi in ascending cell order.  Two DOFs of an edge object joined by
    one of its links have the same coefficient when every component differs
    by at most V2_TOL; edges are re-aggregated through such links only, and
    a DOF left alone becomes a corner.  Faces and corners are unchanged.  With
    the topological weighting every coefficient on an object is 1/|S|, so
    variant 2 leaves the standard objects.
  * The mean value of eq. coarse-dofs is the equal-weight nodal mean
    1/|lambda| sum_{xi in lambda} u(xi) (a row scaling of the constraint,
    which leaves the BDDC space unchanged).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

CORNER, EDGE, FACE = 0, 1, 2
# Variant 2: "the same weighting coefficient, up to machine precision"
# (Sect. 4.5); coefficients lie in [0, 1].
V2_TOL = 1e-12


@dataclass
class Topology:
    m: int
    s: int
    sub_of_active: np.ndarray   # subdomain id of each active cell
    sub_cells: List[np.ndarray] # indices into d.active per subdomain
    sub_dofs: List[np.ndarray]  # local DOFs (ascending) per subdomain
    S_ptr: np.ndarray           # CSR of subdomain sets per DOF
    S_ids: np.ndarray
    obj_ptr: np.ndarray         # CSR of DOFs per object (objects sorted)
    obj_dofs: np.ndarray
    obj_type: np.ndarray        # int8: CORNER / EDGE / FACE
    obj_S: List[tuple]
    coarse_of_obj: np.ndarray   # int32, -1 when the object carries no coarse DOF
    n_coarse: int

    @property
    def n_sub(self) -> int:
        return self.m ** 3

    def S(self, dof: int) -> tuple:
        return tuple(self.S_ids[self.S_ptr[dof]:self.S_ptr[dof + 1]].tolist())

    def card(self) -> np.ndarray:
        return np.diff(self.S_ptr)

    def objects(self):
        for o in range(self.obj_type.size):
            yield self.obj_dofs[self.obj_ptr[o]:self.obj_ptr[o + 1]]


def _cell_ijk(n, cells):
    cells = np.asarray(cells, dtype=np.int64)
    return cells % n, (cells // n) % n, cells // (n * n)


def subdomain_of_cells(n, s, cells):
    i, j, k = _cell_ijk(n, cells)
    m = n // s
    return (i // s) + m * ((j // s) + m * (k // s))


def _set_rows(pairs_dof, pairs_sub, n_dof):
    """CSR of sorted unique subdomain ids per DOF from (dof, sub) pairs."""
    key = np.unique(pairs_dof * (1 << 20) + pairs_sub)
    dofs = key >> 20
    subs = key & ((1 << 20) - 1)
    ptr = np.zeros(n_dof + 1, dtype=np.int64)
    np.add.at(ptr, dofs + 1, 1)
    return np.cumsum(ptr), subs.astype(np.int64)


def _padded_sets(ptr, ids, rows):
    """(len(rows), 8) padded (-1) subdomain sets for the given DOF rows."""
    out = np.full((rows.size, 8), -1, dtype=np.int64)
    lens = ptr[rows + 1] - ptr[rows]
    for t in range(8):
        has = lens > t
        out[has, t] = ids[ptr[rows[has]] + t]
    return out


def segment_class(n, node_lo, axis, centres, radii):
    """Exact class of the FE edge from grid node node_lo = (I, J, K) to
    node_lo + e_axis: 0 interior (t in Omega), 1 exterior (t misses Omega),
    2 cut.  Node coordinates are I * h with h = 1/n."""
    h = 1.0 / n
    p = [float(node_lo[0]) * h, float(node_lo[1]) * h, float(node_lo[2]) * h]
    a = p[axis]
    b = float(node_lo[axis] + 1) * h
    o1, o2 = [d for d in range(3) if d != axis]
    interior = True
    chords = []
    for i in range(radii.shape[0]):
        c = centres[i]
        r2 = radii[i] * radii[i]
        dy = p[o1] - c[o1]
        dz = p[o2] - c[o2]
        p2 = dy * dy + dz * dz
        t = min(max(c[axis], a), b)
        dd = t - c[axis]
        dist2 = p2 + dd * dd
        if not dist2 > r2:
            interior = False
        if p2 <= r2:
            half = np.sqrt(r2 - p2)
            chords.append((c[axis] - half, c[axis] + half))
    if interior:
        return 0
    chords.sort()
    cur = a
    for lo, hi in chords:
        if lo > cur:
            break
        cur = max(cur, hi)
        if cur >= b:
            return 1
    return 2


def stiffness_coefficients(problem, d, S_ptr, S_ids, sub_all):
    """Weighting coefficients of eq. alge-weighting per interface DOF: a dict
    DOF -> array over S(xi) (ascending subdomains) of A^w_xixi / sum_{w'}
    A^w'_xixi, with A^w_xixi = sum of kappa_e h K_e[a, a] over the active
    cells e of w containing xi, in ascending cell order."""
    n, h = problem.n, 1.0 / problem.n
    pos = np.full(n ** 3, -1, dtype=np.int64)
    pos[d.active] = np.arange(d.active.size)
    n1 = n + 1
    out = {}
    for dof in np.flatnonzero(np.diff(S_ptr) >= 2):
        node = int(d.dof_node[dof])
        I, J, K = node % n1, (node // n1) % n1, node // (n1 * n1)
        S = S_ids[S_ptr[dof]:S_ptr[dof + 1]]
        diag = np.zeros(S.size)
        for w in (0, 1):                 # cells in ascending id: k, then j, then i
            for v in (0, 1):
                for u in (0, 1):
                    ci, cj, ck = I - 1 + u, J - 1 + v, K - 1 + w
                    if min(ci, cj, ck) < 0 or max(ci, cj, ck) >= n:
                        continue
                    c = ci + n * (cj + n * ck)
                    if pos[c] < 0:
                        continue
                    a = (1 - u) + 2 * (1 - v) + 4 * (1 - w)     # the node's corner in the cell
                    t = int(np.flatnonzero(S == sub_all[c])[0])
                    diag[t] += d.kappa[c] * h * d.Kunit[pos[c], a, a]
        tot = 0.0
        for t in range(S.size):
            tot += diag[t]
        out[int(dof)] = diag / tot
    return out


def build(problem, d) -> Topology:
    n, s = problem.n, problem.s
    if n % s != 0:
        raise ValueError("subdomain size must divide the mesh size")
    m = n // s
    n1 = n + 1
    nd = d.n_dof
    sub_act = subdomain_of_cells(n, s, d.active)
    order = np.argsort(sub_act, kind="stable")
    bounds = np.searchsorted(sub_act[order], np.arange(m ** 3 + 1))
    sub_cells = [order[bounds[w]:bounds[w + 1]] for w in range(m ** 3)]

    ld = d.dof_of_node[d.nodes]                          # (n_active, 8)
    pd = ld.ravel()
    ps = np.repeat(sub_act, 8)
    keep = pd >= 0
    S_ptr, S_ids = _set_rows(pd[keep], ps[keep], nd)
    sub_dofs = []
    for w in range(m ** 3):
        x = ld[sub_cells[w]].ravel()
        sub_dofs.append(np.unique(x[x >= 0]))
    card = np.diff(S_ptr)
    iface = card >= 2

    # ---- links between axis-adjacent interface DOFs -------------------------
    status_active = np.zeros(n ** 3, dtype=bool)
    status_active[d.active] = True
    sub_all = subdomain_of_cells(n, s, np.arange(n ** 3))
    li, lj = [], []
    link_axis = []
    idof = np.flatnonzero(iface)
    inode = d.dof_node[idof]
    I, J, K = inode % n1, (inode // n1) % n1, inode // (n1 * n1)
    for axis in range(3):
        step = (1, n1, n1 * n1)[axis]
        nb = inode + step
        nbdof = d.dof_of_node[nb]
        ok = nbdof >= 0
        ok[ok] &= iface[nbdof[ok]]
        a_d, b_d = idof[ok], nbdof[ok]
        Sa = _padded_sets(S_ptr, S_ids, a_d)
        Sb = _padded_sets(S_ptr, S_ids, b_d)
        same = (Sa == Sb).all(axis=1)
        a_d, b_d, Sa = a_d[same], b_d[same], Sa[same]
        Ia, Ja, Ka = I[ok][same], J[ok][same], K[ok][same]
        # the 4 cells containing the FE edge
        St = np.full((a_d.size, 4), -1, dtype=np.int64)
        o1, o2 = [dd for dd in range(3) if dd != axis]
        base = [Ia, Ja, Ka]
        t = 0
        for u in (-1, 0):
            for v in (-1, 0):
                c = [base[0].copy(), base[1].copy(), base[2].copy()]
                c[o1] = c[o1] + u
                c[o2] = c[o2] + v
                inside = ((c[0] >= 0) & (c[0] < n) & (c[1] >= 0) & (c[1] < n)
                          & (c[2] >= 0) & (c[2] < n))
                cid = np.where(inside, c[0] + n * (c[1] + n * c[2]), 0)
                act = inside & status_active[cid]
                St[act, t] = sub_all[cid[act]]
                t += 1
        # every subdomain of S(a) must own an active cell containing the edge
        full = np.ones(a_d.size, dtype=bool)
        for col in range(8):
            w = Sa[:, col]
            need = w >= 0
            present = (St == w[:, None]).any(axis=1)
            full &= ~need | present
        li.append(a_d[full])
        lj.append(b_d[full])
        link_axis.append(np.full(full.sum(), axis))
    li = np.concatenate(li) if li else np.zeros(0, np.int64)
    lj = np.concatenate(lj) if lj else np.zeros(0, np.int64)
    link_axis = np.concatenate(link_axis) if link_axis else np.zeros(0, np.int64)

    # ---- objects: connected components of the links -------------------------
    G = sp.coo_matrix((np.ones(li.size), (li, lj)), shape=(nd, nd))
    ncomp, lab = connected_components(G, directed=False)
    lab_i = lab[idof]
    comps = np.unique(lab_i)
    cmap = np.full(ncomp, -1, dtype=np.int64)
    cmap[comps] = np.arange(comps.size)
    obj_of = np.full(nd, -1, dtype=np.int64)
    obj_of[idof] = cmap[lab_i]
    nobj = comps.size
    # faces: mesh faces between cells of two different subdomains
    is_face = np.zeros(nobj, dtype=bool)
    for axis in range(3):
        o1, o2 = [dd for dd in range(3) if dd != axis]
        # cell pairs (c_lo, c_hi) adjacent across a block boundary plane
        cells = np.arange(n ** 3)
        ci, cj, ck = _cell_ijk(n, cells)
        cc = [ci, cj, ck]
        sel = (cc[axis] + 1 < n) & (((cc[axis] + 1) % s) == 0)
        lo = cells[sel]
        hi = lo + (1, n, n * n)[axis]
        both = status_active[lo] & status_active[hi]
        lo, hi = lo[both], hi[both]
        if lo.size == 0:
            continue
        li_, lj_, lk_ = _cell_ijk(n, lo)
        base = [li_, lj_, lk_]
        base[axis] = base[axis] + 1                 # node plane index
        fdofs = []
        for u in (0, 1):
            for v in (0, 1):
                c = [base[0].copy(), base[1].copy(), base[2].copy()]
                c[o1] = c[o1] + u
                c[o2] = c[o2] + v
                fdofs.append(d.dof_of_node[c[0] + n1 * (c[1] + n1 * c[2])])
        fdofs = np.stack(fdofs, axis=1)             # (nf, 4)
        ok = (fdofs >= 0).all(axis=1)
        fdofs, lo, hi = fdofs[ok], lo[ok], hi[ok]
        objs = obj_of[fdofs]
        ok = (objs >= 0).all(axis=1) & (objs == objs[:, :1]).all(axis=1)
        fdofs, lo, hi, objs = fdofs[ok], lo[ok], hi[ok], objs[ok]
        w1 = sub_all[lo]
        w2 = sub_all[hi]
        Sf = _padded_sets(S_ptr, S_ids, fdofs[:, 0])
        two = (Sf[:, 2] < 0) & (Sf[:, 1] >= 0)
        pair = (np.minimum(w1, w2) == Sf[:, 0]) & (np.maximum(w1, w2) == Sf[:, 1])
        is_face[objs[two & pair, 0]] = True

    # group DOFs per object
    idx = np.argsort(obj_of[idof], kind="stable")
    members = idof[idx]
    mptr = np.searchsorted(obj_of[idof][idx], np.arange(nobj + 1))
    objs = []
    for o in range(nobj):
        dofs = np.sort(members[mptr[o]:mptr[o + 1]])
        typ = CORNER if dofs.size == 1 else (FACE if is_face[o] else EDGE)
        objs.append((dofs, typ))

    # ---- variant 1: split edges cut by the boundary (Sect. 4.4) -----------------
    if problem.coarse_variant == 1 and problem.radii.shape[0] > 0:
        link_obj = obj_of[li]
        new = []
        for o, (dofs, typ) in enumerate(objs):
            if typ != EDGE:
                new.append((dofs, typ))
                continue
            sel = np.flatnonzero(link_obj == o)
            cls = np.empty(sel.size, dtype=np.int64)
            for t, e in enumerate(sel):
                node = d.dof_node[li[e]]
                ijk = (node % n1, (node // n1) % n1, node // (n1 * n1))
                cls[t] = segment_class(n, ijk, int(link_axis[e]), problem.centres,
                                       problem.radii)
            if not (cls == 2).any():
                new.append((dofs, typ))
                continue
            cut_dofs = set(li[sel[cls == 2]].tolist()) | set(lj[sel[cls == 2]].tolist())
            for x in sorted(cut_dofs):
                new.append((np.array([x], dtype=np.int64), CORNER))
            rest = np.array([x for x in dofs.tolist() if x not in cut_dofs], dtype=np.int64)
            if rest.size == 0:
                continue
            pos = {x: t for t, x in enumerate(rest.tolist())}
            ra, rb = [], []
            for e in sel[cls != 2]:
                if li[e] in pos and lj[e] in pos:
                    ra.append(pos[li[e]])
                    rb.append(pos[lj[e]])
            Gs = sp.coo_matrix((np.ones(len(ra)), (ra, rb)), shape=(rest.size, rest.size))
            nc, lab2 = connected_components(Gs, directed=False)
            for c in range(nc):
                part = np.sort(rest[lab2 == c])
                new.append((part, CORNER if part.size == 1 else EDGE))
        objs = new

    # ---- variant 2: split edges with non-constant weighting coefficients ------
    if problem.coarse_variant == 2 and problem.weighting == 1:
        coef = stiffness_coefficients(problem, d, S_ptr, S_ids, sub_all)
        link_obj = obj_of[li]
        new = []
        for o, (dofs, typ) in enumerate(objs):
            if typ != EDGE:
                new.append((dofs, typ))
                continue
            sel = np.flatnonzero(link_obj == o)
            pos = {x: t for t, x in enumerate(dofs.tolist())}
            ra, rb = [], []
            for e in sel:
                a, b = int(li[e]), int(lj[e])
                if np.max(np.abs(coef[a] - coef[b])) <= V2_TOL:
                    ra.append(pos[a])
                    rb.append(pos[b])
            Gs = sp.coo_matrix((np.ones(len(ra)), (ra, rb)), shape=(dofs.size, dofs.size))
            nc, lab2 = connected_components(Gs, directed=False)
            for c in range(nc):
                part = np.sort(dofs[lab2 == c])
                new.append((part, CORNER if part.size == 1 else EDGE))
        objs = new

    objs.sort(key=lambda t: int(t[0][0]))
    obj_ptr = np.zeros(len(objs) + 1, dtype=np.int64)
    obj_ptr[1:] = np.cumsum([o[0].size for o in objs])
    obj_dofs = (np.concatenate([o[0] for o in objs]) if objs
                else np.zeros(0, dtype=np.int64))
    obj_type = np.array([o[1] for o in objs], dtype=np.int8)
    obj_S = [tuple(S_ids[S_ptr[o[0][0]]:S_ptr[o[0][0] + 1]].tolist()) for o in objs]
    if problem.objects == 0:        # cef: corners, edges and faces
        selected = np.ones(len(objs), dtype=bool)
    else:                           # ce: corners and edges
        selected = obj_type != FACE
    coarse = np.full(len(objs), -1, dtype=np.int32)
    coarse[selected] = np.arange(selected.sum(), dtype=np.int32)
    return Topology(m=m, s=s, sub_of_active=sub_act, sub_cells=sub_cells,
                    sub_dofs=sub_dofs, S_ptr=S_ptr, S_ids=S_ids, obj_ptr=obj_ptr,
                    obj_dofs=obj_dofs, obj_type=obj_type, obj_S=obj_S,
                    coarse_of_obj=coarse, n_coarse=int(selected.sum()))
