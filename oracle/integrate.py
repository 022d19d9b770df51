"""Cut-cell element matrices (paper Sect. 2.2).

With homogeneous Neumann data on the ball surfaces and strong Dirichlet data
on the cube faces there is no Nitsche term, so the element form of Sect. 2.2
reduces to A_e(u, v) = int_{e cap Omega} kappa_e grad u . grad v dV and the
load to f(v) = int_{e cap Omega} f v dV (f the Q1 interpolant of the nodal
source values).  The integral over e cap Omega is the kept-point rule of
`geometry`: weight 1/512 per kept point in reference coordinates.

Q1 basis on the reference cell [0,1]^3: local node a = ix + 2 iy + 4 iz and
N_a(xi) = prod_d (xi_d if i_d = 1 else 1 - xi_d).  With x = x0 + h xi,
grad_x = grad_xi / h and dV = h^3 dxi, so
  K_e = kappa_e h sum_{kept q} (1/512) gradN_a(xi_q) . gradN_b(xi_q),
  M_e = h^3 sum_{kept q} (1/512) N_a(xi_q) N_b(xi_q),   b_e = M_e f_e.
"""
from __future__ import annotations

import numpy as np

from .geometry import axis_offsets

LOCAL_NODE_OFFSETS = np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1]
                               for a in range(8)], dtype=np.int64)


def point_tables():
    """Per point q (q = kx + 8 (ky + 8 kz)): shape values N[q, a] and
    reference gradients G[q, a, d]."""
    xi = axis_offsets()
    N = np.empty((512, 8))
    G = np.empty((512, 8, 3))
    for kz in range(8):
        for ky in range(8):
            for kx in range(8):
                q = kx + 8 * (ky + 8 * kz)
                p = (xi[kx], xi[ky], xi[kz])
                for a in range(8):
                    o = LOCAL_NODE_OFFSETS[a]
                    f1 = [p[d] if o[d] else 1.0 - p[d] for d in range(3)]
                    df = [1.0 if o[d] else -1.0 for d in range(3)]
                    N[q, a] = f1[0] * f1[1] * f1[2]
                    G[q, a, 0] = df[0] * f1[1] * f1[2]
                    G[q, a, 1] = f1[0] * df[1] * f1[2]
                    G[q, a, 2] = f1[0] * f1[1] * df[2]
    return N, G


_TABLES = None


def _tables():
    global _TABLES
    if _TABLES is None:
        N, G = point_tables()
        # per-point outer products, flattened (a, b) -> 8 a + b
        KT = np.einsum("qad,qbd->qab", G, G).reshape(512, 64) / 512.0
        MT = np.einsum("qa,qb->qab", N, N).reshape(512, 64) / 512.0
        _TABLES = (KT, MT)
    return _TABLES


def unit_stiffness(keep: np.ndarray) -> np.ndarray:
    """Reference stiffness sum_{kept q} (1/512) gradN_a . gradN_b (kappa = 1,
    h = 1) for each row of the boolean (n_cells, 512) keep mask -> (n, 8, 8)."""
    KT, _ = _tables()
    return (keep.astype(np.float64) @ KT).reshape(-1, 8, 8)


def unit_mass(keep: np.ndarray) -> np.ndarray:
    """Reference mass sum_{kept q} (1/512) N_a N_b for each keep row -> (n, 8, 8)."""
    _, MT = _tables()
    return (keep.astype(np.float64) @ MT).reshape(-1, 8, 8)


def cell_nodes(n: int, cells: np.ndarray) -> np.ndarray:
    """(len(cells), 8) global node ids g = I + (n+1)(J + (n+1) K) of each
    cell's local nodes a = ix + 2 iy + 4 iz."""
    cells = np.asarray(cells, dtype=np.int64)
    i = cells % n
    j = (cells // n) % n
    k = cells // (n * n)
    o = LOCAL_NODE_OFFSETS
    n1 = n + 1
    return ((i[:, None] + o[None, :, 0])
            + n1 * ((j[:, None] + o[None, :, 1]) + n1 * (k[:, None] + o[None, :, 2])))
