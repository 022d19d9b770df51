"""Level-set geometry and cell classification (paper Sect. 2.1).

The domain is Omega = {phi > 0} with phi(x) = min_i (|x - c_i| - r_i): the
unit cube minus a union of closed balls.  Each background cell is split
into 4^3 sub-cells carrying a 2x2x2 Gauss rule, i.e. 8 points per axis and
512 per cell.  A point is kept when it lies in Omega.  Following Sect. 2.1,
a cell is internal when it lies in Omega (here: all 512 points kept),
external when it misses Omega (no point kept) and cut otherwise; active
cells are internal or cut.

Floating-point reading (the classification decides integer data, so it is
written as one fixed expression): per axis, xi_k = (a + g_p) * 0.25 for
k = 2a + p with g_0 = 0.5 - 0.5/sqrt(3), g_1 = 0.5 + 0.5/sqrt(3); the
physical coordinate is (i + xi_k) * h with h = 1/N; a point is kept iff for
every ball (dx*dx + dy*dy) + dz*dz > r*r, evaluated left to right without
fused multiply-adds, dx = x - c_x.  phi = 0 counts as outside Omega.
"""
from __future__ import annotations

import numpy as np

INTERIOR = 2
CUT = 1
INACTIVE = 0


def axis_offsets() -> np.ndarray:
    """The 8 reference coordinates xi_k in [0,1] along one axis, k = 2a + p."""
    g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    xi = np.empty(8)
    for a in range(4):
        for p in range(2):
            xi[2 * a + p] = (a + g[p]) * 0.25
    return xi


def axis_coords(n: int) -> np.ndarray:
    """(n, 8) physical coordinates (i + xi_k) * h of the points of cell i."""
    h = 1.0 / n
    xi = axis_offsets()
    return (np.arange(n, dtype=np.float64)[:, None] + xi[None, :]) * h


def kept_points(n: int, centres: np.ndarray, radii: np.ndarray,
                cells: np.ndarray) -> np.ndarray:
    """Boolean (len(cells), 512) mask of kept points for the given cell ids.

    Cell id = i + n (j + n k); point index q = kx + 8 (ky + 8 kz)."""
    cells = np.asarray(cells, dtype=np.int64)
    i = cells % n
    j = (cells // n) % n
    k = cells // (n * n)
    X = axis_coords(n)
    keep = np.ones((cells.size, 8, 8, 8), dtype=bool)   # [cell, kz, ky, kx]
    for b in range(radii.shape[0]):
        cx, cy, cz = centres[b]
        r2 = radii[b] * radii[b]
        dx = X[i] - cx
        dy = X[j] - cy
        dz = X[k] - cz
        dx2 = dx * dx
        dy2 = dy * dy
        dz2 = dz * dz
        d2 = (dx2[:, None, None, :] + dy2[:, None, :, None]) + dz2[:, :, None, None]
        keep &= d2 > r2
    return keep.reshape(cells.size, 512)


def classify(n: int, centres: np.ndarray, radii: np.ndarray,
             chunk: int = 4096):
    """Per-cell kept-point counts and classes over all n^3 cells.

    Returns (status uint8[n^3] in {INACTIVE, CUT, INTERIOR}, count int32[n^3])."""
    ncell = n ** 3
    count = np.empty(ncell, dtype=np.int32)
    for start in range(0, ncell, chunk):
        ids = np.arange(start, min(ncell, start + chunk))
        count[ids] = kept_points(n, centres, radii, ids).sum(axis=1)
    status = np.full(ncell, INACTIVE, dtype=np.uint8)
    status[count > 0] = CUT
    status[count == 512] = INTERIOR
    return status, count
