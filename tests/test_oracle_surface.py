"""Pins of the oracle's Nitsche part (oracle/surface.py, paper Sect. 2.2):
the sphere rule against exact surface integrals, the kept part of the
surface against spherical-zone and cap areas, the surface matrices against
the Q1 identities and the closed forms of a plane, and beta_e against the
coercivity it must guarantee."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import assemble, surface


@pytest.mark.parametrize("r,h", [(0.1, 1 / 16), (0.3, 1 / 8), (0.05, 1 / 64)])
def test_sphere_rule_is_exact_for_area_and_second_moments(r, h):
    d, w = surface.sphere_rule(r, h)
    area = 4.0 * math.pi * r * r
    assert abs(w.sum() - area) <= 1e-13 * area
    assert np.abs(w @ d).max() <= 1e-14 * area                          # first moments vanish
    M = (w[:, None, None] * d[:, :, None] * d[:, None, :]).sum(axis=0)  # int n n^T = (A/3) I
    assert np.abs(M - area / 3.0 * np.eye(3)).max() <= 1e-13 * area
    assert np.allclose((d * d).sum(axis=1), 1.0, atol=1e-15)


def _area(problem):
    cells, x, n, w = surface.surface_points(problem)
    return w.sum(), x, n


def test_surface_of_a_ball_inside_the_cube_is_kept_whole():
    p = W.Problem(n=16, s=4, centres=np.array([[0.4, 0.5, 0.55]]), radii=np.array([0.2]))
    a, x, n = _area(p)
    assert abs(a - 4 * math.pi * 0.04) <= 1e-13
    # outward normal of Omega points into the ball
    assert np.allclose(n, -(x - p.centres[0]) / 0.2, atol=1e-14)


def test_ball_poking_out_of_the_cube_keeps_the_inner_zone():
    """Centre 0.05 above the face z = 0, r = 0.1: the kept surface is the
    spherical zone z in (0, 0.15], area 2 pi r (0.15).  The rule is a global
    one restricted to a region, so its error is of the order of its spacing
    (about h/4 on the sphere) relative to the zone."""
    p = W.Problem(n=32, s=4, centres=np.array([[0.5, 0.5, 0.05]]), radii=np.array([0.1]))
    a, x, _ = _area(p)
    assert np.all(x[:, 2] > 0.0)
    exact = 2 * math.pi * 0.1 * 0.15
    assert abs(a - exact) <= 0.02 * exact


def test_overlapping_balls_drop_the_cap_inside_the_other():
    """Ball 1 (r1 = 0.2) loses the cap inside ball 2 (r2 = 0.15, centres
    0.25 apart): cap height h1 = r1 - (d^2 + r1^2 - r2^2) / (2 d), area
    2 pi r1 h1; ball 2 loses its own cap likewise."""
    c = np.array([[0.4, 0.5, 0.5], [0.65, 0.5, 0.5]])
    r = np.array([0.2, 0.15])
    p = W.Problem(n=32, s=4, centres=c, radii=r)
    a, _, _ = _area(p)
    d = 0.25
    cap1 = 2 * math.pi * r[0] * (r[0] - (d * d + r[0] ** 2 - r[1] ** 2) / (2 * d))
    cap2 = 2 * math.pi * r[1] * (r[1] - (d * d + r[1] ** 2 - r[0] ** 2) / (2 * d))
    exact = 4 * math.pi * (r[0] ** 2 + r[1] ** 2) - cap1 - cap2
    assert abs(a - exact) <= 0.02 * exact


def test_surface_matrices_q1_identities():
    """sum_a N_a = 1 and sum_a grad N_a = 0: column sums of T and U vanish,
    the entries of S sum to the cell's surface weight, and S and U are
    symmetric positive semidefinite."""
    p = W.random_balls(16, 4, 6, 3)
    d = assemble.discretise(p)
    S, T, U = surface.surface_matrices(p, d.cut)
    assert np.any(S.sum(axis=(1, 2)) > 0)
    cells, x, n, w = surface.surface_points(p)
    pos = {int(c): i for i, c in enumerate(d.cut)}
    tot = np.zeros(d.cut.size)
    for c, wi in zip(cells, w):
        if int(c) in pos:
            tot[pos[int(c)]] += wi * p.n ** 2
    scale = max(1.0, tot.max())
    assert np.abs(S.sum(axis=(1, 2)) - tot).max() <= 1e-12 * scale
    assert np.abs(T.sum(axis=1)).max() <= 1e-12 * scale
    assert np.abs(U.sum(axis=1)).max() <= 1e-12 * scale
    for M in (S, U):
        assert np.abs(M - np.transpose(M, (0, 2, 1))).max() <= 1e-14 * scale
        assert np.linalg.eigvalsh(M).min() >= -1e-12 * scale


def test_surface_matrices_of_a_nearly_plane_cut():
    """A ball of radius 5 whose top (its pole) is at the centre of cell
    (1, 1) of a 4^3 mesh, at height 0.40: in cell (1, 1, 1) = [0.25, 0.5]^3
    the surface is nearly the plane xi_z = 0.6 with normal -z (into the
    ball).  Closed forms with the 1-D mass m = [[1/3, 1/6], [1/6, 1/3]] and
    Z_0 = 1 - xi, Z_1 = xi, Z'_0 = -1, Z'_1 = 1:
      S[a,b] =  m[ax,bx] m[ay,by] Z_az Z_bz,
      T[a,b] = -m[ax,bx] m[ay,by] Z'_az Z_bz,
      U[a,b] =  m[ax,bx] m[ay,by] Z'_az Z'_bz.
    The rule is only as fine as h/4 near the cell's borders (and the surface
    bends by about 0.01 over the cell), so the comparison is to 30% of the
    largest entry, which still tells every sign and the orientation of T."""
    R = 5.0
    p = W.Problem(n=4, s=2, centres=np.array([[0.375, 0.375, 0.40 - R]]), radii=np.array([R]))
    cell = 1 + 4 * (1 + 4 * 1)
    S, T, U = surface.surface_matrices(p, np.array([cell]))
    m = np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])
    c = 0.6
    Z = [1 - c, c]
    Zp = [-1.0, 1.0]
    Se, Te, Ue = np.zeros((8, 8)), np.zeros((8, 8)), np.zeros((8, 8))
    for a in range(8):
        for b in range(8):
            mm = m[a & 1, b & 1] * m[(a >> 1) & 1, (b >> 1) & 1]
            az, bz = (a >> 2) & 1, (b >> 2) & 1
            Se[a, b] = mm * Z[az] * Z[bz]
            Te[a, b] = -mm * Zp[az] * Z[bz]
            Ue[a, b] = mm * Zp[az] * Zp[bz]
    for got, want in ((S[0], Se), (T[0], Te), (U[0], Ue)):
        assert np.abs(got - want).max() <= 0.3 * np.abs(want).max(), (got, want)
    # T is not symmetric: its transpose is far from the closed form
    assert np.abs(T[0].T - Te).max() > 0.5 * np.abs(Te).max()


@pytest.mark.parametrize("seed", [3, 11])
def test_beta_makes_the_nitsche_form_coercive(seed):
    """beta_e = 2 lambda_max gives x^T A_e x >= x^T K_e x / 2 on the
    complement of the constants (Young's inequality with the bound
    x^T U x <= lambda_max x^T K x), up to the shift that bounds lambda_max
    on cells where K is singular there (alpha x^T K_ref x / 2); with an
    eighth of beta the bound fails on some cell."""
    p = W.random_balls(16, 4, 8, seed)
    d = assemble.discretise(p)
    pos = np.searchsorted(d.active, d.cut)
    K = d.Kunit[pos]
    S, T, U = surface.surface_matrices(p, d.cut)
    beta = surface.beta_unit(K, U)
    assert np.all(beta >= 0) and np.any(beta > 0)
    Q = surface._complement_basis()
    Kref = surface.reference_stiffness()

    def worst(b):
        m = np.inf
        for e in range(K.shape[0]):
            if not np.any(U[e]):
                continue
            A = K[e] + b[e] * S[e] - T[e] - T[e].T
            K7 = Q.T @ K[e] @ Q
            E = Q.T @ (A - 0.5 * K[e] + 0.5 * surface.BETA_REG * Kref) @ Q
            scale = max(np.abs(Q.T @ A @ Q).max(), np.trace(K7), 1e-300)   # rounding of the largest term
            m = min(m, np.linalg.eigvalsh(E).min() / scale)
        return m
    assert worst(beta) >= -1e-10
    assert worst(beta / 8.0) < -1e-6


def test_nitsche_problem_is_symmetric_positive_definite():
    p = W.single_ball().with_options(cut_boundary=1)
    d = assemble.discretise(p)
    A = d.A.toarray()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0
    # the surface terms changed only cut cells
    d0 = assemble.discretise(W.single_ball())
    changed = np.flatnonzero(np.abs(d.Kunit - d0.Kunit).max(axis=(1, 2)) > 0)
    assert set(d.active[changed].tolist()) <= set(d.cut.tolist())
    assert changed.size > 0
