"""Pins of the oracle's manufactured-solution part (oracle/manufactured.py,
paper Sect. 5.1): the exact solution against finite differences, linear
solutions that Q1 reproduces exactly, the Neumann surface load of a ball
concentric with the radial solution against its closed form, the Nitsche
data terms against the surface matrices, and the convergence rates of the
discretisation error."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import assemble, manufactured as mm, surface


def _linear(a, c):
    a = np.asarray(a, dtype=np.float64)

    def sol(x):
        x = np.asarray(x, dtype=np.float64)
        m = x.shape[0]
        return x @ a + c, np.tile(a, (m, 1)), np.zeros(m)
    return sol


def _solve(problem, sol):
    d = assemble.discretise(problem)
    b = mm.load(problem, d, sol)
    u, info = spla.cg(d.A, b, rtol=1e-14, maxiter=5000, M=sp.diags(1.0 / d.A.diagonal()))
    assert info == 0
    return d, u


def test_exact_solution_against_finite_differences():
    rng = np.random.default_rng(5)
    x = rng.uniform(0.1, 0.9, size=(20, 3))
    k = 5.0 * np.pi
    x0 = np.array([0.05, -0.1, 0.2])
    u, g, f = mm.exact(x, x0, k)
    assert np.allclose(u, np.sin(k * np.linalg.norm(x - x0, axis=1)), atol=1e-15)
    hs = 1e-5
    lap = np.zeros(20)
    for a in range(3):
        e = np.zeros(3)
        e[a] = hs
        up = mm.exact(x + e, x0, k)[0]
        um = mm.exact(x - e, x0, k)[0]
        assert np.abs((up - um) / (2 * hs) - g[:, a]).max() <= 1e-6 * k
        e[a] = 1e-4
        lap += (mm.exact(x + e, x0, k)[0] - 2 * u + mm.exact(x - e, x0, k)[0]) / 1e-8
    assert np.abs(-lap - f).max() <= 1e-4 * k * k


def test_linear_solution_is_reproduced_on_the_uncut_cube():
    """f = 0 and u linear: the Q1 solution with the lifted face values is the
    nodal interpolant, and both errors vanish."""
    p = W.uncut(8, 4)
    sol = _linear([0.7, -1.3, 0.4], 0.25)
    d, u = _solve(p, sol)
    n1 = p.n + 1
    g = d.dof_node
    xn = np.stack([g % n1, (g // n1) % n1, g // (n1 * n1)], axis=1) / p.n
    assert np.abs(u - sol(xn)[0]).max() <= 1e-13
    l2, h1 = mm.errors(p, d, u, sol)
    assert l2 <= 1e-14 and h1 <= 1e-13


def test_lift_holds_the_face_values_only():
    p = W.uncut(4, 2)
    ud = mm.lift(p, _linear([1.0, 2.0, 3.0], 0.0))
    n1 = p.n + 1
    gid = np.arange(n1 ** 3)
    I, J, K = gid % n1, (gid // n1) % n1, gid // (n1 * n1)
    face = (I == 0) | (I == 4) | (J == 0) | (J == 4) | (K == 0) | (K == 4)
    assert np.allclose(ud[face], (I + 2 * J + 3 * K)[face] / 4.0, atol=1e-15)
    assert not ud[~face].any()


def test_neumann_load_of_a_concentric_ball_has_the_closed_form():
    """u = sin(k |x - c|) around the ball's own centre c: on its sphere
    grad u . n = -k cos(k r) everywhere (n points into the ball), so the
    corner loads sum to -k cos(k r) 4 pi r^2 and, the Q1 shape functions
    reproducing linear functions, their first moment about the nodes is
    that total times c."""
    c = np.array([0.5, 0.5, 0.5])
    r, k = 0.3, 2.0 * np.pi
    p = W.Problem(n=16, s=4, centres=c[None, :], radii=np.array([r]))
    d = assemble.discretise(p)
    sc, sl = mm.surface_load(p, d, mm.radial(c, k))
    total = -k * math.cos(k * r) * 4.0 * math.pi * r * r
    assert abs(sl.sum() - total) <= 1e-12 * abs(total)
    n1 = p.n + 1
    nodes = assemble.integrate.cell_nodes(p.n, sc)
    xn = np.stack([nodes % n1, (nodes // n1) % n1, nodes // (n1 * n1)], axis=2) / p.n
    moment = (sl[:, :, None] * xn).sum(axis=(0, 1))
    assert np.abs(moment - total * c).max() <= 1e-12 * abs(total)


def test_nitsche_data_terms_equal_the_surface_matrices_on_q1_data():
    """For Dirichlet data u that is trilinear on every cell, the data terms
    sum w (beta N_a - n . grad N_a) u equal h (beta S - T) u_e."""
    p = W.single_ball(8, 4).with_options(cut_boundary=W.CUT_NITSCHE)
    d = assemble.discretise(p)
    sol = _linear([0.3, -0.8, 1.1], -0.2)
    sc, sl = mm.surface_load(p, d, sol)
    assert np.array_equal(sc, d.cut)
    keep = assemble.keep_masks(p, d.cut)
    S, T, U = surface.surface_matrices(p, d.cut)
    # the cut cells' volume stiffness without the Nitsche terms
    beta = surface.beta_unit(assemble.integrate.unit_stiffness(keep), U)
    n1 = p.n + 1
    nodes = assemble.integrate.cell_nodes(p.n, d.cut)
    xn = np.stack([nodes % n1, (nodes // n1) % n1, nodes // (n1 * n1)], axis=2) / p.n
    ue = sol(xn.reshape(-1, 3))[0].reshape(-1, 8)
    want = (1.0 / p.n) * np.einsum("eab,eb->ea", beta[:, None, None] * S - T, ue)
    assert np.abs(sl - want).max() <= 1e-12 * np.abs(want).max()


def _rates(problem_of_n, ns, sol):
    errs = []
    for n in ns:
        p = problem_of_n(n)
        d, u = _solve(p, sol)
        errs.append(mm.errors(p, d, u, sol))
    e = np.array(errs)
    return np.log2(e[:-1] / e[1:]), e


def test_neumann_data_reach_sphere_points_outside_cut_cells():
    """Sphere points in cells that the volume rule classifies interior or
    inactive keep their flux: the corner loads of the concentric ball sum to
    the whole sphere's flux on a mesh where some points lie in such cells."""
    c = np.array([0.51, 0.52, 0.49])
    r, k = 0.3, 2.0 * np.pi
    p = W.Problem(n=32, s=8, centres=c[None, :], radii=np.array([r]))
    d = assemble.discretise(p)
    cells = surface.surface_points(p)[0]
    assert not np.isin(cells, d.cut).all()      # premise: such points exist here
    sc, sl = mm.surface_load(p, d, mm.radial(c, k))
    total = -k * math.cos(k * r) * 4.0 * math.pi * r * r
    assert abs(sl.sum() - total) <= 1e-12 * abs(total)


def test_rates_on_the_uncut_cube():
    rates, e = _rates(lambda n: W.uncut(n, 4), (8, 16), mm.radial(k=np.pi))
    assert rates[-1, 0] >= 1.9 and rates[-1, 1] >= 0.95, (rates, e)


@pytest.mark.parametrize("boundary", [W.CUT_NEUMANN, W.CUT_NITSCHE])
def test_rates_with_a_ball(boundary):
    """Single ball inside the cube, sin(pi |x|): optimal rates (L2 ~ h^2,
    H1 ~ h) between 8^3 and 16^3 cells."""
    def prob(n):
        return W.single_ball(n, 4).with_options(cut_boundary=boundary)
    rates, e = _rates(prob, (8, 16), mm.radial(k=np.pi))
    assert rates[-1, 0] >= 1.8 and rates[-1, 1] >= 0.9, (rates, e)


def test_planted_sign_error_in_the_neumann_data_breaks_convergence(monkeypatch):
    """The rate test above fails when the Neumann data takes the wrong sign."""
    orig = mm.surface_load

    def flipped(problem, d, sol=None):
        sc, sl = orig(problem, d, sol)
        return sc, -sl
    monkeypatch.setattr(mm, "surface_load", flipped)
    rates, e = _rates(lambda n: W.single_ball(n, 4), (8, 16), mm.radial(k=np.pi))
    assert not (rates[-1, 0] >= 1.8 and rates[-1, 1] >= 0.9)
