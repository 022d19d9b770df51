"""Pins for oracle.geometry and oracle.integrate against facts fixed by the
mathematics: Gauss-rule exactness, closed-form Q1 matrices on uncut cells,
and special geometries whose kept-point sets are known by hand."""
import numpy as np
import pytest

from oracle import geometry, integrate


def test_axis_offsets_are_two_point_gauss_on_each_subcell():
    xi = geometry.axis_offsets()
    # A 2-point Gauss rule on each of 4 sub-intervals integrates x^p exactly
    # for p <= 3 (composite rule, weight 1/8 per point on [0,1]).
    for p in range(4):
        assert np.isclose((xi ** p).sum() / 8.0, 1.0 / (p + 1), rtol=0, atol=1e-15)
    # x^4 on one sub-interval is not exact: the rule is genuinely 2-point
    assert not np.isclose((xi ** 4).sum() / 8.0, 1.0 / 5, rtol=0, atol=1e-12)
    assert np.all(np.diff(xi) > 0) and xi[0] > 0 and xi[-1] < 1


def test_no_balls_all_interior_and_big_ball_all_inactive():
    st, cnt = geometry.classify(4, np.zeros((0, 3)), np.zeros(0))
    assert (st == geometry.INTERIOR).all() and (cnt == 512).all()
    st, cnt = geometry.classify(4, np.array([[0.5, 0.5, 0.5]]), np.array([1.0]))
    assert (st == geometry.INACTIVE).all() and (cnt == 0).all()


def test_plane_like_cut_counts_by_hand():
    # A ball of huge radius whose surface crosses x = x0 acts as the
    # half-space x <= x0 over the unit cube (sagitta < 3e-5).  Points with
    # x > x0 are kept; the count per cell is 64 x (#axis points beyond x0).
    n = 4
    x0 = 0.40
    R = 1.0e4
    st, cnt = geometry.classify(n, np.array([[x0 - R, 0.5, 0.5]]), np.array([R]))
    h = 1.0 / n
    xi = geometry.axis_offsets()
    for c in range(n ** 3):
        i = c % n
        beyond = sum(1 for k in range(8) if (i + xi[k]) * h > x0 + 1e-4)
        assert cnt[c] == 64 * beyond
    # x0 = 0.4 lies in cell i = 1 (0.25..0.5): that column is cut
    assert set(np.unique(st.reshape(n, n, n)[:, :, 1])) == {geometry.CUT}


def test_small_ball_at_a_node_removes_one_point_per_cell():
    # Ball at grid node (2,2,2) of an 4^3 mesh with radius 0.15 h: the
    # nearest Gauss point of each of the 8 surrounding cells is at distance
    # sqrt(3) * g0/4 * h ~ 0.0915 h, the next ones at >= 0.21 h.
    n = 4
    h = 1.0 / n
    c = np.array([[2 * h, 2 * h, 2 * h]])
    st, cnt = geometry.classify(n, c, np.array([0.15 * h]))
    near = [i + n * (j + n * k) for i in (1, 2) for j in (1, 2) for k in (1, 2)]
    for cell in range(n ** 3):
        assert cnt[cell] == (511 if cell in near else 512)


def _closed_form_q1():
    s = np.array([[1.0, -1.0], [-1.0, 1.0]])
    m = np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])
    K = np.zeros((8, 8))
    M = np.zeros((8, 8))
    for a in range(8):
        for b in range(8):
            ia = [(a >> d) & 1 for d in range(3)]
            ib = [(b >> d) & 1 for d in range(3)]
            S = [s[ia[d], ib[d]] for d in range(3)]
            Mm = [m[ia[d], ib[d]] for d in range(3)]
            K[a, b] = S[0] * Mm[1] * Mm[2] + Mm[0] * S[1] * Mm[2] + Mm[0] * Mm[1] * S[2]
            M[a, b] = Mm[0] * Mm[1] * Mm[2]
    return K, M


def test_uncut_cell_matrices_equal_closed_form():
    K, M = _closed_form_q1()
    keep = np.ones((1, 512), dtype=bool)
    Ku = integrate.unit_stiffness(keep)[0]
    Mu = integrate.unit_mass(keep)[0]
    np.testing.assert_allclose(Ku, K, rtol=0, atol=1e-15)
    np.testing.assert_allclose(Mu, M, rtol=0, atol=1e-16)
    # entries by node distance: diag 1/3, one axis apart 0, two or three -1/12
    for a in range(8):
        for b in range(8):
            nd = bin(a ^ b).count("1")
            expect = {0: 1 / 3, 1: 0.0, 2: -1 / 12, 3: -1 / 12}[nd]
            assert abs(Ku[a, b] - expect) < 1e-15


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cut_cell_invariants(seed):
    rng = np.random.default_rng(seed)
    keep = rng.uniform(size=(40, 512)) < rng.uniform(0.002, 0.9, size=(40, 1))
    keep[0] = False
    keep[0, rng.integers(512)] = True            # exactly one kept point
    K = integrate.unit_stiffness(keep)
    M = integrate.unit_mass(keep)
    for c in range(keep.shape[0]):
        k = keep[c].sum()
        np.testing.assert_allclose(K[c].sum(axis=1), 0.0, atol=1e-15)   # grad of sum N_a = 0
        np.testing.assert_allclose(K[c], K[c].T, atol=0)
        ev = np.linalg.eigvalsh(K[c])
        assert ev.min() > -1e-15
        assert np.sum(ev > 1e-13) <= min(7, 3 * k)
        # sum_ab N_a N_b = 1 at every point: total mass = kept volume fraction
        assert abs(M[c].sum() - k / 512.0) < 1e-15
    assert np.sum(np.linalg.eigvalsh(K[0]) > 1e-13) == 3


def test_cell_nodes_lexicographic():
    n = 3
    nodes = integrate.cell_nodes(n, np.array([0, n ** 3 - 1]))
    n1 = n + 1
    assert nodes[0].tolist() == [0, 1, n1, n1 + 1, n1 * n1, n1 * n1 + 1,
                                 n1 * n1 + n1, n1 * n1 + n1 + 1]
    assert nodes[1, 7] == n1 ** 3 - 1
