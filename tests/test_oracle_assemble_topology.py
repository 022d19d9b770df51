"""Pins for oracle.assemble and oracle.topology: the Q1 Laplacian stencil on
uncut meshes, the load of a constant source, object counts of uniform
partitions, and the variant-1 edge classification on hand-made geometry."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import assemble, topology

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_uncut_global_stencil_and_constant_load():
    p = W.uncut(6, 3)
    d = assemble.discretise(p)
    n, h = p.n, 1.0 / p.n
    assert d.n_dof == (n - 1) ** 3
    A = d.A.toarray()
    n1 = n + 1
    centre = d.dof_of_node[3 + n1 * (3 + n1 * 3)]
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                other = d.dof_of_node[(3 + di) + n1 * ((3 + dj) + n1 * (3 + dk))]
                nd = abs(di) + abs(dj) + abs(dk)
                expect = {0: 8 * h / 3, 1: 0.0, 2: -h / 6, 3: -h / 12}[nd]
                assert abs(A[centre, other] - expect) < 1e-15
    b = assemble.load(d, None)
    # integral of each interior hat function = h^3
    np.testing.assert_allclose(b, h ** 3, rtol=1e-14)
    # A is SPD on the uncut mesh
    assert np.linalg.eigvalsh(A).min() > 0


def test_dof_numbering_is_ascending_node_order():
    d = assemble.discretise(W.single_ball())
    assert np.all(np.diff(d.dof_node) > 0)
    assert np.all(d.dof_of_node[d.dof_node] == np.arange(d.n_dof))


def test_floating_pocket_detected():
    # Balls packed on a sphere around the cube centre seal a cavity whose
    # active cells touch no cube face.
    rng = np.random.default_rng(0)
    dirs = rng.standard_normal((400, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    centres = 0.5 + 0.3 * dirs
    radii = np.full(400, 0.12)
    p = W.Problem(n=16, s=4, centres=centres, radii=radii)
    d = assemble.discretise(p, check_floating=False)
    assert assemble.floating_components(d) >= 1
    with pytest.raises(assemble.SingularProblem):
        assemble.discretise(p)
    assert assemble.floating_components(assemble.discretise(W.single_ball())) == 0


@pytest.mark.parametrize("n,s", [(6, 3), (9, 3), (8, 4), (12, 4)])
def test_uncut_object_counts(n, s):
    p = W.uncut(n, s)
    d = assemble.discretise(p)
    t = topology.build(p, d)
    m = n // s
    counts = np.bincount(t.obj_type, minlength=3)
    assert counts[topology.CORNER] == (m - 1) ** 3
    assert counts[topology.EDGE] == 3 * m * (m - 1) ** 2
    assert counts[topology.FACE] == 3 * m * m * (m - 1)
    # every edge holds s-1 DOFs and every face (s-1)^2
    sizes = np.diff(t.obj_ptr)
    assert set(sizes[t.obj_type == topology.EDGE].tolist()) == {s - 1}
    assert set(sizes[t.obj_type == topology.FACE].tolist()) == {(s - 1) ** 2}
    # objects partition the interface DOFs and are ordered by smallest DOF
    iface = np.flatnonzero(t.card() >= 2)
    assert np.array_equal(np.sort(t.obj_dofs), iface)
    firsts = t.obj_dofs[t.obj_ptr[:-1]]
    assert np.all(np.diff(firsts) > 0)
    # faces have two subdomains, edges four, corners eight
    for o, S in enumerate(t.obj_S):
        assert len(S) == {topology.FACE: 2, topology.EDGE: 4, topology.CORNER: 8}[t.obj_type[o]]
    assert t.n_coarse == counts.sum()


def test_uncut_s2_every_object_is_a_corner():
    # with s = 2 every edge and face of the partition holds a single DOF
    p = W.uncut(6, 2)
    t = topology.build(p, assemble.discretise(p))
    m = 3
    assert (t.obj_type == topology.CORNER).all()
    assert t.obj_type.size == (m - 1) ** 3 + 3 * m * (m - 1) ** 2 + 3 * m * m * (m - 1)


def test_table1_subdomain_shape():
    """Table 1: at H/h = 8 a subdomain holds at most 512 cells and 729 DOFs."""
    vals = {}
    with open(os.path.join(GOLDEN, "table1_subdomain_shape.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = int(v)
    p = W.uncut(24, 8)
    d = assemble.discretise(p)
    t = topology.build(p, d)
    assert max(c.size for c in t.sub_cells) == vals["max_cells_per_subdomain"]
    # the centre block touches no cube face: all (s+1)^3 of its nodes are DOFs
    assert max(x.size for x in t.sub_dofs) == vals["max_dofs_per_subdomain"]
    assert p.n // (p.n // p.s) == vals["H_over_h"]


def test_single_ball_centre_corner_missing():
    # The only cross-point of the 2x2x2 partition is (0.5, 0.5, 0.5), inside
    # the ball: it is not a DOF and no 8-subdomain corner exists.
    p = W.single_ball().with_options(coarse_variant=0)
    d = assemble.discretise(p)
    assert d.dof_of_node[4 + 9 * (4 + 9 * 4)] == -1
    t = topology.build(p, d)
    assert all(len(S) < 8 for S in t.obj_S)
    pu = W.uncut(8, 4)
    tu = topology.build(pu, assemble.discretise(pu))
    assert sum(1 for S in tu.obj_S if len(S) == 8) == 1 and tu.n_coarse == 19


def test_segment_classification_cases():
    n = 10
    h = 0.1
    c = np.array([[0.55, 0.5, 0.5]])
    # segment x in [0.5, 0.6] at y = z = 0.5 inside a ball of radius 0.3
    assert topology.segment_class(n, (5, 5, 5), 0, c, np.array([0.3])) == 1
    # far away
    assert topology.segment_class(n, (0, 0, 0), 0, c, np.array([0.3])) == 0
    # ball surface crosses the segment (radius 0.02 around its midpoint)
    assert topology.segment_class(n, (5, 5, 5), 0, c, np.array([0.02])) == 2
    # tangent from outside: distance exactly > r keeps it interior
    c2 = np.array([[0.55, 0.5 + 0.05, 0.5]])
    assert topology.segment_class(n, (5, 5, 5), 0, c2, np.array([0.049])) == 0
    # two overlapping balls cover the segment; two with a gap do not
    cc = np.array([[0.5, 0.5, 0.5], [0.6, 0.5, 0.5]])
    assert topology.segment_class(n, (5, 5, 5), 0, cc, np.array([0.06, 0.06])) == 1
    assert topology.segment_class(n, (5, 5, 5), 0, cc, np.array([0.04, 0.04])) == 2
    # along z, same geometry rotated
    cz = np.array([[0.5, 0.5, 0.55]])
    assert topology.segment_class(n, (5, 5, 5), 2, cz, np.array([0.3])) == 1
    assert topology.segment_class(n, (5, 5, 5), 2, cz, np.array([0.02])) == 2
    _ = h


def test_variant1_splits_cut_edges_into_corners():
    # A small ball sitting on the block edge x = y = 0.5 (z-line) of a 2x2x1
    # style partition cuts FE edges on that coarse edge.
    p = W.Problem(n=8, s=4, centres=np.array([[0.5, 0.5, 0.45]]),
                  radii=np.array([0.08]), coarse_variant=0)
    d = assemble.discretise(p)
    t0 = topology.build(p, d)
    t1 = topology.build(p.with_options(coarse_variant=1), d)
    assert t1.n_coarse > t0.n_coarse
    # every DOF of a cut FE edge of a standard edge object is a corner in v1
    n1 = p.n + 1
    corner_dofs = set(t1.obj_dofs[t1.obj_ptr[:-1][t1.obj_type == topology.CORNER]].tolist())
    found_cut = False
    for o, dofs in enumerate(t0.objects()):
        if t0.obj_type[o] != topology.EDGE:
            continue
        for a in dofs:
            for b in dofs:
                na, nb = d.dof_node[a], d.dof_node[b]
                diff = nb - na
                if diff not in (1, n1, n1 * n1):
                    continue
                axis = (1, n1, n1 * n1).index(diff)
                ijk = (na % n1, (na // n1) % n1, na // (n1 * n1))
                if topology.segment_class(p.n, ijk, axis, p.centres, p.radii) == 2:
                    found_cut = True
                    assert a in corner_dofs and b in corner_dofs
    assert found_cut
    # the split objects still partition the interface
    assert np.array_equal(np.sort(t1.obj_dofs), np.flatnonzero(t1.card() >= 2))


# ---- hand-made cut partitions: the link and face rules of Sect. 3.2 ----------
#
# The objects below are written out by hand, not computed by the oracle.  On an
# uncut mesh with 2 x 2 x 2 blocks of s^3 cells (block planes at index s), an
# interface node belongs to the object given by which of its coordinates equal
# s and, for the others, on which side of s they lie; three coordinates at s
# make the corner, two an edge, one a face.

def _uncut_two_block_objects(n, s):
    objs = {}
    for K in range(1, n):
        for J in range(1, n):
            for I in range(1, n):
                key = tuple("s" if v == s else ("lo" if v < s else "hi") for v in (I, J, K))
                n_at = key.count("s")
                if n_at == 0:
                    continue
                objs.setdefault(key, set()).add((I, J, K))
    typ = {3: topology.CORNER, 2: topology.EDGE, 1: topology.FACE}
    return {frozenset(v): typ[k.count("s")] for k, v in objs.items()}


def _oracle_objects(p, count):
    d = assemble.discretise(p, count=count)
    t = topology.build(p, d)
    n1 = p.n + 1
    got = {}
    for o, dofs in enumerate(t.objects()):
        nodes = d.dof_node[dofs]
        key = frozenset((int(g % n1), int((g // n1) % n1), int(g // (n1 * n1))) for g in nodes)
        got[key] = int(t.obj_type[o])
    return d, t, got


def _counts(n, inactive):
    c = np.full(n ** 3, 512, dtype=np.int32)
    for (i, j, k) in inactive:
        c[i + n * (j + n * k)] = 0
    return c


def test_hand_cut_partition_breaks_links():
    """n = 8, s = 4.  The column of cells (3, 1, k), k = 0..3, of subdomain 0
    is removed.  Every node of the face x = 0.5 (I = 4) between subdomains 0
    and 1 keeps S = {0, 1} (cells (3, 0, k) and (3, 2, k) stay), but the FE
    edges from row J = 1 to row J = 2 of that face lie only in removed cells
    on the subdomain-0 side, so they link nothing: the face splits into the
    3-node line J = 1 (an edge: it holds no mesh face) and a 6-node face.  The
    same happens on the coarse edge I = 4, K = 4 (S = {0, 1, 4, 5}): its FE
    edge from J = 1 to J = 2 lies in cell (3, 1, 3) of subdomain 0 only, so
    node (4, 1, 4) becomes a corner and (4, 2, 4)-(4, 3, 4) an edge."""
    n, s = 8, 4
    p = W.uncut(n, s)
    count = _counts(n, [(3, 1, k) for k in range(4)])
    expect = _uncut_two_block_objects(n, s)
    face = frozenset((4, J, K) for J in (1, 2, 3) for K in (1, 2, 3))
    edge = frozenset((4, J, 4) for J in (1, 2, 3))
    assert expect.pop(face) == topology.FACE and expect.pop(edge) == topology.EDGE
    expect[frozenset((4, 1, K) for K in (1, 2, 3))] = topology.EDGE
    expect[frozenset((4, J, K) for J in (2, 3) for K in (1, 2, 3))] = topology.FACE
    expect[frozenset({(4, 1, 4)})] = topology.CORNER
    expect[frozenset({(4, 2, 4), (4, 3, 4)})] = topology.EDGE
    d, t, got = _oracle_objects(p, count)
    assert d.n_dof == (n - 1) ** 3          # every node is still in an active cell
    assert got == expect
    assert t.n_coarse == len(expect) == 21
    # objects ordered by their smallest DOF, coarse ids in that order (cef)
    firsts = t.obj_dofs[t.obj_ptr[:-1]]
    assert np.all(np.diff(firsts) > 0)
    assert np.array_equal(t.coarse_of_obj, np.arange(len(expect)))
    # S of the split face's nodes is still {0, 1}
    n1 = n + 1
    for J in (1, 2, 3):
        for K in (1, 2, 3):
            assert t.S(d.dof_of_node[4 + n1 * (J + n1 * K)]) == (0, 1)


def test_hand_cut_partition_face_needs_two_active_cells():
    """n = 6, s = 3.  Cell (2, 1, 1) of subdomain 0 is removed.  The 2 x 2
    interface nodes (3, J, K), J, K in {1, 2}, stay linked (each of their FE
    edges also lies in another active cell of subdomain 0), but the only mesh
    face among them has the removed cell on one side, so the object is an
    edge, not a face.  All other objects are those of the uncut mesh."""
    n, s = 6, 3
    p = W.uncut(n, s)
    count = _counts(n, [(2, 1, 1)])
    expect = _uncut_two_block_objects(n, s)
    key = frozenset((3, J, K) for J in (1, 2) for K in (1, 2))
    assert expect[key] == topology.FACE
    expect[key] = topology.EDGE
    _, t, got = _oracle_objects(p, count)
    assert got == expect
    # BDDC(ce) drops faces only: the demoted object keeps its coarse DOF
    _, t_ce, _ = _oracle_objects(p.with_options(objects=1), count)
    assert t_ce.n_coarse == sum(1 for v in expect.values() if v != topology.FACE)


# ---- the load b = M_cut f for a non-constant source ---------------------------

def test_load_of_tensor_product_source_on_uncut_mesh():
    """Uncut mesh, nodal source f(I, J, K) = a_I b_J c_K.  Its Q1 interpolant
    is a product of 1-D piecewise-linear functions, and so is every hat
    function, so b_i = int f phi_i = h^3 (w * a)_I (w * b)_J (w * c)_K with the
    1-D mass stencil w = (1, 4, 1) / 6 (per unit length).  Exact in the
    kept-point rule (degree <= 2 per axis); any exchange of a cell's local
    nodes between the source and the test function breaks it."""
    n = 6
    h = 1.0 / n
    rng = np.random.default_rng(3)
    a, bb, c = rng.uniform(0.5, 2.0, (3, n + 1))
    n1 = n + 1
    f = (a[None, None, :] * bb[None, :, None] * c[:, None, None]).ravel()
    p = W.uncut(n, 3)
    d = assemble.discretise(p)
    b = assemble.load(d, f)

    def w(v, i):
        return (v[i - 1] + 4.0 * v[i] + v[i + 1]) / 6.0

    for dof, g in enumerate(d.dof_node):
        I, J, K = g % n1, (g // n1) % n1, g // (n1 * n1)
        expect = h ** 3 * w(a, I) * w(bb, J) * w(c, K)
        assert abs(b[dof] - expect) <= 1e-15 * abs(expect), (I, J, K)


def test_load_on_cut_mesh_by_global_hats():
    """Cut mesh (n = 4, one ball), arbitrary nodal source: b_i equals the sum,
    over every kept point x_q of every active cell, of (h^3 / 512) phi_i(x_q)
    f_h(x_q), where phi_i and f_h are evaluated from the global tent functions
    prod_d max(0, 1 - |x_d - X_d| / h) at the physical point (no element-local
    node numbering).  Brute force over all nodes."""
    from oracle import geometry
    n = 4
    h = 1.0 / n
    p = W.Problem(n=n, s=2, centres=np.array([[0.45, 0.6, 0.4]]), radii=np.array([0.33]))
    d = assemble.discretise(p)
    assert d.cut.size > 0
    rng = np.random.default_rng(5)
    n1 = n + 1
    f = rng.uniform(-1.0, 1.0, n1 ** 3)
    b = assemble.load(d, f)
    X = geometry.axis_coords(n)                     # (n, 8) physical coordinates
    keep = geometry.kept_points(n, p.centres, p.radii, d.active)
    grid = np.arange(n1) * h
    expect = np.zeros(n1 ** 3)
    for t, cell in enumerate(d.active):
        i, j, k = cell % n, (cell // n) % n, cell // (n * n)
        q = np.flatnonzero(keep[t])
        px = X[i][q % 8]
        py = X[j][(q // 8) % 8]
        pz = X[k][q // 64]
        tx = np.maximum(0.0, 1.0 - np.abs(px[:, None] - grid[None, :]) / h)   # (nq, n1)
        ty = np.maximum(0.0, 1.0 - np.abs(py[:, None] - grid[None, :]) / h)
        tz = np.maximum(0.0, 1.0 - np.abs(pz[:, None] - grid[None, :]) / h)
        phi = (tz[:, :, None, None] * ty[:, None, :, None] * tx[:, None, None, :]).reshape(q.size, -1)
        fq = phi @ f
        expect += (h ** 3 / 512.0) * (phi * fq[:, None]).sum(axis=0)
    np.testing.assert_allclose(b, expect[d.dof_node], rtol=1e-13, atol=1e-16)


# ---- variant 2 (Sect. 4.5): edges split where the weighting coefficient changes ----
#
# On an uncut 8^3 mesh with 2 x 2 x 2 blocks of 4^3 cells, every uncut cell
# has the same diagonal stiffness entries, so a node's stiffness weight on
# subdomain w is proportional to the sum of kappa over the cells of w that
# contain it.  The nodes (4, 4, K), K = 1..3, form the coarse edge shared by
# the four lower subdomains 0..3; node (4, 4, K) lies in the cell layers K-1
# and K.  Raising kappa in one layer of subdomain 0's cells changes the
# coefficients of the edge nodes that touch that layer and no others: the
# expected objects below are the standard ones with that edge re-split by
# hand.  No other edge node touches layers 0-2 of subdomain 0.

def _kappa_layer(n, s, layer, value):
    kap = np.ones(n ** 3)
    for j in range(s):
        for i in range(s):
            kap[i + n * (j + n * layer)] = value
    return kap


def _objects_of(p):
    d = assemble.discretise(p)
    t = topology.build(p, d)
    n1 = p.n + 1
    got = {}
    for o, dofs in enumerate(t.objects()):
        nodes = d.dof_node[dofs]
        key = frozenset((int(g % n1), int((g // n1) % n1), int(g // (n1 * n1))) for g in nodes)
        got[key] = int(t.obj_type[o])
    return d, t, got


@pytest.mark.parametrize("layer,corners,edge", [
    (0, [1], [2, 3]),     # (4,4,1) sees kappa 10 + 1, the others 1 + 1
    (1, [3], [1, 2]),     # (4,4,1) and (4,4,2) both see 1 + 10; (4,4,3) sees 1 + 1
    (2, [1], [2, 3]),     # (4,4,2) and (4,4,3) both see 10 + 1; (4,4,1) sees 1 + 1
])
def test_variant2_splits_edge_at_coefficient_changes(layer, corners, edge):
    n, s = 8, 4
    p = W.uncut(n, s).with_options(kappa=_kappa_layer(n, s, layer, 10.0), coarse_variant=2)
    expect = _uncut_two_block_objects(n, s)
    assert expect.pop(frozenset((4, 4, K) for K in (1, 2, 3))) == topology.EDGE
    for K in corners:
        expect[frozenset({(4, 4, K)})] = topology.CORNER
    expect[frozenset((4, 4, K) for K in edge)] = topology.EDGE
    d, t, got = _objects_of(p)
    assert got == expect
    assert t.n_coarse == len(expect)
    # the standard objects of the same problem are the uncut two-block ones
    _, _, got0 = _objects_of(p.with_options(coarse_variant=0))
    assert got0 == _uncut_two_block_objects(n, s)


def test_variant2_three_distinct_coefficients_give_three_corners():
    """kappa 10 in layer 0 and 100 in layer 1 of subdomain 0: the nodes
    (4,4,1), (4,4,2), (4,4,3) see 10 + 100, 100 + 1 and 1 + 1: all three
    coefficients differ, so the edge becomes three corners."""
    n, s = 8, 4
    kap = _kappa_layer(n, s, 0, 10.0) * _kappa_layer(n, s, 1, 100.0)
    p = W.uncut(n, s).with_options(kappa=kap, coarse_variant=2)
    expect = _uncut_two_block_objects(n, s)
    expect.pop(frozenset((4, 4, K) for K in (1, 2, 3)))
    for K in (1, 2, 3):
        expect[frozenset({(4, 4, K)})] = topology.CORNER
    assert _objects_of(p)[2] == expect


def test_variant2_is_standard_with_constant_coefficients():
    """Topological weights are 1/|S| on every object, and on an uncut mesh
    with constant kappa every edge node has two equal cells per subdomain:
    in both cases variant 2 keeps the standard objects."""
    cut = W.random_balls(16, 4, 6, 3)
    for p in (cut.with_options(weighting=0), W.uncut(12, 4)):
        _, t0, got0 = _objects_of(p.with_options(coarse_variant=0))
        _, t2, got2 = _objects_of(p.with_options(coarse_variant=2))
        assert got2 == got0


def test_variant2_refines_the_standard_edges():
    """On cut meshes with stiffness weights variant 2 only splits edges:
    faces and corners are the standard ones, every new object lies in one
    standard edge, and the objects still partition the interface."""
    for p in (W.random_balls(16, 4, 6, 3), W.single_ball(), W.random_balls(24, 8, 10, 4)):
        d, t0, got0 = _objects_of(p.with_options(coarse_variant=0))
        _, t2, got2 = _objects_of(p.with_options(coarse_variant=2))
        std_edges = [k for k, v in got0.items() if v == topology.EDGE]
        for k, v in got2.items():
            if k in got0 and got0[k] == v:
                continue
            assert v in (topology.CORNER, topology.EDGE)
            assert sum(k <= e for e in std_edges) == 1
        for k, v in got0.items():
            if v != topology.EDGE:
                assert got2.get(k) == v
        assert np.array_equal(np.sort(t2.obj_dofs), np.flatnonzero(t2.card() >= 2))


def test_variant2_counts_only_active_cells_of_each_subdomain():
    """Cell (3, 3, 0) of subdomain 0 removed (hand-made cell data): node
    (4, 4, 1) then lies in one active cell of subdomain 0 and two of each of
    subdomains 1-3, (4, 4, 2) and (4, 4, 3) in two of each.  The standard
    edge {(4,4,K)} stays whole (its links still lie in active cells of all
    four subdomains); variant 2 makes (4, 4, 1) a corner."""
    n, s = 8, 4
    count = _counts(n, [(3, 3, 0)])
    p = W.uncut(n, s).with_options(coarse_variant=2)
    _, _, got0 = _oracle_objects(p.with_options(coarse_variant=0), count)
    assert got0 == _uncut_two_block_objects(n, s)
    _, _, got2 = _oracle_objects(p, count)
    expect = _uncut_two_block_objects(n, s)
    expect.pop(frozenset((4, 4, K) for K in (1, 2, 3)))
    expect[frozenset({(4, 4, 1)})] = topology.CORNER
    expect[frozenset({(4, 4, 2), (4, 4, 3)})] = topology.EDGE
    assert got2 == expect


@pytest.mark.parametrize("corner,splits", [(7, True), (0, False), (6, False)])
def test_variant2_uses_the_nodes_own_diagonal_entry(corner, splits):
    """Uncut 8^3 mesh; the diagonal entry K_e[corner, corner] of cell
    (3, 3, 0) (subdomain 0) is tripled by hand in the discretisation.  Node
    (4, 4, 1) is corner 7 of that cell (local node a = ix + 2 iy + 4 iz with
    offsets (1, 1, 1)), so only corner 7 changes its coefficient and splits
    the edge; corner 0 is node (3, 3, 0) on the cube face (not a DOF) and
    corner 6 is node (3, 4, 1) of a face object (faces are never split)."""
    n, s = 8, 4
    p = W.uncut(n, s).with_options(coarse_variant=2)
    d = assemble.discretise(p)
    pos = int(np.searchsorted(d.active, 3 + n * (3 + n * 0)))
    d.Kunit[pos, corner, corner] *= 3.0
    t = topology.build(p, d)
    n1 = n + 1
    node1 = d.dof_of_node[4 + n1 * (4 + n1 * 1)]
    o = [k for k, dofs in enumerate(t.objects()) if node1 in dofs][0]
    assert (t.obj_type[o] == topology.CORNER) == splits
