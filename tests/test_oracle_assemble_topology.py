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
