"""Pins for oracle.bddc, oracle.pcg and oracle.adjoint against what the
mathematics fixes: partition of unity of the weights, the coarse basis
identities, symmetry and the lower eigenvalue 1 of M A (Sect. 3.4, proof of
the theorem), the limits M = A^{-1} (one subdomain; all interface DOFs as
corners, Sect. 4.2's enlarged coarse space), sparse direct solves, and
finite differences for the gradient."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import OracleSolver, assemble, topology, bddc, pcg, adjoint


def _dense_M(s):
    nd = s.n_dof
    return np.column_stack([s.M.apply(e) for e in np.eye(nd)])


@pytest.mark.parametrize("weighting", [0, 1])
def test_weights_partition_of_unity(weighting):
    p = W.random_balls(8, 4, 3, 7).with_options(weighting=weighting)
    s = OracleSolver(p)
    total = np.zeros(s.n_dof)
    for sw in s.M.subs:
        if sw is not None:
            total[sw.dofs] += sw.D
    cnt = np.zeros(s.n_dof)
    for sw in s.M.subs:
        if sw is not None:
            cnt[sw.dofs] += 1
    np.testing.assert_allclose(total, 1.0, rtol=0, atol=1e-15)


def test_stiffness_equals_cardinality_on_uncut_constant_kappa():
    p = W.uncut(8, 4)
    s1 = OracleSolver(p.with_options(weighting=1))
    s0 = OracleSolver(p.with_options(weighting=0))
    for a, b in zip(s1.M.subs, s0.M.subs):
        np.testing.assert_allclose(a.D, b.D, rtol=1e-15, atol=0)  # 1 ulp


def test_coarse_basis_identities_on_floating_subdomain():
    # 12^3 uncut mesh with 3^3 subdomains: the centre block is floating.
    p = W.uncut(12, 4)
    s = OracleSolver(p)
    w = 13
    sw = s.M.subs[w]
    np.testing.assert_allclose(sw.A @ np.ones(sw.dofs.size), 0.0, atol=1e-14)
    np.testing.assert_allclose(sw.C @ sw.Phi, np.eye(sw.C.shape[0]), atol=1e-12)
    np.testing.assert_allclose(sw.Phi.sum(axis=1), 1.0, atol=1e-12)


@pytest.mark.parametrize("make", [
    lambda: W.single_ball(),
    lambda: W.single_ball().with_options(weighting=0, coarse_variant=0),
    lambda: W.random_balls(8, 4, 4, 11, lognormal_kappa=True),
])
def test_M_symmetric_and_lambda_min_one(make):
    s = OracleSolver(make())
    M = _dense_M(s)
    A = s.d.A.toarray()
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
    # eigenvalues of M A = those of A^{1/2} M A^{1/2}: real, >= 1, with
    # lambda_min = 1 reached on (at least) the interior bubble space
    L = np.linalg.cholesky(A)
    ev = np.linalg.eigvalsh(L.T @ M @ L)
    n_I = int((s.topo.card() == 1).sum())
    assert ev.min() > 1 - 1e-9
    assert np.sum(np.abs(ev - 1) < 1e-8) >= n_I


def test_one_subdomain_gives_exact_inverse():
    p = W.random_balls(8, 8, 3, 5)
    s = OracleSolver(p)
    assert s.topo.n_sub == 1 and s.topo.n_coarse == 0
    M = _dense_M(s)
    np.testing.assert_allclose(M @ s.d.A.toarray(), np.eye(s.n_dof), atol=1e-10)
    b = s.rhs()
    x, it, rel = s.solve_rhs(b)
    assert it == 1 and rel < 1e-12


def test_all_interface_corners_gives_exact_inverse():
    # Enlarged coarse space of Sect. 4.2 in its limit: every interface DOF
    # is its own corner, so the BDDC space is the continuous space.
    p = W.single_ball()
    d = assemble.discretise(p)
    t = topology.build(p, d)
    iface = np.flatnonzero(t.card() >= 2)
    t.obj_ptr = np.arange(iface.size + 1)
    t.obj_dofs = iface.copy()
    t.obj_type = np.zeros(iface.size, dtype=np.int8)
    t.obj_S = [t.S(x) for x in iface]
    t.coarse_of_obj = np.arange(iface.size, dtype=np.int32)
    t.n_coarse = iface.size
    M = bddc.BDDC(d, t, stiffness=True)
    Md = np.column_stack([M.apply(e) for e in np.eye(d.n_dof)])
    np.testing.assert_allclose(Md @ d.A.toarray(), np.eye(d.n_dof), atol=1e-9)


@pytest.mark.parametrize("make", [
    lambda: W.single_ball(),
    lambda: W.random_balls(16, 4, 6, 3),
    lambda: W.random_balls(24, 8, 8, 4, lognormal_kappa=True),
])
def test_pcg_matches_sparse_direct(make):
    s = OracleSolver(make())
    b = s.rhs()
    x, it, rel = s.solve_rhs(b, rtol=1e-10)
    xd = spla.spsolve(s.d.A.tocsc(), b)
    assert rel < 1e-10
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-8
    # the recursive residual agrees with the true residual
    assert np.linalg.norm(b - s.d.A @ x) / np.linalg.norm(b) < 1e-9
    lmin, lmax = pcg.lanczos_condition(*s.last_coeffs)
    assert lmin > 1 - 1e-6 and lmax < 50


def test_pcg_zero_rhs_and_iteration_cap():
    s = OracleSolver(W.single_ball())
    x, it, rel = s.solve_rhs(np.zeros(s.n_dof))
    assert it == 0 and not x.any()
    x, it, rel, _, _ = pcg.pcg(lambda v: s.d.A @ v, lambda v: v, s.rhs(), rtol=1e-14, max_iter=3)
    assert it == 3 and rel > 1e-14


def test_adjoint_gradient_matches_finite_differences():
    gc = W.gradient_case(n=8, s=4, n_balls=3, seed=4)
    p = gc.problem
    s = OracleSolver(p)
    b = s.rhs()
    A = s.d.A.tocsc()
    u = spla.spsolve(A, b)
    ut = u * 0.9 + 0.01
    lam = spla.spsolve(A, u - ut)
    dth, df = adjoint.gradients(s.d, u, lam)

    def J(theta=None, f=None):
        q = p.with_options(kappa=np.exp(theta) if theta is not None else p.kappa,
                           f=f if f is not None else p.f)
        dq = assemble.discretise(q)
        uq = spla.spsolve(dq.A.tocsc(), assemble.load(dq, q.f))
        return 0.5 * np.sum((uq - ut) ** 2)

    theta = gc.theta
    eps = 1e-6
    for cell in s.d.active[:: max(1, s.d.active.size // 6)]:
        tp, tm = theta.copy(), theta.copy()
        tp[cell] += eps
        tm[cell] -= eps
        fd = (J(theta=tp) - J(theta=tm)) / (2 * eps)
        assert abs(fd - dth[cell]) <= 1e-5 * max(abs(fd), 1e-12) + 1e-14
    for node in [10, 300, 400]:
        fp, fm = p.f.copy(), p.f.copy()
        fp[node] += eps
        fm[node] -= eps
        fd = (J(f=fp) - J(f=fm)) / (2 * eps)
        assert abs(fd - df[node]) <= 1e-5 * max(abs(fd), 1e-12) + 1e-14
