"""Adjoint gradient through torch.autograd on the GPU, against the oracle's
adjoint gradient and central finite differences of the GPU forward solve
(h = 1e-6, solves at rtol 1e-12 so that the difference quotient is not
dominated by solver error)."""
import os

import numpy as np
import pytest

try:
    import torch
except ImportError:  # pragma: no cover
    torch = None

import scipy.sparse.linalg as spla

import workloads as W
from oracle import OracleSolver, adjoint

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def loss_and_grads(problem, theta, f, ut, rtol=1e-12):
    from paper_1703_06323_amd import autograd as AG
    th = torch.tensor(theta, dtype=torch.float64, device="cuda", requires_grad=True)
    fv = torch.tensor(f, dtype=torch.float64, device="cuda", requires_grad=True)
    u = AG.solve(th, fv, problem, rtol=rtol)
    J = 0.5 * torch.sum((u - torch.tensor(ut, device="cuda")) ** 2)
    J.backward()
    return float(J), th.grad.cpu().numpy(), fv.grad.cpu().numpy()


def forward_J(problem, theta, f, ut, rtol=1e-13):
    from paper_1703_06323_amd import Solver
    s = Solver(problem.with_options(kappa=np.exp(theta)))
    s.factor()
    u, it, rel = s.solve(torch.tensor(f, device="cuda"), rtol=rtol)
    return 0.5 * float(torch.sum((u - torch.tensor(ut, device="cuda")) ** 2))


def test_gradient_matches_oracle_small():
    gc = W.gradient_case(n=16, s=8, n_balls=6, seed=4)
    p = gc.problem
    o = OracleSolver(p)
    A = o.d.A.tocsc()
    b = o.rhs()
    u = spla.spsolve(A, b)
    ut = u * 0.8 + gc.target_noise[o.d.dof_node]
    lam = spla.spsolve(A, u - ut)
    dth_o, df_o = adjoint.gradients(o.d, u, lam)
    print("[gpu] autograd small", flush=True)
    J, dth, df = loss_and_grads(p, gc.theta, p.f, ut)
    assert abs(J - 0.5 * np.sum((u - ut) ** 2)) <= 1e-9 * J
    assert np.linalg.norm(dth - dth_o) / np.linalg.norm(dth_o) < 1e-8
    assert np.linalg.norm(df - df_o) / np.linalg.norm(df_o) < 1e-8
    # inactive cells carry no gradient
    inactive = np.setdiff1d(np.arange(p.n ** 3), o.d.active)
    assert np.all(dth[inactive] == 0.0)


def test_gradient_finite_differences_small():
    gc = W.gradient_case(n=16, s=8, n_balls=6, seed=4)
    p = gc.problem
    o = OracleSolver(p)
    ut = gc.target_noise[o.d.dof_node]
    J, dth, df = loss_and_grads(p, gc.theta, p.f, ut)
    eps = 1e-6
    rng = np.random.default_rng(11)
    for cell in rng.choice(o.d.active, size=6, replace=False):
        tp, tm = gc.theta.copy(), gc.theta.copy()
        tp[cell] += eps
        tm[cell] -= eps
        fd = (forward_J(p, tp, p.f, ut) - forward_J(p, tm, p.f, ut)) / (2 * eps)
        assert abs(fd - dth[cell]) <= 1e-4 * abs(fd) + 1e-12
    for node in rng.choice((p.n + 1) ** 3, size=3, replace=False):
        fp, fm = p.f.copy(), p.f.copy()
        fp[node] += eps
        fm[node] -= eps
        fd = (forward_J(p, gc.theta, fp, ut) - forward_J(p, gc.theta, fm, ut)) / (2 * eps)
        assert abs(fd - df[node]) <= 1e-4 * abs(fd) + 1e-12


def test_gradient_full_size_against_oracle_and_fd():
    path = os.path.join(GOLDEN, "gradient_64.npz")
    if not os.path.exists(path):
        pytest.skip("gradient golden values not generated")
    g = np.load(path)
    gc = W.gradient_case()
    p = gc.problem
    print("[gpu] autograd 64^3", flush=True)
    J, dth, df = loss_and_grads(p, gc.theta, p.f, g["ut"])
    assert abs(J - g["J"][0]) <= 1e-8 * g["J"][0]
    cells = g["cells"]
    np.testing.assert_allclose(dth[cells], g["dtheta_cells"], rtol=1e-7, atol=1e-7 * np.abs(g["dtheta_cells"]).max())
    assert abs(np.linalg.norm(dth) - g["dtheta_norm"][0]) <= 1e-7 * g["dtheta_norm"][0]
    np.testing.assert_allclose(df[g["nodes"]], g["df_nodes"], rtol=1e-7, atol=1e-7 * np.abs(g["df_nodes"]).max())
    eps = 1e-6
    worst = 0.0
    floor = 1e-6 * np.abs(dth[cells]).max()
    for cell in cells:
        tp, tm = gc.theta.copy(), gc.theta.copy()
        tp[cell] += eps
        tm[cell] -= eps
        fd = (forward_J(p, tp, p.f, g["ut"]) - forward_J(p, tm, p.f, g["ut"])) / (2 * eps)
        err = abs(fd - dth[cell]) / max(abs(fd), floor)
        worst = max(worst, err)
    print(f"worst relative FD error over 32 cells: {worst:.2e}")
    assert worst <= 1e-4
