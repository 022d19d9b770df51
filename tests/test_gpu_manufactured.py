"""Manufactured-solution accuracy on the GPU (Sect. 5.1): the load and the
L2 / H1 errors of u = sin(k |x - x0|) against the oracle, and the
convergence of the discrete solution under refinement.

The load sums sin / cos values of the device's libm and the oracle's in
different orders, and the Nitsche data terms carry beta_e, which the two
sides compute by different eigen solvers (agreeing to about 1e-11 of the
cell matrices): every DOF of the load agrees to 1e-10 of the largest
entry.  The errors of one given vector agree to 1e-10 relative; the GPU
solve (rtol 1e-10) gives errors within 1e-6 of the oracle's direct
solution."""
import ctypes

import numpy as np
import pytest
import scipy.sparse.linalg as spla

try:
    import torch
except ImportError:  # pragma: no cover
    torch = None

import workloads as W
from oracle import assemble, manufactured as mm

pytestmark = pytest.mark.gpu

K = 5.0 * np.pi
X0 = (0.0, 0.0, 0.0)

CASES = {
    "uncut16": lambda: W.uncut(16, 4),
    "single_ball_neumann": lambda: W.single_ball(16, 4),
    "single_ball_nitsche": lambda: W.single_ball(16, 4).with_options(cut_boundary=1),
    "single_ball_full_elements": lambda: W.single_ball(16, 4).with_options(full_elements=1),
    "balls16_s4_neumann": lambda: W.random_balls(16, 4, 6, 3, random_f=False),
    "balls24_s8_nitsche_v2": lambda: W.random_balls(24, 8, 8, 4, random_f=False).with_options(
        cut_boundary=1, coarse_variant=2),
}
_cache = {}


def case(name):
    if name not in _cache:
        from paper_1703_06323_amd import Solver
        p = CASES[name]()
        d = assemble.discretise(p)
        b = mm.load(p, d)
        u = spla.spsolve(d.A.tocsc(), b)
        print(f"[gpu] setup+factor {name}", flush=True)
        s = Solver(p)
        s.factor()
        _cache[name] = (p, d, b, u, s)
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_load_matches_the_oracle(name):
    p, d, b, u, s = case(name)
    bg = s.manufactured_load(X0, K).cpu().numpy()
    assert bg.shape == b.shape
    err = np.abs(bg - b).max() / np.abs(b).max()
    print(f"{name}: load error {err:.2e} over {b.size} DOFs")
    assert err <= 1e-10


@pytest.mark.parametrize("name", list(CASES))
def test_errors_match_the_oracle(name):
    p, d, b, u, s = case(name)
    want = mm.errors(p, d, u)
    got = s.manufactured_errors(torch.as_tensor(u, device="cuda"), X0, K)
    print(f"{name}: L2 {got[0]:.6e} (oracle {want[0]:.6e}), H1 {got[1]:.6e} (oracle {want[1]:.6e})")
    assert abs(got[0] - want[0]) <= 1e-10 * want[0]
    assert abs(got[1] - want[1]) <= 1e-10 * want[1]


@pytest.mark.parametrize("name", list(CASES))
def test_gpu_solution_has_the_oracle_errors(name):
    p, d, b, u, s = case(name)
    bg = s.manufactured_load(X0, K)
    ug, it, rel = s.solve_rhs(bg, rtol=1e-10)
    got = s.manufactured_errors(ug, X0, K)
    want = mm.errors(p, d, u)
    print(f"{name}: {it} iterations, L2 {got[0]:.6e} (oracle {want[0]:.6e}), H1 {got[1]:.6e}")
    assert abs(got[0] - want[0]) <= 1e-6 * want[0]
    assert abs(got[1] - want[1]) <= 1e-6 * want[1]


def test_rejects_batches_kappa_and_bad_parameters():
    from paper_1703_06323_amd import BatchSolver, Solver, cutbddc
    lib = cutbddc.load_library()
    x0 = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    bs = BatchSolver([W.uncut(8, 4), W.uncut(8, 4)])
    out = torch.empty(bs.n_dofs()[0], dtype=torch.float64, device="cuda")
    assert lib.cb_manufactured_load(bs.ctx, x0, K, out.data_ptr()) == cutbddc.CB_ERR_STATE
    bs.close()
    kap = W.uncut(8, 4).with_options(kappa=np.full(512, 2.0))
    s = Solver(kap)
    out = torch.empty(s.n_dof, dtype=torch.float64, device="cuda")
    assert lib.cb_manufactured_load(s.ctx, x0, K, out.data_ptr()) == cutbddc.CB_ERR_ARG
    s.close()
    s = Solver(W.uncut(8, 4))
    bad = (ctypes.c_double * 3)(0.0, float("nan"), 0.0)
    assert lib.cb_manufactured_load(s.ctx, bad, K, out.data_ptr()) == cutbddc.CB_ERR_ARG
    assert lib.cb_manufactured_load(s.ctx, x0, float("inf"), out.data_ptr()) == cutbddc.CB_ERR_ARG
    s.close()


@pytest.mark.parametrize("boundary", [W.CUT_NEUMANN, W.CUT_NITSCHE])
def test_convergence_under_refinement(boundary):
    """The paper's solution sin(5 pi |x|) on the single-ball domain with
    8^3-cell subdomains at 32^3, 64^3 and 128^3 cells: the L2 error falls
    like h^2 and the H1 error like h on both pairs.  (Neumann data must
    reach the sphere points in cells that the volume rule does not class as
    cut: dropping them held the L2 rate near 1.7 between 64^3 and 128^3.)"""
    from paper_1703_06323_amd import Solver
    errs = []
    for n in (32, 64, 128):
        p = W.single_ball(n, 8).with_options(cut_boundary=boundary)
        print(f"[gpu] refinement n={n} boundary={boundary}", flush=True)
        s = Solver(p)
        s.factor()
        b = s.manufactured_load(X0, K)
        u, it, rel = s.solve_rhs(b, rtol=1e-10)
        errs.append(s.manufactured_errors(u, X0, K))
        print(f"  n={n}: {it} iterations, L2 {errs[-1][0]:.4e}, H1 {errs[-1][1]:.4e}", flush=True)
        s.close()
    e = np.array(errs)
    rates = np.log2(e[:-1] / e[1:])
    print(f"  rates L2 {rates[:, 0].round(3).tolist()}, H1 {rates[:, 1].round(3).tolist()}")
    assert (rates[:, 0] >= 1.9).all() and (rates[:, 1] >= 0.95).all(), (rates, e)
