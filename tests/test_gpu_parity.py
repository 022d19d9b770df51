"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bars: bit-exact for the integer data (cell classification, DOF numbering,
subdomain sets, objects, coarse numbering); relative 1e-13 for cut-cell
matrices, operator and load (same arithmetic up to summation order); 1e-10
for the FP64 preconditioner, coarse matrix and PCG solution at rtol 1e-8
(both sides run the same PCG from x0 = 0 with the same stopping rule, so the
iterates differ only by rounding; iteration counts may differ by one when the
residual lands at the threshold); 1e-6 for the FP32-local path.
"""
import sys

import numpy as np
import pytest

try:  # first import of torch on a fresh box is slow: do it at collection time
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

import workloads as W
from oracle import OracleSolver, topology

pytestmark = pytest.mark.gpu

def _kappa_layer0():
    """kappa 10 in the bottom cell layer of subdomain 0 of an 8^3 mesh with
    4^3-cell subdomains (variant 2 then splits one coarse edge)."""
    k = np.ones(512)
    for j in range(4):
        for i in range(4):
            k[i + 8 * j] = 10.0
    return k


CASES = {
    "single_ball_standard_cardinality": lambda: W.single_ball().with_options(weighting=0, coarse_variant=0),
    "single_ball_standard_stiffness": lambda: W.single_ball().with_options(coarse_variant=0),
    "single_ball_v1_stiffness": lambda: W.single_ball(),
    "balls16_s4": lambda: W.random_balls(16, 4, 6, 3),
    "balls24_s8_lognormal": lambda: W.random_balls(24, 8, 8, 4, lognormal_kappa=True),
    "balls32_s8_ce": lambda: W.random_balls(32, 8, 12, 9).with_options(objects=1),
    "uncut16_s4": lambda: W.uncut(16, 4),
    "one_subdomain": lambda: W.random_balls(8, 8, 3, 5),
    "full_elements": lambda: W.random_balls(16, 8, 5, 6).with_options(full_elements=1),
    "single_ball_v2_stiffness": lambda: W.single_ball().with_options(coarse_variant=2),
    "balls16_s4_v2": lambda: W.random_balls(16, 4, 6, 3).with_options(coarse_variant=2),
    "balls24_s8_lognormal_v2": lambda: W.random_balls(24, 8, 8, 4, lognormal_kappa=True).with_options(
        coarse_variant=2),
    "uncut8_kappa_layer_v2": lambda: W.uncut(8, 4).with_options(coarse_variant=2, kappa=_kappa_layer0()),
}

_oracles = {}
_gpus = {}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle(name):
    if name not in _oracles:
        _oracles[name] = OracleSolver(CASES[name]())
    return _oracles[name]


def gpu(name):
    from paper_1703_06323_amd import Solver
    if name not in _gpus:
        say(f"[gpu] setup+factor {name}")
        s = Solver(CASES[name]())
        s.factor()
        _gpus[name] = s
    return _gpus[name]


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def elementwise(a, b):
    """max_i |a_i - b_i| / max_i |b_i|: a few wrong entries in a long vector
    hide under the relative 2-norm, not under this."""
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)) if b.size else 0.0


@pytest.mark.parametrize("name", list(CASES))
def test_indexing_bit_exact(name):
    o = oracle(name)
    g = gpu(name).export_indexing()
    assert np.array_equal(g["cell_count"], o.d.count)
    assert np.array_equal(g["cell_status"], o.d.status)
    assert np.array_equal(g["dof_node"], o.d.dof_node)
    assert np.array_equal(g["card"], o.topo.card())
    assert np.array_equal(g["obj_ptr"], o.topo.obj_ptr)
    assert np.array_equal(g["obj_dofs"], o.topo.obj_dofs)
    assert np.array_equal(g["obj_type"], o.topo.obj_type)
    assert np.array_equal(g["coarse_of_obj"], o.topo.coarse_of_obj)
    # subdomain-local DOF lists (the sub-assembled spaces of Sect. 3.1)
    ptr, dofs = gpu(name).export_subdomains()
    assert ptr.size == o.topo.n_sub + 1
    for w in range(o.topo.n_sub):
        assert np.array_equal(dofs[ptr[w]:ptr[w + 1]], o.topo.sub_dofs[w]), w


@pytest.mark.parametrize("name", list(CASES))
def test_cut_cell_matrices(name):
    from paper_1703_06323_amd.cutbddc import unpack36
    o = oracle(name)
    K, M, cells = gpu(name).export_cut_matrices()
    if CASES[name]().full_elements:
        assert cells.size == 0
        return
    assert np.array_equal(cells, o.d.cut)
    pos = np.searchsorted(o.d.active, cells)
    Ko = o.d.Kunit[pos]
    Mo = o.d.Munit[pos]
    np.testing.assert_allclose(unpack36(K), Ko, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(unpack36(M), Mo, rtol=1e-13, atol=1e-17)


@pytest.mark.parametrize("name", list(CASES))
def test_operator_and_load(name):
    o = oracle(name)
    s = gpu(name)
    rng = np.random.default_rng(42)
    x = rng.standard_normal(o.n_dof)
    say(f"[gpu] apply_operator {name}")
    y = s.apply_operator(x).cpu().numpy()
    yo = o.d.A @ x
    assert rel(y, yo) < 1e-13
    assert elementwise(y, yo) < 1e-13
    p = CASES[name]()
    say(f"[gpu] load {name}")
    b = s.load(p.f).cpu().numpy()
    bo = o.rhs()
    assert rel(b, bo) < 1e-13
    assert elementwise(b, bo) < 1e-13


@pytest.mark.parametrize("name", list(CASES))
def test_coarse_matrix(name):
    o = oracle(name)
    if o.topo.n_coarse == 0:
        return
    Ac = gpu(name).export_coarse()
    assert rel(Ac, o.M.Ac) < 1e-10


def test_coarse_matrix_global_rows(monkeypatch):
    """The coarse assembly builds rows longer than its LDS limit in place in
    global memory: forcing that path must give the same matrix bit for bit
    (same sums in the same order) and the same solve."""
    from paper_1703_06323_amd import Solver
    name = "balls32_s8_ce"
    ref = gpu(name).export_coarse()
    monkeypatch.setenv("CUTBDDC_COARSE_ROW_LDS", "1")
    say(f"[gpu] setup+factor {name} with global coarse rows")
    s = Solver(CASES[name]())
    s.factor()
    assert np.array_equal(s.export_coarse(), ref)
    p = CASES[name]()
    u, it, relres = s.solve(p.f, rtol=1e-8)
    u0, it0, _ = gpu(name).solve(p.f, rtol=1e-8)
    assert it == it0 and np.array_equal(u.cpu().numpy(), u0.cpu().numpy())
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_preconditioner_apply(name):
    o = oracle(name)
    s = gpu(name)
    rng = np.random.default_rng(7)
    r = rng.standard_normal(o.n_dof)
    say(f"[gpu] apply_preconditioner {name}")
    z = s.apply_preconditioner(r).cpu().numpy()
    zo = o.M.apply(r)
    assert rel(z, zo) < 1e-10
    assert elementwise(z, zo) < 1e-10


@pytest.mark.parametrize("name", list(CASES))
def test_solve_fp64(name):
    o = oracle(name)
    s = gpu(name)
    p = CASES[name]()
    say(f"[gpu] solve {name}")
    u, it, relres = s.solve(p.f, rtol=1e-8)
    x, it_o, rel_o = o.solve(rtol=1e-8)
    assert relres < 1e-8
    assert abs(it - it_o) <= 1, (it, it_o)
    assert rel(u.cpu().numpy(), x) < 1e-10
    assert elementwise(u.cpu().numpy(), x) < 1e-10


def test_solve_fp32_local():
    p = W.random_balls(24, 8, 8, 4, lognormal_kappa=True).with_options(local_precision=1)
    from paper_1703_06323_amd import Solver
    say("[gpu] fp32-local balls24")
    s = Solver(p)
    s.factor()
    u, it, relres = s.solve(p.f, rtol=1e-8)
    o = oracle("balls24_s8_lognormal")
    x, it_o, _ = o.solve(rtol=1e-8)
    assert relres < 1e-8
    err = rel(u.cpu().numpy(), x)
    print(f"fp32-local balls24: iterations {it} (FP64 oracle {it_o}), relative error {err:.2e}")
    assert err < 1e-6
    assert elementwise(u.cpu().numpy(), x) < 1e-6
    assert abs(it - it_o) <= 1


def test_zero_rhs_and_iteration_cap():
    import torch
    s = gpu("single_ball_v1_stiffness")
    say("[gpu] zero rhs")
    u, it, relres = s.solve_rhs(torch.zeros(s.n_dof, dtype=torch.float64))
    assert it == 0 and float(u.abs().max()) == 0.0
    from paper_1703_06323_amd.cutbddc import CBError, CB_ERR_NO_CONVERGENCE
    say("[gpu] max_iter=1")
    with pytest.raises(CBError) as e:
        s.solve(rtol=1e-14, max_iter=1)
    assert e.value.code == CB_ERR_NO_CONVERGENCE


def test_invalid_arguments_rejected():
    from paper_1703_06323_amd import Solver
    from paper_1703_06323_amd.cutbddc import CBError, CB_ERR_ARG, CB_ERR_SINGULAR
    say("[gpu] invalid arguments")
    with pytest.raises(CBError) as e:
        Solver(W.uncut(10, 4))
    assert e.value.code == CB_ERR_ARG
    bad = W.uncut(8, 4)
    bad.kappa = -np.ones(512)
    with pytest.raises(CBError) as e:
        Solver(bad)
    assert e.value.code == CB_ERR_ARG
    rng = np.random.default_rng(0)
    dirs = rng.standard_normal((400, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    pocket = W.Problem(n=16, s=4, centres=0.5 + 0.3 * dirs, radii=np.full(400, 0.12))
    with pytest.raises(CBError) as e:
        Solver(pocket)
    assert e.value.code == CB_ERR_SINGULAR


def test_state_errors():
    """Calls out of order, and single-problem entry points on a batch
    context, are CB_ERR_STATE."""
    import torch
    from paper_1703_06323_amd import BatchSolver, Solver
    from paper_1703_06323_amd.cutbddc import CBError, CB_ERR_STATE
    say("[gpu] state errors")
    s = Solver(W.uncut(8, 4))
    for call in (lambda: s.solve(), lambda: s.apply_preconditioner(torch.zeros(s.n_dof, dtype=torch.float64)),
                 lambda: s.time_kernel("apply_interior"), lambda: s.export_coarse()):
        with pytest.raises(CBError) as e:
            call()
        assert e.value.code == CB_ERR_STATE
    s.factor()
    u, it, _ = s.solve()
    assert it >= 1
    b = BatchSolver([W.uncut(8, 4), W.single_ball()])
    from paper_1703_06323_amd import cutbddc
    with pytest.raises(CBError) as e:
        cutbddc._export_indexing(b.ctx, None, 8, b.problem_info(0))
    assert e.value.code == CB_ERR_STATE
    b.factor()
    with pytest.raises(CBError) as e:
        cutbddc._check(cutbddc._lib.cb_apply_operator(b.ctx, u.data_ptr(), u.data_ptr()))
    assert e.value.code == CB_ERR_STATE


def test_fp32_breakdown_refactored_in_fp64(monkeypatch):
    """A subdomain whose FP32 local Cholesky breaks down is factored again in
    FP64 (its operators then stored in FP32 like the others) and counted in
    n_fp64_fallbacks.  The breakdown is forced from the host on one
    subdomain; the solve must still meet the FP32-local bar."""
    from paper_1703_06323_amd import Solver
    p = CASES["balls24_s8_lognormal"]().with_options(local_precision=1)
    say("[gpu] fp32 factor without forced breakdown")
    s0 = Solver(p)
    s0.factor()
    assert s0.info()["n_fp64_fallbacks"] == 0
    u0, it0, _ = s0.solve(p.f, rtol=1e-8)
    monkeypatch.setenv("CUTBDDC_FORCE_FP32_BREAKDOWN", "13")
    say("[gpu] fp32 factor with subdomain 13 refactored in fp64")
    s = Solver(p)
    s.factor()
    assert s.info()["n_fp64_fallbacks"] == 1
    u, it, relres = s.solve(p.f, rtol=1e-8)
    x, it_o, _ = oracle("balls24_s8_lognormal").solve(rtol=1e-8)
    err = rel(u.cpu().numpy(), x)
    print(f"fallback solve: iterations {it} (oracle {it_o}), error {err:.2e}")
    assert relres < 1e-8 and err < 1e-6 and abs(it - it_o) <= 1
    # the refactored subdomain changes its operators only by FP32 rounding
    r = np.random.default_rng(3).standard_normal(s.n_dof)
    z, z0 = s.apply_preconditioner(r).cpu().numpy(), s0.apply_preconditioner(r).cpu().numpy()
    assert rel(z, z0) < 1e-5


BOX_CASES = ["single_ball_v1_stiffness", "balls16_s4", "balls24_s8_lognormal", "balls32_s8_ce", "uncut16_s4",
             "one_subdomain", "full_elements"]


@pytest.mark.parametrize("per_box", [1, 2048])
@pytest.mark.parametrize("name", BOX_CASES)
def test_operator_node_boxes(name, per_box, monkeypatch):
    """The node-box form of the operator (chosen by setup for large meshes),
    forced on the small cases: one plane per box, and boxes marching over up
    to 32 planes."""
    from paper_1703_06323_amd import Solver
    monkeypatch.setenv("CUTBDDC_OPERATOR", f"box:{per_box}")
    o = oracle(name)
    say(f"[gpu] node-box operator {name} {per_box}")
    s = Solver(CASES[name]())
    x = np.random.default_rng(43).standard_normal(o.n_dof)
    y = s.apply_operator(x).cpu().numpy()
    yo = o.d.A @ x
    assert elementwise(y, yo) < 1e-13
    s.close()


def test_node_box_solves_match_node_block_solves(monkeypatch):
    """PCG (whose p.q parts come from the operator kernel) with node boxes,
    one problem and a batch of three, against the node-block form."""
    from paper_1703_06323_amd import BatchSolver, Solver
    probs = [W.random_balls(16, 4, 6, 3), W.random_balls(24, 4, 8, 4, lognormal_kappa=True), W.single_ball()]
    res = {}
    for mode in ("block", "box:2048"):
        monkeypatch.setenv("CUTBDDC_OPERATOR", mode)
        say(f"[gpu] solves with operator {mode}")
        s = Solver(probs[0])
        s.factor()
        u, it, _ = s.solve(probs[0].f, rtol=1e-8)
        b = BatchSolver(probs)
        b.factor()
        us, its, _ = b.solve([p.f for p in probs], rtol=1e-8)
        res[mode] = (u.cpu().numpy(), it, [v.cpu().numpy() for v in us], list(its))
        s.close()
        b.close()
    ub, itb, usb, itsb = res["block"]
    ux, itx, usx, itsx = res["box:2048"]
    assert itx == itb and itsx == itsb
    assert elementwise(ux, ub) < 1e-10
    for a, c in zip(usx, usb):
        assert elementwise(a, c) < 1e-10


ND_CASES = ["single_ball_v1_stiffness", "balls16_s4", "balls24_s8_lognormal", "balls32_s8_ce", "uncut16_s4",
            "full_elements", "balls16_s4_v2", "balls24_s8_lognormal_v2", "uncut8_kappa_layer_v2"]


@pytest.mark.parametrize("name", ND_CASES)
def test_nested_dissection_coarse_solve(name, monkeypatch):
    """The coarse problem by nested dissection (octant blocks and the Schur
    complement of the separator; chosen by the size rule for large single
    meshes), forced on the small cases: the preconditioner and the PCG
    solution against the oracle's dense coarse solve."""
    from paper_1703_06323_amd import Solver
    monkeypatch.setenv("CUTBDDC_COARSE", "nd")
    o = oracle(name)
    say(f"[gpu] nested-dissection coarse solve {name}")
    s = Solver(CASES[name]())
    s.factor()
    inf = s.info()
    assert 0 < inf["coarse_separator"] <= inf["n_coarse"]
    assert inf["coarse_separator"] + inf["coarse_octant_max"] <= inf["n_coarse"]
    r = np.random.default_rng(7).standard_normal(o.n_dof)
    z = s.apply_preconditioner(r).cpu().numpy()
    zo = o.M.apply(r)
    assert elementwise(z, zo) < 1e-10
    p = CASES[name]()
    u, it, relres = s.solve(p.f, rtol=1e-8)
    x, it_o, _ = o.solve(rtol=1e-8)
    assert relres < 1e-8 and abs(it - it_o) <= 1, (it, it_o)
    assert elementwise(u.cpu().numpy(), x) < 1e-10
    s.close()


def test_nested_dissection_is_the_default_for_large_coarse_problems(monkeypatch):
    """48^3 cells in 4^3-cell subdomains (12^3 subdomains, about 5 000 coarse
    DOFs): the size rule picks nested dissection; its preconditioner and
    solution agree with the dense coarse Cholesky's."""
    from paper_1703_06323_amd import Solver
    p = W.random_balls(48, 4, 30, 11)
    r = None
    out = {}
    for mode in ("", "dense"):
        if mode:
            monkeypatch.setenv("CUTBDDC_COARSE", mode)
        else:
            monkeypatch.delenv("CUTBDDC_COARSE", raising=False)
        say(f"[gpu] 48^3 coarse {mode or 'default'}")
        s = Solver(p)
        s.factor()
        inf = s.info()
        if r is None:
            r = np.random.default_rng(3).standard_normal(s.n_dof)
        z = s.apply_preconditioner(r).cpu().numpy()
        u, it, relres = s.solve(p.f, rtol=1e-8)
        out[mode] = (inf, z, u.cpu().numpy(), it)
        s.close()
    inf, z, u, it = out[""]
    assert inf["coarse_separator"] > 0 and inf["n_coarse"] >= 1024
    assert out["dense"][0]["coarse_separator"] == 0
    say(f"  n_coarse {inf['n_coarse']}, separator {inf['coarse_separator']}, "
        f"largest octant {inf['coarse_octant_max']}, iterations {it} / {out['dense'][3]}")
    assert elementwise(z, out["dense"][1]) < 1e-10
    assert abs(it - out["dense"][3]) <= 1
    assert elementwise(u, out["dense"][2]) < 1e-9
