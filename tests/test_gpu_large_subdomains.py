"""Subdomains of 12^3 and 16^3 cells (H/h = 12 and 16, Sect. 5.2): their
padded local operators are too large for the single-workgroup packed
applies and for the LDS row buffers of the assembly, so the library takes
the block-row applies and the large-subdomain assembly.  The preconditioner
and the PCG solution against the oracle, at the tolerances of the parity
tests (1e-10 in FP64, 1e-6 for the FP32-local path)."""
import sys

import numpy as np
import pytest

try:  # first import of torch on a fresh box is slow: do it at collection time
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

import workloads as W
from oracle import OracleSolver

pytestmark = pytest.mark.gpu

CASES = {
    "balls24_s12": lambda: W.random_balls(24, 12, 6, 21),
    "balls24_s12_fp32": lambda: W.random_balls(24, 12, 6, 21).with_options(local_precision=1),
    "single_ball32_s16": lambda: W.single_ball(32, 16),
    "balls32_s16_nitsche_v2": lambda: W.random_balls(32, 16, 5, 22).with_options(cut_boundary=1,
                                                                                coarse_variant=2),
}
_oracles = {}
ORACLE_OF = {"balls24_s12_fp32": "balls24_s12"}   # the oracle is FP64 throughout


def oracle(name):
    key = ORACLE_OF.get(name, name)
    if key not in _oracles:
        _oracles[key] = OracleSolver(CASES[key]())
    return _oracles[key]


def elementwise(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("name", list(CASES))
def test_large_subdomains_match_the_oracle(name):
    from paper_1703_06323_amd import Solver
    p = CASES[name]()
    tol = 1e-6 if p.local_precision else 1e-10
    o = oracle(name)
    print(f"[gpu] large subdomains {name}", flush=True)
    sys.stdout.flush()
    s = Solver(p)
    s.factor()
    r = np.random.default_rng(5).standard_normal(o.n_dof)
    z = s.apply_preconditioner(r).cpu().numpy()
    assert elementwise(z, o.M.apply(r)) < tol
    u, it, relres = s.solve(p.f, rtol=1e-8)
    x, it_o, _ = o.solve(rtol=1e-8)
    print(f"  n_dof {o.n_dof}: {it} iterations (oracle {it_o})", flush=True)
    assert relres < 1e-8 and abs(it - it_o) <= 1, (it, it_o)
    assert elementwise(u.cpu().numpy(), x) < tol
    s.close()
