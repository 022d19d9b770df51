"""The eps sweep of the single-ball problem (51 ball positions across one
cell, Sect. 5.2) on the GPU, one batch of 51 problems per (weighting,
coarse variant: standard, variant 1, variant 2): FP64 iteration counts
equal to the oracle's and solutions within 1e-10; the stiffness-weighted
counts stay within one iteration."""
import numpy as np
import pytest

try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

import workloads as W
from oracle import OracleSolver

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("weighting", [W.W_CARDINALITY, W.W_STIFFNESS])
@pytest.mark.parametrize("variant", [W.CV_STANDARD, W.CV_V1, W.CV_V2])
def test_eps_sweep_matches_oracle(weighting, variant):
    from paper_1703_06323_amd import BatchSolver
    probs = [W.single_ball(shift_x=float(e)).with_options(weighting=weighting, coarse_variant=variant)
             for e in W.eps_sweep_shifts()]
    print(f"[gpu] eps sweep weighting={weighting} variant={variant}", flush=True)
    b = BatchSolver(probs)
    b.factor()
    us, its, rels = b.solve(None, rtol=1e-8)
    for k, p in enumerate(probs):
        o = OracleSolver(p)
        x, it, _ = o.solve(rtol=1e-8)
        assert its[k] == it, k
        u = us[k].cpu().numpy()
        assert np.linalg.norm(u - x) <= 1e-10 * np.linalg.norm(x), k
        assert b.problem_info(k)["n_coarse"] == o.topo.n_coarse
    print("  iterations:", its.tolist())
    if weighting == W.W_STIFFNESS:
        assert its.max() - its.min() <= 1
