"""Robustness of the preconditioner to the cut location (Sect. 5.2): the
ball of the single-ball problem is moved through 51 positions across one
cell (eps in [-h, h]).  With the stiffness weighting (eq. alge-weighting)
the PCG iteration count stays flat, while with the cardinality weighting
(eq. weighting) it grows as small cuts appear near the subdomain interface.
Variant 1 (Sect. 4.4) turns the DOFs of cut coarse edges into corners, so
its coarse space is never smaller than the standard one; variant 2 (Sect.
4.5) splits coarse edges where the weighting coefficient changes."""
import numpy as np
import pytest

import workloads as W
from oracle import OracleSolver


def sweep(weighting, variant):
    its, ncs = [], []
    for e in W.eps_sweep_shifts():
        p = W.single_ball(shift_x=float(e)).with_options(weighting=weighting, coarse_variant=variant)
        o = OracleSolver(p)
        its.append(o.solve(rtol=1e-8)[1])
        ncs.append(o.topo.n_coarse)
    return np.array(its), np.array(ncs)


@pytest.fixture(scope="module")
def sweeps():
    return {(w, v): sweep(w, v) for w in (W.W_CARDINALITY, W.W_STIFFNESS)
            for v in (W.CV_STANDARD, W.CV_V1, W.CV_V2)}


def test_stiffness_weighting_is_robust_to_the_cut(sweeps):
    for v in (W.CV_STANDARD, W.CV_V1, W.CV_V2):
        it_s, _ = sweeps[(W.W_STIFFNESS, v)]
        it_c, _ = sweeps[(W.W_CARDINALITY, v)]
        assert it_s.max() - it_s.min() <= 1
        # the cardinality weighting degrades somewhere in the sweep
        assert it_c.max() >= it_s.max() + 2
        assert np.all(it_s <= it_c)


def test_variant_one_only_adds_coarse_dofs(sweeps):
    for w in (W.W_CARDINALITY, W.W_STIFFNESS):
        _, nc_std = sweeps[(w, W.CV_STANDARD)]
        _, nc_v1 = sweeps[(w, W.CV_V1)]
        assert np.all(nc_v1 >= nc_std)
        assert nc_v1.max() > nc_std.max()


def test_variant_two(sweeps):
    """Variant 2 (Sect. 4.5) changes nothing under the topological weighting
    (constant coefficients); under the stiffness weighting its iteration
    count varies by at most one over the 51 cut positions (the paper's
    robustness claim for this variant) and its coarse space is never
    smaller than the standard one."""
    it_c2, nc_c2 = sweeps[(W.W_CARDINALITY, W.CV_V2)]
    it_c0, nc_c0 = sweeps[(W.W_CARDINALITY, W.CV_STANDARD)]
    assert np.array_equal(it_c2, it_c0) and np.array_equal(nc_c2, nc_c0)
    it_s2, nc_s2 = sweeps[(W.W_STIFFNESS, W.CV_V2)]
    _, nc_s0 = sweeps[(W.W_STIFFNESS, W.CV_STANDARD)]
    assert it_s2.max() - it_s2.min() <= 1
    assert np.all(nc_s2 >= nc_s0)
