"""Device indexing (DOFs, subdomain sets, objects, variant-1 splitting,
coarse numbering) against the library's host indexing, bit-exact: the host
indexing is fed the device's own cell classification, so any difference is
in the indexing.  Problems with an enclosed active pocket must be rejected
by both.  Batched setups must give every problem the host's counts."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("dof_node", "card", "obj_ptr", "obj_dofs", "obj_type", "coarse_of_obj")


def _cases():
    out = {}
    shapes = [(8, 2), (8, 4), (12, 4), (16, 4), (16, 8), (24, 8), (32, 8), (12, 3), (10, 5)]
    rng = np.random.default_rng(7)
    for k in range(27):
        n, s = shapes[k % len(shapes)]
        nb = int(rng.integers(0, 41))
        p = W.random_balls(n, s, nb, 100 + k).with_options(coarse_variant=int(k % 3 != 0),
                                                           objects=int(k % 4 == 3))
        out[f"r{k}_n{n}_s{s}_b{nb}_v{p.coarse_variant}_o{p.objects}"] = p
    out["single_ball_v1"] = W.single_ball()
    out["single_ball_standard"] = W.single_ball().with_options(coarse_variant=0)
    out["single_ball_ce"] = W.single_ball().with_options(objects=1)
    out["uncut12_s4"] = W.uncut(12, 4)
    out["uncut6_s2"] = W.uncut(6, 2)
    out["one_subdomain"] = W.random_balls(8, 8, 3, 5)
    out["full_elements"] = W.random_balls(16, 4, 8, 9).with_options(full_elements=1)
    out["cut_cube_64"] = W.cut_cube_64()
    return out


CASES = _cases()

@pytest.mark.parametrize("name", list(CASES))
def test_device_indexing_matches_host(name):
    from paper_1703_06323_amd import Solver
    from paper_1703_06323_amd.cutbddc import CBError, CB_ERR_SINGULAR, host_indexing
    p = CASES[name]
    print(f"[gpu] indexing {name}", flush=True)
    try:
        s = Solver(p)
    except CBError as e:
        assert e.code == CB_ERR_SINGULAR, name
        from oracle import assemble
        d = assemble.discretise(p, check_floating=False)
        with pytest.raises(CBError) as e2:
            host_indexing(p, d.count)
        assert e2.value.code == CB_ERR_SINGULAR
        return
    g = s.export_indexing()
    h = host_indexing(p, g["cell_count"])
    for k in KEYS:
        assert np.array_equal(g[k], h[k]), (name, k)
    inf = s.info()
    assert inf["n_coarse"] == h["n_coarse"]
    assert inf["n_objects"] == h["obj_type"].size
    assert inf["n_dof"] == h["dof_node"].size


def test_batch_indexing_counts_match_host():
    from oracle import assemble
    from paper_1703_06323_amd import BatchSolver
    from paper_1703_06323_amd.cutbddc import host_indexing
    rng = np.random.default_rng(11)
    probs = []
    for k in range(12):
        n = int(rng.choice([8, 16, 24]))
        probs.append(W.random_balls(n, 8, int(rng.integers(3, 15)), 200 + k))
    probs.append(W.uncut(16, 8))
    print(f"[gpu] batch indexing of {len(probs)} problems", flush=True)
    b = BatchSolver(probs)
    for k, p in enumerate(probs):
        h = host_indexing(p, assemble.discretise(p).count)
        inf = b.problem_info(k)
        assert inf["n_dof"] == h["dof_node"].size, k
        assert inf["n_coarse"] == h["n_coarse"], k
        assert inf["n_objects"] == h["obj_type"].size, k
        assert inf["n_iface"] == h["obj_dofs"].size, k
