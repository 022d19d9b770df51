"""The library's host C++ indexing (DOFs, subdomain sets, objects, variant-1
splitting, coarse numbering) against the oracle, bit-exact, on the CPU: the
cell classification is taken from the oracle and fed to the library."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import assemble, topology

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1703_06323_amd", "libcutbddc.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")

CASES = {
    "single_ball_standard": lambda: W.single_ball().with_options(coarse_variant=0),
    "single_ball_v1": lambda: W.single_ball(),
    "balls16_s4_v1": lambda: W.random_balls(16, 4, 6, 3),
    "balls24_s8_ce": lambda: W.random_balls(24, 8, 10, 4).with_options(objects=1),
    "balls32_s8_v1": lambda: W.random_balls(32, 8, 14, 5),
    "balls20_s4_dense": lambda: W.random_balls(20, 4, 30, 8),
    "uncut12_s4": lambda: W.uncut(12, 4),
    "uncut6_s2": lambda: W.uncut(6, 2),
    "one_subdomain": lambda: W.random_balls(8, 8, 3, 5),
}


@pytest.mark.parametrize("name", list(CASES))
def test_host_indexing_matches_oracle(name):
    from paper_1703_06323_amd.cutbddc import host_indexing
    p = CASES[name]()
    d = assemble.discretise(p)
    t = topology.build(p, d)
    g = host_indexing(p, d.count)
    assert np.array_equal(g["dof_node"], d.dof_node)
    assert np.array_equal(g["card"], t.card())
    assert np.array_equal(g["obj_ptr"], t.obj_ptr)
    assert np.array_equal(g["obj_dofs"], t.obj_dofs)
    assert np.array_equal(g["obj_type"], t.obj_type)
    assert np.array_equal(g["coarse_of_obj"], t.coarse_of_obj)
    assert g["n_coarse"] == t.n_coarse


def test_host_indexing_rejects_floating_pocket():
    from paper_1703_06323_amd.cutbddc import host_indexing, CBError, CB_ERR_SINGULAR
    rng = np.random.default_rng(0)
    dirs = rng.standard_normal((400, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    p = W.Problem(n=16, s=4, centres=0.5 + 0.3 * dirs, radii=np.full(400, 0.12))
    d = assemble.discretise(p, check_floating=False)
    with pytest.raises(CBError) as e:
        host_indexing(p, d.count)
    assert e.value.code == CB_ERR_SINGULAR


_REPEAT = r"""
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import numpy as np
import workloads as W
from oracle import assemble
from paper_1703_06323_amd.cutbddc import host_indexing
cases = []
for k, (n, s, nb) in enumerate([(12, 4, 28), (8, 4, 25), (8, 2, 38)]):
    p = W.random_balls(n, s, nb, 102 + k)
    cases.append((p, assemble.discretise(p, check_floating=False).count, None))
cases = [(p, c, host_indexing(p, c)["dof_node"]) for p, c, _ in cases]
for it in range({reps}):
    for p, c, ref in cases:
        assert np.array_equal(host_indexing(p, c)["dof_node"], ref)
print("ok", flush=True)
"""


def test_host_indexing_many_calls_finish():
    """Back-to-back calls reuse the indexing's worker pool thousands of times;
    a task claimed twice around the start of a run used to leave the caller
    waiting for ever.  Run in a child process under a time limit."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = _REPEAT.format(root=root, tests=os.path.join(root, "tests"), reps=2500)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-2000:]


def _hand_counts(n, inactive):
    c = np.full(n ** 3, 512, dtype=np.int32)
    for (i, j, k) in inactive:
        c[i + n * (j + n * k)] = 0
    return c


@pytest.mark.parametrize("n,s,inactive", [
    (8, 4, [(3, 1, k) for k in range(4)]),      # links broken on a face and on a coarse edge
    (6, 3, [(2, 1, 1)]),                        # a face demoted to an edge
])
def test_host_indexing_hand_cut_partitions(n, s, inactive):
    """The hand-made partitions whose objects are written out in
    test_oracle_assemble_topology: the library's host indexing agrees with
    the oracle bit for bit."""
    from paper_1703_06323_amd.cutbddc import host_indexing
    p = W.uncut(n, s)
    count = _hand_counts(n, inactive)
    d = assemble.discretise(p, count=count)
    t = topology.build(p, d)
    g = host_indexing(p, count)
    assert np.array_equal(g["dof_node"], d.dof_node)
    assert np.array_equal(g["card"], t.card())
    assert np.array_equal(g["obj_ptr"], t.obj_ptr)
    assert np.array_equal(g["obj_dofs"], t.obj_dofs)
    assert np.array_equal(g["obj_type"], t.obj_type)
    assert np.array_equal(g["coarse_of_obj"], t.coarse_of_obj)
