"""Full-size GPU parity on the benchmark workloads against stored oracle
values (tests/golden/make_golden.py, oracle only): the integer indexing
by SHA-256 of every array, the PCG iteration count, and the solution on a
seeded sample of 16384 DOFs (relative error of the sample vector)."""
import hashlib
import json
import os

import numpy as np
import pytest

try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    torch = None

import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def load(tag):
    path = os.path.join(GOLDEN, tag + ".json")
    if not os.path.exists(path):
        pytest.skip(f"{tag} golden values not generated")
    meta = json.load(open(path))
    smp = np.load(os.path.join(GOLDEN, tag + "_sample.npz"))
    return meta, smp


def sample_err(u, smp):
    x = smp["u"]
    return np.linalg.norm(u[smp["idx"]] - x) / np.linalg.norm(x)


_solvers = {}


def solver(tag, precision):
    from paper_1703_06323_amd import Solver
    key = (tag, precision)
    if key not in _solvers:
        p = W.cut_cube_64() if tag == "cut_cube_64" else W.cut_cube_96_lognormal()
        p = p.with_options(local_precision=precision)
        print(f"[gpu] setup+factor {tag} precision={precision}", flush=True)
        s = Solver(p)
        s.factor()
        _solvers[key] = (s, p)
    return _solvers[key]


def check_hashes(s, meta):
    g = s.export_indexing()
    inf = s.info()
    assert inf["n_dof"] == meta["n_dof"] and inf["n_coarse"] == meta["n_coarse"]
    assert inf["n_cut"] == meta["n_cut"]
    h = meta["sha256"]
    assert sha(g["cell_count"].astype(np.int32)) == h["cell_count"]
    assert sha(g["dof_node"].astype(np.int64)) == h["dof_node"]
    assert sha(g["card"].astype(np.int32)) == h["card"]
    assert sha(g["obj_ptr"].astype(np.int64)) == h["obj_ptr"]
    assert sha(g["obj_dofs"].astype(np.int64)) == h["obj_dofs"]
    assert sha(g["obj_type"].astype(np.int8)) == h["obj_type"]
    assert sha(g["coarse_of_obj"].astype(np.int32)) == h["coarse_of_obj"]


def test_cut_cube_64_indexing_matches_oracle():
    meta, _ = load("cut_cube_64")
    s, _ = solver("cut_cube_64", 0)
    check_hashes(s, meta)


def test_cut_cube_96_indexing_matches_oracle():
    meta, _ = load("cut_cube_96")
    s, _ = solver("cut_cube_96", 1)
    check_hashes(s, meta)


def test_cut_cube_64_fp64_solution():
    meta, smp = load("cut_cube_64")
    s, p = solver("cut_cube_64", 0)
    print("[gpu] solve cut_cube_64 fp64", flush=True)
    u, it, rel = s.solve(p.f, rtol=1e-8)
    assert rel < 1e-8
    assert abs(it - meta["iterations_rtol_1e-8"]) <= 1
    assert sample_err(u.cpu().numpy(), smp) < 1e-10
    assert abs(float(u.norm()) - smp["norm"][0]) / smp["norm"][0] < 1e-10


def test_cut_cube_64_fp32_local_solution():
    meta, smp = load("cut_cube_64")
    s, p = solver("cut_cube_64", 1)
    print("[gpu] solve cut_cube_64 fp32-local", flush=True)
    u, it, rel = s.solve(p.f, rtol=1e-8)
    assert rel < 1e-8
    err = sample_err(u.cpu().numpy(), smp)
    print(f"fp32-local cut_cube_64: iterations {it} vs FP64 oracle {meta['iterations_rtol_1e-8']}, "
          f"sample error {err:.2e}")
    assert err < 1e-6
    assert abs(it - meta["iterations_rtol_1e-8"]) <= 1


def test_cut_cube_96_fp32_local_solution():
    meta, smp = load("cut_cube_96")
    s, p = solver("cut_cube_96", 1)
    print("[gpu] solve cut_cube_96 fp32-local", flush=True)
    u, it, rel = s.solve(p.f, rtol=1e-8)
    assert rel < 1e-8
    err = sample_err(u.cpu().numpy(), smp)
    print(f"fp32-local cut_cube_96: iterations {it} vs FP64 oracle {meta['iterations_rtol_1e-8']}, "
          f"sample error {err:.2e}")
    assert err < 1e-6
    assert abs(it - meta["iterations_rtol_1e-8"]) <= 1
