"""Writes the stored expected values for the full-size parity tests.

Calls only the oracle (and the seeded input generators).  Run from the repo
root:  python tests/golden/make_golden.py
Outputs (next to this script):
  cut_cube_64.json        sizes, iteration count, SHA-256 of the integer
                          indexing arrays (cell counts, DOF nodes, |S|,
                          objects, object types, coarse ids)
  cut_cube_64_sample.npz  seeded sample (16384 DOFs) of the FP64 PCG solution
                          at rtol 1e-8, plus its full 2-norm
With the argument `96`, the same files for the 96^3 forty-ball workload with
log-normal conductivity (cut_cube_96.json, cut_cube_96_sample.npz); with
`grad`, gradient_64.npz (adjoint gradient of the differentiation workload);
with `batch`, batch_256.json + batch_256_sample.npz (per problem of the
256-problem batch: sizes, SHA-256 of the DOF nodes, iteration count and a
16-DOF sample plus the 2-norm of the FP64 PCG solution at rtol 1e-8); with
`batch_full`, batch_256_full.npz (the whole FP64 PCG solution of the first
problem of each mesh size of that batch).
"""
import hashlib
import json
import os
import sys
import time

os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import OracleSolver  # noqa: E402


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main(which="64"):
    p = W.cut_cube_64() if which == "64" else W.cut_cube_96_lognormal().with_options(local_precision=0)
    tag = "cut_cube_" + which
    t0 = time.time()
    s = OracleSolver(p)
    x, it, rel = s.solve(rtol=1e-8)
    t = s.topo
    meta = {
        "workload": p.name, "n": p.n, "s": p.s, "n_balls": int(p.n_balls),
        "n_dof": int(s.n_dof), "n_active": int(s.d.active.size), "n_cut": int(s.d.cut.size),
        "n_coarse": int(t.n_coarse), "n_objects": int(t.obj_type.size),
        "object_types": np.bincount(t.obj_type, minlength=3).tolist(),
        "iterations_rtol_1e-8": int(it), "relres": float(rel),
        "sha256": {
            "cell_count": sha(s.d.count.astype(np.int32)),
            "dof_node": sha(s.d.dof_node.astype(np.int64)),
            "card": sha(t.card().astype(np.int32)),
            "obj_ptr": sha(t.obj_ptr.astype(np.int64)),
            "obj_dofs": sha(t.obj_dofs.astype(np.int64)),
            "obj_type": sha(t.obj_type.astype(np.int8)),
            "coarse_of_obj": sha(t.coarse_of_obj.astype(np.int32)),
        },
        "oracle_seconds": time.time() - t0,
        "oracle_phase_seconds": s.times,
    }
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(s.n_dof, size=16384, replace=False))
    np.savez_compressed(os.path.join(HERE, tag + "_sample.npz"), idx=idx, u=x[idx],
                        norm=np.array([np.linalg.norm(x)]))
    with open(os.path.join(HERE, tag + ".json"), "w") as fh:
        json.dump(meta, fh, indent=1)
    print(json.dumps(meta, indent=1))


def gradient():
    """Adjoint gradient of J = 0.5 |u - u_t|^2 on the 64^3 twenty-ball
    workload with kappa = exp(theta): u_t = solution at theta = 0 plus the
    seeded noise; 32 cells drawn from the active cells (generator stream
    continued).  Solves at rtol 1e-12."""
    from oracle import adjoint
    gc = W.gradient_case()
    p = gc.problem
    t0 = time.time()
    s0 = OracleSolver(p.with_options(kappa=None))
    u0, it0, _ = s0.solve(rtol=1e-12)
    ut = u0 + gc.target_noise[s0.d.dof_node]
    s = OracleSolver(p)
    u, it, _ = s.solve(rtol=1e-12)
    lam, itl, _ = s.solve_rhs(u - ut, rtol=1e-12)
    dth, df = adjoint.gradients(s.d, u, lam)
    cells = np.sort(gc.rng.choice(s.d.active, size=32, replace=False))
    rng = np.random.default_rng(777)
    nodes = np.sort(rng.choice((p.n + 1) ** 3, size=4096, replace=False))
    np.savez_compressed(os.path.join(HERE, "gradient_64.npz"), ut=ut, cells=cells, dtheta_cells=dth[cells],
                        nodes=nodes, df_nodes=df[nodes], dtheta_norm=np.array([np.linalg.norm(dth)]),
                        df_norm=np.array([np.linalg.norm(df)]), J=np.array([0.5 * np.sum((u - ut) ** 2)]))
    print("gradient golden written", time.time() - t0, "s; iterations", it0, it, itl)


def _batch_one(k):
    p = W.batch_256()[k].with_options(local_precision=0)
    t0 = time.time()
    s = OracleSolver(p)
    x, it, rel = s.solve(rtol=1e-8)
    rng = np.random.default_rng(1000 + k)
    idx = np.sort(rng.choice(s.n_dof, size=min(16, s.n_dof), replace=False))
    return {"k": k, "name": p.name, "n": p.n, "n_dof": int(s.n_dof), "n_coarse": int(s.topo.n_coarse),
            "iterations": int(it), "relres": float(rel), "norm": float(np.linalg.norm(x)),
            "dof_node_sha256": sha(s.d.dof_node.astype(np.int64)),
            "idx": idx.tolist(), "u": x[idx].tolist(), "seconds": time.time() - t0}


def batch(workers=6):
    """The 256-problem batch (FP64 oracle; the GPU batch runs FP32 local
    solves and is compared at the FP32 tolerance)."""
    from multiprocessing import Pool
    t0 = time.time()
    with Pool(workers) as pool:
        rows = []
        for r in pool.imap_unordered(_batch_one, range(256)):
            rows.append(r)
            print(f"{len(rows):3d}/256 problem {r['k']} n={r['n']} ndof={r['n_dof']} it={r['iterations']} "
                  f"{r['seconds']:.1f}s", flush=True)
    rows.sort(key=lambda r: r["k"])
    idx = np.full((256, 16), -1, dtype=np.int64)
    u = np.zeros((256, 16))
    for r in rows:
        idx[r["k"], :len(r["idx"])] = r["idx"]
        u[r["k"], :len(r["u"])] = r["u"]
    np.savez_compressed(os.path.join(HERE, "batch_256_sample.npz"), idx=idx, u=u,
                        norm=np.array([r["norm"] for r in rows]))
    meta = [{k: r[k] for k in ("k", "name", "n", "n_dof", "n_coarse", "iterations", "relres",
                               "dof_node_sha256")} for r in rows]
    with open(os.path.join(HERE, "batch_256.json"), "w") as fh:
        json.dump({"workload": "batch_256 (seed 3)", "rtol": 1e-8, "oracle_seconds": time.time() - t0,
                   "problems": meta}, fh, indent=0)
    print("batch golden written", time.time() - t0, "s")


def batch_full():
    """Whole solution vectors of one problem per mesh size of the batch (the
    first of each size), FP64 oracle at rtol 1e-8."""
    probs = W.batch_256()
    first = {}
    for k, p in enumerate(probs):
        first.setdefault(p.n, k)
    out = {"k": np.array(sorted(first.values()), dtype=np.int64)}
    for k in out["k"]:
        p = probs[k].with_options(local_precision=0)
        s = OracleSolver(p)
        x, it, rel = s.solve(rtol=1e-8)
        out[f"u{k}"] = x
        print(f"problem {k} n={p.n} n_dof={s.n_dof} iterations {it}", flush=True)
    np.savez_compressed(os.path.join(HERE, "batch_256_full.npz"), **out)


if __name__ == "__main__":
    arg = sys.argv[1] if len(sys.argv) > 1 else "64"
    if arg == "grad":
        gradient()
    elif arg == "batch":
        batch()
    elif arg == "batch_full":
        batch_full()
    else:
        main(arg)
