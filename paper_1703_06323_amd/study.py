"""Algorithmic-scalability study on the GPU (paper Sect. 5.2): PCG iteration
counts and coarse-space sizes under mesh refinement at fixed subdomain size
(weak scaling), for H/h = s = 4, 8 and 16, with the BDDC variants of the
paper's methods table (standard objects, variant 1, variant 2; all with the
stiffness weighting, BDDC(cef)) and with full elements (every active cell
integrated as uncut: the body-fitted reference the paper compares with).
Neumann or Nitsche-Dirichlet data on the ball surfaces.

The geometry is fixed while the mesh is refined: the unit cube minus the 20
seeded balls of the 64^3 benchmark workload, f = 1.  Each run is a
setup + factor + solve to rtol 1e-8 through the C ABI.  Also reported: the
coarse DOFs per subdomain (the load-balance histogram of Sect. 5.2).

With --mms it reports instead the accuracy of the discretisation (Sect.
5.1): the L2 and H1-seminorm errors of the paper's exact solution
sin(5 pi |x|) and their rates under the same refinement, H/h = 8, both
kinds of ball-surface data, with the PCG iteration counts.

    python -m paper_1703_06323_amd.study [--quick] [--mms] [--subs 4,8,16]

prints one JSON object.  Subdomains of 12^3 cells and more run on the
large-subdomain kernels (block-row operator applies, assembly rows built
a few at a time).
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

METHODS = {          # name -> (coarse_variant, full_elements)
    "full_elements": (0, 1),
    "standard": (0, 0),
    "variant1": (1, 0),
    "variant2": (2, 0),
}


def run(ns=(16, 32, 48, 64, 96), subs=(4, 8, 16), boundaries=(0, 1), rtol=1e-8):
    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as W
    from paper_1703_06323_amd import CBError, Solver

    base = W.cut_cube_64()
    out = []
    for bc in boundaries:
        for s in subs:
            for n in ns:
                if n % s:
                    continue
                for name, (var, full) in METHODS.items():
                    p = W.Problem(n=n, s=s, centres=base.centres, radii=base.radii, coarse_variant=var,
                                  full_elements=full, cut_boundary=bc, name=f"weak_n{n}_s{s}")
                    row = {"boundary": "nitsche" if bc else "neumann", "H_over_h": s, "n": n,
                           "subdomains": (n // s) ** 3, "method": name}
                    try:
                        sol = Solver(p)
                        sol.factor()
                        _, it, rel = sol.solve(None, rtol=rtol)
                        inf = sol.info()
                        per_sub = _coarse_per_subdomain(sol, inf)
                        row.update({"iterations": it, "relres": rel, "n_dof": int(inf["n_dof"]),
                                    "n_coarse": int(inf["n_coarse"]),
                                    "coarse_per_sub": {"min": int(per_sub.min()), "max": int(per_sub.max()),
                                                       "mean": float(per_sub.mean())}})
                        sol.close()
                    except CBError as e:
                        row["error"] = str(e)
                    torch.cuda.synchronize()
                    out.append(row)
                    print(json.dumps(row), file=sys.stderr, flush=True)
    return out


def run_mms(ns=(32, 64, 128, 192), s=8, boundaries=(0, 1), rtol=1e-10, k=5.0 * np.pi):
    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as W
    from paper_1703_06323_amd import CBError, Solver

    base = W.cut_cube_64()
    out = []
    for bc in boundaries:
        prev = None
        for n in ns:
            p = W.Problem(n=n, s=s, centres=base.centres, radii=base.radii, cut_boundary=bc, name=f"mms_n{n}")
            row = {"boundary": "nitsche" if bc else "neumann", "H_over_h": s, "n": n, "k": k}
            try:
                sol = Solver(p)
                sol.factor()
                b = sol.manufactured_load((0.0, 0.0, 0.0), k)
                u, it, rel = sol.solve_rhs(b, rtol=rtol)
                l2, h1 = sol.manufactured_errors(u, (0.0, 0.0, 0.0), k)
                row.update({"iterations": it, "relres": rel, "l2": l2, "h1": h1})
                if prev is not None:
                    f = np.log(n / prev[0])
                    row["rate_l2"] = float(np.log(prev[1] / l2) / f)
                    row["rate_h1"] = float(np.log(prev[2] / h1) / f)
                prev = (n, l2, h1)
                sol.close()
            except CBError as e:
                row["error"] = str(e)
                prev = None
            torch.cuda.synchronize()
            out.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
    return out


def _coarse_per_subdomain(sol, inf):
    """Number of coarse DOFs whose object touches each (non-empty) subdomain."""
    g = sol.export_indexing()
    ptr, dofs = sol.export_subdomains()
    obj_of = np.full(int(inf["n_dof"]), -1, dtype=np.int64)
    for o in range(g["obj_type"].size):
        obj_of[g["obj_dofs"][g["obj_ptr"][o]:g["obj_ptr"][o + 1]]] = o
    counts = []
    for w in range(ptr.size - 1):
        d = dofs[ptr[w]:ptr[w + 1]]
        if d.size == 0:
            continue
        objs = np.unique(obj_of[d])
        objs = objs[objs >= 0]
        counts.append(int((g["coarse_of_obj"][objs] >= 0).sum()))
    return np.array(counts if counts else [0])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="N in {16, 32} only (--mms: {32, 64})")
    ap.add_argument("--mms", action="store_true", help="discretisation errors of the exact solution")
    ap.add_argument("--subs", default="4,8,16", help="subdomain sizes H/h of the weak-scaling study")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    if args.mms:
        rows = run_mms(ns=(32, 64) if args.quick else (32, 64, 128, 192))
        print(json.dumps({"study": "manufactured solution sin(5 pi |x|) (Sect. 5.1)", "rows": rows}))
        return
    subs = tuple(int(v) for v in args.subs.split(","))
    rows = run(ns=(16, 32) if args.quick else (16, 32, 48, 64, 96), subs=subs)
    print(json.dumps({"study": "weak scaling and H/h (Sect. 5.2)", "rows": rows}))


if __name__ == "__main__":
    main()
