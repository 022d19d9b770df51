"""Benchmark: DOFs solved per second to rtol 1e-8 on one MI355X.

Workload (one "step" = the whole hot path on one synthetic problem): the
unit cube minus 20 seeded balls, 64^3 background cells, 8^3 subdomains of
8^3 cells, f ~ U(0,1) per node, kappa = 1.  A step runs cell classification
and cut-cell integration, host indexing, sub-assembly, the local and coarse
factorisations and the BDDC-preconditioned CG solve to |r| < 1e-8 |b|, and
releases the problem.  The source vector is resident in HBM before the
timed region; ball data are passed from the host (80 doubles).

Prints one JSON line.  `value` is the FP64 path; the FP32-local path (local
factorisations and solves in FP32, outer PCG and coarse solve in FP64) is
reported alongside with its speedup.  Also reported:
  * the 96^3 workload (40 balls, log-normal kappa, 12^3 subdomains) in FP64
    and FP32-local, each with its error against the FP64 oracle's stored
    solution sample and its iteration count against the oracle's, and the
    coarse factorisation's share of the step;
  * the batch of 256 independent problems (sizes 16^3..48^3, FP32 local)
    set up, factored and solved as one context (sum of their DOFs over the
    wall time of the whole batch), with the HBM rate of its three streaming
    kernels on first-sweep launches (every problem still iterating) and the
    MFMA rate of its local factorisation.

Kernel rates come from one more (untimed, profiled) cycle on the same
workload: the library brackets every launch of a kernel group with two HIP
events on the context stream (HIP graphs are off while profiling), so each
duration is that of a launch inside the solve.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
# HBM bytes per launch of apply_interior_kernel<double> on the 64^3 workload,
# from rocprofv3 FETCH_SIZE and WRITE_SIZE runs (profiles/
# apply_interior_cut_cube_64_traffic.md), each scaled by the same counter on
# a copy of known size (FETCH x 2.0, WRITE x 1.0).  Valid for the packed
# symmetric apply kernel as it stands; set to None when that kernel changes.
APPLY_INTERIOR_TRAFFIC_BYTES = 277.4e6
FP64_PEAK_TFLOPS = 78.6        # MI355X dense FP64 (vector and matrix)
FP32_PEAK_TFLOPS = 157.3       # MI355X dense FP32 matrix


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the 256-problem batch (for profiling) and print its object")
    ap.add_argument("--no-96", action="store_true", help="skip the 96^3 workload")
    ap.add_argument("--no-256", action="store_true", help="skip the 256^3 operator measurement")
    ap.add_argument("--steps-96", type=int, default=2)
    return ap.parse_args()


def run_steps(problem, f_dev, steps, warmup, rtol, profile, check=None):
    """Times `steps` setup + factor + solve cycles on the production path.
    With profile, one more (untimed) cycle follows with the library's
    per-launch event timing: kt holds the group totals, the in-solve launch
    durations of apply_interior (`apply_interior_launches_ms`) and, for
    comparison, its average over 20 back-to-back launches on the factored
    context.  check(u) (untimed, on that cycle) adds its result as
    kt["check"]."""
    import torch
    from paper_1703_06323_amd import Solver

    def one(prof):
        s = Solver(problem)
        if prof:
            s.profile(True)
        s.factor()
        u, it, rel = s.solve(f_dev, rtol=rtol)
        info = s.info()
        kt = {}
        if prof:
            kt = s.profile_times()
            kt["apply_interior_launches_ms"] = s.profile_launches("apply_interior")
            kt["apply_interior_b2b_ms"] = s.time_kernel("apply_interior", 20)
            if check is not None:
                kt["check"] = check(u)
        s.close()
        return it, rel, info, kt

    for _ in range(warmup):
        one(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [one(False) for _ in range(steps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    kt = one(True)[3] if profile else {}
    return dt, res, kt


def apply_bytes(info, probs, s_bytes):
    """Algorithmic HBM bytes of one launch of each streaming kernel, summed
    over the problems of a context (all of them active):
      apply_A: x read and y written once per node (16 B), the cell code of
        every cell (4 B), kappa of every active cell (8 B) and the packed
        unit stiffness of every stored cut cell (36 x 8 B);
      apply_interior: the unique entries of every subdomain's symmetric
        Dirichlet inverse (s_bytes each) plus 2.5 gathered / scattered
        vectors of n_I doubles on average (2 on the first launch of an
        apply, 3 on the second);
      apply_neumann: the unique entries of Kt and the n_G n_c entries of
        Phi (s_bytes each: Phi is kept in the local precision for these
        products) and four vectors of n_G doubles (two inputs, the weights,
        the output)."""
    nodes = sum((p.n + 1) ** 3 for p in probs)
    cells = sum(p.n ** 3 for p in probs)
    a = 16.0 * nodes + 4.0 * cells + 8.0 * info["n_active"] + 288.0 * info["n_cut_stored"]
    i = s_bytes * (info["sum_nI2"] + info["sum_nI"]) / 2.0 + 8.0 * 2.5 * info["sum_nI"]
    g = s_bytes * (info["sum_nG2"] + info["sum_nG"]) / 2.0 + s_bytes * info["sum_nGnC"] + 32.0 * info["sum_nG"]
    return {"apply_A": a, "apply_interior": i, "apply_neumann": g}


def hbm_rate(name, kernel, alg_bytes, launches_ms):
    import numpy as np
    d = np.asarray(launches_ms, dtype=np.float64)
    if d.size == 0:
        return None
    avg_s = float(d.mean()) * 1e-3
    achieved = alg_bytes / avg_s / 1e9
    return {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "launches": int(d.size), "avg_launch_us": avg_s * 1e6,
            "alg_bytes_per_launch": alg_bytes}


def run_batch(steps, warmup, rtol):
    """The 256-problem batch: per step, setup + factor + solve of every
    problem in one context, then release.  Sources resident in HBM.  One
    more (untimed) cycle is profiled for the kernel rates: first-sweep
    launches are those of the initial preconditioner apply and the first
    PCG iteration (apply_A 5, apply_interior 4, apply_neumann 2), when every
    problem still iterates."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1703_06323_amd import BatchSolver

    probs = W.batch_256()
    fs = [torch.tensor(p.f, dtype=torch.float64, device="cuda") for p in probs]

    def one(prof=False):
        b = BatchSolver(probs)
        if prof:
            b.profile(True)
        b.factor()
        us, its, rels = b.solve(fs, rtol=rtol)
        info = b.info()
        kt = {}
        if prof:
            kt = b.profile_times()
            for g in ("apply_A", "apply_interior", "apply_neumann"):
                kt[g + "_launches_ms"] = b.profile_launches(g)
        b.close()
        return its, rels, info, kt

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [one() for _ in range(steps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    its, rels, info, _ = res[-1]
    _, _, pinfo, kt = one(True)
    n_dof = int(info["n_dof"])
    sizes = {}
    for p in probs:
        sizes[f"{p.n}^3"] = sizes.get(f"{p.n}^3", 0) + 1
    rates = {}
    if int(np.min(its)) >= 2:
        by = apply_bytes(pinfo, probs, 4.0)
        first = {"apply_A": 5, "apply_interior": 4, "apply_neumann": 2}
        names = {"apply_A": "apply_A_kernel", "apply_interior": "apply_interior_kernel<float>",
                 "apply_neumann": "apply_neumann_kernel<float>"}
        for g, k in first.items():
            rates[g] = hbm_rate(g, names[g], by[g], kt[g + "_launches_ms"][:k])
    return {
        "value": n_dof / dt, "unit": "DOF/s", "ms_per_batch": dt * 1e3, "steps": steps, "warmup": warmup,
        "dtype": "f32 local factor/solves, f64 PCG and coarse",
        "workload": "batch_256 (seed 3): 256 independent cut cubes, N in {16,24,32,48} uniform, "
                    "5-30 balls each, f ~ U(0,1), 8^3-cell subdomains, PCG rtol 1e-8",
        "mesh_sizes": sizes, "n_dof_total": n_dof, "n_subdomains": int(info["n_sub"]),
        "n_coarse_total": int(info["n_coarse"]),
        "iterations": {"min": int(np.min(its)), "max": int(np.max(its)), "mean": float(np.mean(its))},
        "max_relres": float(np.max(rels)),
        "phase_ms": {k: round(float(info[k]), 3) for k in
                     ("t_integrate_ms", "t_topology_ms", "t_factor_ms", "t_solve_ms")},
        "flops_local_chol": float(info["flops_local_chol"]),
        "first_sweep_hbm": rates,
        "mfma": mfma_util(kt, pinfo, fp32=True),
    }


def run_operator_256(reps=10):
    """The operator alone on the 256^3 mesh (workloads.operator_256, setup
    only): `reps` applies of A-bar to a seeded vector through the C ABI with
    per-launch event timing; the working set is about twice the MALL, so
    every launch streams from HBM."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1703_06323_amd import Solver

    p = W.operator_256()
    s = Solver(p)
    inf = s.info()
    x = torch.as_tensor(np.random.default_rng(7).uniform(-1.0, 1.0, int(inf["n_dof"])), device="cuda")
    s.profile(True)
    for _ in range(reps):
        s.apply_operator(x)
    torch.cuda.synchronize()
    d = s.profile_launches("apply_A")
    by = apply_bytes(inf, [p], 8.0)["apply_A"]
    out = hbm_rate("apply_A", "apply_A_kernel", by, d)
    out.update({"workload": "operator_256_balls200: 256^3 cells, 200 balls r ~ U(0.02,0.05), kappa = 1",
                "n_dof": int(inf["n_dof"]), "n_cut": int(inf["n_cut_stored"]),
                "first_launch_us": float(d[0]) * 1e3 if len(d) else None})
    s.close()
    return out


def run_96(args, fp32):
    """The 96^3 workload (40 balls, log-normal kappa) with its error against
    the FP64 oracle's stored solution sample (16384 DOFs, written by
    tests/golden/make_golden.py from the oracle alone) and the oracle's
    iteration count."""
    import numpy as np
    import torch

    import workloads as W

    meta = json.load(open(os.path.join(ROOT, "tests", "golden", "cut_cube_96.json")))
    smp = np.load(os.path.join(ROOT, "tests", "golden", "cut_cube_96_sample.npz"))
    idx = torch.as_tensor(smp["idx"], device="cuda")
    ref = smp["u"]

    def check(u):
        v = u[idx].cpu().numpy()
        return float(np.linalg.norm(v - ref) / np.linalg.norm(ref))

    p = W.cut_cube_96_lognormal().with_options(local_precision=1 if fp32 else 0)
    f = torch.tensor(p.f, dtype=torch.float64, device="cuda")
    dt, res, kt = run_steps(p, f, args.steps_96, 1, args.rtol, profile=True, check=check)
    it, rel, info, _ = res[-1]
    n_dof = int(info["n_dof"])
    coarse = kt.get("coarse_factor", (0.0, 0))[0]
    return {
        "value": n_dof / dt, "unit": "DOF/s", "ms_per_step": dt * 1e3, "steps": args.steps_96, "warmup": 1,
        "dtype": "f32 local factor/solves, f64 PCG and coarse" if fp32 else "f64",
        "workload": "cut_cube_96_balls40_lognormal: unit cube minus 40 seeded balls, 96^3 Q1 cells, "
                    "12^3 subdomains of 8^3 cells, kappa = exp(N(0,1)) per cell, f ~ U(0,1)",
        "n_dof": n_dof, "n_coarse": int(info["n_coarse"]),
        "coarse_separator": int(info["coarse_separator"]), "coarse_octant_max": int(info["coarse_octant_max"]),
        "iterations": it, "relres": rel,
        "oracle_iterations": int(meta["iterations_rtol_1e-8"]),
        "iteration_change": it - int(meta["iterations_rtol_1e-8"]),
        "rel_error_vs_fp64_oracle": kt.get("check"),
        "phase_ms": {k: round(float(info[k]), 3) for k in
                     ("t_integrate_ms", "t_topology_ms", "t_factor_ms", "t_solve_ms")},
        "coarse_factor_ms": coarse,
        "coarse_factor_share_of_step": coarse / (dt * 1e3),
        "mfma": mfma_util(kt, info, fp32=fp32),
    }


def cpu_info():
    """CPU model and the BLAS library the oracle's NumPy / SciPy call."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = []
    try:
        from threadpoolctl import threadpool_info
        for d in threadpool_info():
            if d.get("user_api") == "blas":
                blas.append(f"{d.get('internal_api')} {d.get('version')} ({os.path.basename(d.get('filepath', ''))})")
    except Exception:  # noqa: BLE001  (reporting only)
        pass
    return model, ", ".join(sorted(set(blas))) or "unknown"


def cpu_baseline():
    """The oracle, as it stands, with as many BLAS threads as the host
    gives this process (at most 16, the host share of one GPU).  It first
    runs the octant [0, 0.5]^3 of the same 20-ball geometry at the same cell
    size (32^3 cells, 4^3 subdomains of 8^3 cells, mapped onto the unit
    cube); when eight times that time fits the budget (45 s) it then runs the
    whole workload and reports that, else it reports the octant.  Full path:
    integrate, indexing, factor, PCG to rtol 1e-8."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import OracleSolver

    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    model, blas = cpu_info()
    base = W.cut_cube_64()
    n = 32
    keep = np.ones(base.radii.size, dtype=bool)
    p = W.Problem(n=n, s=8, centres=base.centres[keep] * 2.0, radii=base.radii[keep] * 2.0,
                  name="octant_of_cut_cube_64")
    n1 = n + 1
    g = np.arange(n1 ** 3)
    I, J, K = g % n1, (g // n1) % n1, g // (n1 * n1)
    # the workload's nodal source restricted to the octant (same h)
    N1 = 65
    p.f = base.f[I + N1 * (J + N1 * K)]
    common = {"unit": "DOF/s", "cores": threads, "kind": "oracle", "cpu_model": model, "blas": blas,
              "host_cpus_visible": len(os.sched_getaffinity(0))}
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        s = OracleSolver(p)
        x, it, rel = s.solve(rtol=1e-8)
        dt = time.perf_counter() - t0
        if 8.0 * dt < 45.0:
            t0 = time.perf_counter()
            sf = OracleSolver(base)
            xf, itf, relf = sf.solve(rtol=1e-8)
            dtf = time.perf_counter() - t0
            return dict(common, value=sf.n_dof / dtf,
                        sample=(f"whole workload (64^3 cells, 512 subdomains, {sf.n_dof} DOFs, {itf} PCG "
                                f"iterations), full oracle path in {dtf:.1f} s with {threads} BLAS threads; "
                                f"octant probe {s.n_dof} DOFs in {dt:.1f} s"))
    return dict(common, value=s.n_dof / dt,
                sample=(f"octant [0,0.5]^3 of the workload at the same h: {n}^3 cells, "
                        f"{(n // 8) ** 3} subdomains of 8^3, {s.n_dof} DOFs, {it} PCG iterations, "
                        f"full oracle path in {dt:.1f} s with {threads} BLAS threads"))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as W
    from paper_1703_06323_amd import Solver  # noqa: F401  (fails loudly without the library)

    torch.cuda.set_device(0)
    if args.batch_only:
        print(json.dumps({"batch_256": run_batch(args.batch_steps, args.warmup, args.rtol)}), flush=True)
        return
    p64 = W.cut_cube_64()
    f_dev = torch.tensor(p64.f, dtype=torch.float64, device="cuda")

    dt64, res64, kt64 = run_steps(p64, f_dev, args.steps, args.warmup, args.rtol, profile=True)
    it64, rel64, info64, _ = res64[-1]
    n_dof = int(info64["n_dof"])
    out = {
        "metric": "DOFs solved/s to rtol 1e-8 (FP32-precond vs FP64) + MFMA util / HBM GB/s",
        "value": n_dof / dt64,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "cut_cube_64_balls20: unit cube minus 20 seeded balls, 64^3 Q1 cells, "
                        "8^3 subdomains of 8^3 cells, BDDC(cef) variant 1, stiffness weighting, "
                        "PCG rtol 1e-8, FP64",
            "n_dof": n_dof, "n_cut": int(info64["n_cut"]), "n_coarse": int(info64["n_coarse"]),
            "coarse_separator": int(info64["coarse_separator"]),
            "coarse_octant_max": int(info64["coarse_octant_max"]),
            "iterations": it64, "relres": rel64,
            "phase_ms": {k: round(float(info64[k]), 3) for k in
                         ("t_integrate_ms", "t_topology_ms", "t_factor_ms", "t_solve_ms")},
        },
    }
    if not args.no_fp32:
        from paper_1703_06323_amd import CBError
        p32 = p64.with_options(local_precision=1)
        try:
            dt32, res32, kt32 = run_steps(p32, f_dev, args.steps, args.warmup, args.rtol, profile=True)
        except CBError as e:
            res32 = None
            out["fp32_local"] = {"error": str(e)}
    if not args.no_fp32 and res32 is not None:
        it32, rel32, info32, _ = res32[-1]
        out["fp32_local"] = {
            "value": n_dof / dt32, "unit": "DOF/s", "ms_per_step": dt32 * 1e3,
            "iterations": it32, "relres": rel32, "speedup_vs_fp64": dt64 / dt32,
            "phase_ms": {k: round(float(info32[k]), 3) for k in
                         ("t_integrate_ms", "t_topology_ms", "t_factor_ms", "t_solve_ms")},
            "mfma": mfma_util(kt32, info32, fp32=True),
        }
    if not args.no_96:
        out["cut_cube_96"] = {"fp64": run_96(args, False)}
        if not args.no_fp32:
            out["cut_cube_96"]["fp32_local"] = run_96(args, True)
            out["cut_cube_96"]["fp32_speedup_vs_fp64"] = (out["cut_cube_96"]["fp32_local"]["value"] /
                                                          out["cut_cube_96"]["fp64"]["value"])
    if not args.no_batch:
        out["batch_256"] = run_batch(args.batch_steps, 1, args.rtol)
    if not args.no_256:
        out["operator_256"] = run_operator_256()
    # the step's dominant work is the local factorisation (MFMA); the HBM
    # rate of its largest streaming kernel is reported beside it
    out["roofline"] = mfma_roofline(kt64, info64)
    out["roofline_hbm"] = roofline(kt64, info64)
    out["mfma"] = mfma_util(kt64, info64)
    out["kernel_ms"] = {k: {"total_ms": round(v[0], 4), "launches": v[1]} for k, v in kt64.items()
                        if isinstance(v, tuple)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def roofline(kt, info):
    """Dominant kernel's achieved rate: algorithmic bytes per launch over
    the mean duration of its launches inside the profiled solve (two HIP
    events on the context stream around each launch).  The average over 20
    back-to-back launches on the factored context is reported beside it."""
    d = kt.get("apply_interior_launches_ms")
    if d is None or len(d) == 0:
        return None
    # per launch: the unique entries of every subdomain's symmetric
    # Dirichlet inverse (lower triangle with diagonal, 8 B each) plus the
    # gathered input(s) and the scattered output (2 vectors on the first
    # launch of an apply, 3 on the second: 2.5 on average)
    alg_bytes = 8.0 * (info["sum_nI2"] + info["sum_nI"]) / 2.0 + 8.0 * 2.5 * info["sum_nI"]
    out = hbm_rate("apply_interior", "apply_interior_kernel<double>", alg_bytes, d)
    out["traffic"] = APPLY_INTERIOR_TRAFFIC_BYTES
    out["timing"] = "mean of the in-solve launches of the profiled cycle"
    b2b = kt.get("apply_interior_b2b_ms")
    if b2b:
        out["back_to_back_us"] = b2b * 1e3
    return out


def mfma_roofline(kt, info):
    """The local factorisation as the roofline line: algorithmic Cholesky
    flops (active DOFs only) over the event-timed blocked Cholesky of all
    local matrices (its diagonal-block kernels, panel and trailing-update
    GEMMs), against the FP64 MFMA peak."""
    m = mfma_util(kt, info)
    if m is None:
        return None
    return {"bound": "mfma", "kernel": "local Cholesky: diag_block_kernel<double> + gemm_kernel<double> "
                                       "panels and trailing updates",
            "achieved": m["achieved"], "peak": m["peak"], "unit": "TFLOP/s", "frac": m["frac"],
            "traffic": None, "flops_per_factorisation": m["flops"], "ms": m["ms"],
            "timing": "HIP events around the local Cholesky of the profiled cycle"}


def mfma_util(kt, info, fp32=False):
    """MFMA utilisation of the subdomain factorisations: the algorithmic
    Cholesky flops, sum over subdomains of n_N^3/3 + n_I^3/3 with active DOFs
    only, over the event-timed blocked Cholesky of all local matrices
    (diagonal blocks, panels and trailing updates), against the dense peak
    of the type the factorisation runs in (FP64, or FP32 on the precision
    path)."""
    v = kt.get("local_cholesky")
    if not v or v[0] <= 0:
        return None
    flops = float(info["flops_local_chol"])
    tf = flops / (v[0] * 1e-3) / 1e12
    peak = FP32_PEAK_TFLOPS if fp32 else FP64_PEAK_TFLOPS
    return {"kernel": "local Cholesky (blocked, %s)" % ("FP32" if fp32 else "FP64"), "flops": flops, "ms": v[0],
            "achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak}


if __name__ == "__main__":
    main()
