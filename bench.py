"""Benchmark: PCG DOF/s to a 1e-8 relative residual on one MI355X.

Workload (one step = one full PCG solve, setup excluded): Poisson on the unit
cube, uniform Cartesian 16 x 16 x 16 hexahedra, Q_7 (1,367,631 free DOFs),
right-hand side from seeded U[-1, 1] samples at the quadrature points, hybrid
V(1,1) vertex-star FDM/sparse preconditioner with FP32 relaxation under FP64
PCG (the chosen form).  The plain FP64 path is timed beside it.  Inputs are
resident in HBM before the timed region starts.

Prints one JSON line.  --gpus above 1 is rejected: this build runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
WORKLOAD = "poisson_cart_16x16x16_q7"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha():
    with open(os.path.join(ROOT, "paper_2107_14758_amd", "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the interior patch-solve kernel from the committed rocprofv3
    counter summary, or None if the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "patch_interior_fp32_poisson_cart_16x16x16_q7_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != kernel_source_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def solve_timed(vsr, torch, w, relax_fp32, steps, warmup, profile):
    prob = vsr.Problem(w["vertices"], w["p"], kappa=w["kappa"], relax_fp32=relax_fp32, seed=0)
    n = prob.n
    f = torch.tensor(w["f"], dtype=torch.float64, device="cuda")
    b = torch.zeros(n, dtype=torch.float64, device="cuda")
    prob.load_vector(f, b)
    x = torch.zeros_like(b)
    info = None
    for _ in range(warmup):
        info = prob.pcg_solve(b, x, rtol=1e-8)
    if profile:
        prob.set_profiling(True)
        prob.kernel_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for _ in range(steps):
        info = prob.pcg_solve(b, x, rtol=1e-8)
        iters.append(info["iterations"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = prob.kernel_stats() if profile else None
    prob.set_profiling(False)
    npatch, nentries = prob.factor_info()
    out = dict(n=n, seconds=dt, iterations=iters[-1], info=info, stats=stats, setup_s=info["setup_seconds"],
               patches=npatch, factor_entries=nentries)
    prob.close()
    return out


def cpu_baseline(p, cells=4, seed=0):
    """The FP64 oracle (untuned) on a bounded sample of the workload: the same degree,
    RHS distribution and solver on a cells^3 Cartesian mesh; PCG solve time only."""
    from oracle.fdm1d import setup_1d
    from oracle.operator import Discretization
    from oracle.solver import Solver
    from paper_2107_14758_amd import inputs
    try:
        from threadpoolctl import threadpool_info
        cores = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        cores = 1
    w = inputs.make_problem(cells, p, seed=seed)
    d = Discretization(w["vertices"], p)
    b = d.load_vector(w["f"])
    s = Solver(d, setup_1d(p), seed=0)
    t0 = time.perf_counter()
    _, it = s.pcg(b)
    dt = time.perf_counter() - t0
    return {"value": d.n / dt, "unit": "DOF/s", "cores": int(cores), "kind": "oracle",
            "sample": f"oracle PCG solve (setup excluded) on a {cells}x{cells}x{cells}-cell Cartesian mesh at p={p}, "
                      f"{d.n} DOFs, {it} iterations, {dt:.1f} s; same RHS distribution and preconditioner"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is described, "
              f"not built", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy // 8
        src = torch.rand(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 8, "copies": 3}), flush=True)
        return
    from paper_2107_14758_amd import inputs, vsr
    vsr.lib()
    w = inputs.workload(WORKLOAD, seed=0)
    log(f"[bench] workload {WORKLOAD}: {len(w['f'])} cells, p={w['p']}")
    r32 = solve_timed(vsr, torch, w, True, args.steps, args.warmup, profile=True)
    log(f"[bench] fp32-relaxation: {r32['iterations']} iterations, {1e3 * r32['seconds'] / args.steps:.2f} ms/solve")
    r64 = None
    if not args.no_fp64:
        r64 = solve_timed(vsr, torch, w, False, max(3, args.steps // 4), 1, profile=False)
        log(f"[bench] fp64 plain: {r64['iterations']} iterations, "
            f"{1e3 * r64['seconds'] / max(3, args.steps // 4):.2f} ms/solve")
    n = r32["n"]
    ms = 1e3 * r32["seconds"] / args.steps
    value = n / (ms * 1e-3)
    launches, total_ms, bytes_per_launch = r32["stats"]
    avg_ms = total_ms / max(launches, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": measured_traffic(),
                "kernel": "k_patch_interior<float,7>", "avg_launch_ms": avg_ms, "launches": launches,
                "algorithmic_bytes_per_launch": bytes_per_launch}
    out = {
        "metric": "PCG DOF/s to 1e-8 rel. residual, FP32-precond vs FP64 plain; iters at p=7,15",
        "value": value, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (PCG, outer operator) + f32 (relaxation, coarse, inner operator)",
        "data": "synthetic (seeded U[-1,1] RHS at quadrature points)",
        "config": {"workload": WORKLOAD, "cells": [16, 16, 16], "p": 7, "dofs": n, "rtol": 1e-8,
                   "preconditioner": "hybrid V(1,1), vertex-star patches at all vertices, Q1 coarse",
                   "parallelism": "single GPU"},
        "iterations_p7": r32["iterations"],
        "true_rel_residual": r32["info"]["true_rel_residual"],
        "setup_seconds": r32["setup_s"],
        "patches": r32["patches"], "factor_entries": r32["factor_entries"],
        "roofline": roofline,
    }
    if r64:
        ms64 = 1e3 * r64["seconds"] / max(3, args.steps // 4)
        out["fp64_plain"] = {"value": n / (ms64 * 1e-3), "unit": "DOF/s", "ms_per_step": ms64,
                             "iterations": r64["iterations"], "true_rel_residual": r64["info"]["true_rel_residual"]}
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(7, cells=6)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
