"""Benchmark: PCG DOF/s to a 1e-8 relative residual on one MI355X.

Workload (one step = one full PCG solve, setup excluded): Poisson on the unit
cube, uniform Cartesian 16 x 16 x 16 hexahedra, Q_7 (1,367,631 free DOFs),
right-hand side from seeded U[-1, 1] samples at the quadrature points, hybrid
V(1,1) vertex-star FDM/sparse preconditioner with FP32 relaxation under FP64
PCG (the chosen form).  The plain FP64 path is timed beside it.  Inputs are
resident in HBM before the timed region starts.

--workload batch64 times the batched solve instead: 64 independent problems of uneven
size (cells per axis from {4, 6, 8, 12}, degree from {4, 7, 11, 15}, half the meshes
jittered), members spread over streams, one lockstep iteration replayed from a hipGraph,
launch shapes autotuned per degree; value = total DOFs of the batch / batch solve time.
The same members solved one after another are timed beside it.

--workload elasticity_8x8x8 times primal linear elasticity with the SDC relaxation (Sec.
3.1) on 8^3 boxes at Q7 (lambda = mu = 1), the operator's rate and the iteration table over
p in {3, 7, 15} and lambda in {0, 1, 10, 100, 1000}; the default line carries the same solve
as its "elasticity" entry.

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
WORKLOADS = ("poisson_cart_16x16x16_q7", "poisson_jitter_8x8x8_q15_lognormal", "poisson_jitter_12x12x12_q11_lognormal",
             "poisson_cart_32x32x32_q7")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha():
    """Hash of the sources that define the patch-solve kernel."""
    h = hashlib.sha256()
    for name in ("patch_kernels.h", "device_common.h"):
        with open(os.path.join(ROOT, "paper_2107_14758_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the patch-solve kernel from the committed rocprofv3
    counter summary, or None if the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "patch_all_fp32_poisson_cart_16x16x16_q7_counters.txt")
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


def error_vs_oracle(name, x):
    """Error of a solution against the FP64 oracle's PCG solution of the same workload, stored
    at sampled entries by tests/golden/make_fullsize_oracle.py (None if not stored): max-abs
    error over max |x_oracle| and 2-norm error over the 2-norm of x_oracle, on the sample."""
    path = os.path.join(ROOT, "tests", "golden", f"oracle_pcg_{name}.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    idx = np.array(g["indices"], dtype=np.int64)
    xo = np.array([float.fromhex(v) for v in g["x_sample_hex"]])
    if g["n"] != len(x):
        return None
    e = x[idx] - xo
    return {"max_abs_rel": float(np.abs(e).max() / np.abs(xo).max()),
            "norm2_rel": float(np.linalg.norm(e) / np.linalg.norm(xo)),
            "sampled_entries": int(len(idx)), "oracle_iterations": int(g["iterations"])}


def solve_timed(vsr, torch, w, relax_fp32, steps, warmup, profile, autotune=False, share_factors=False,
                coarse_solver="auto"):
    prob = vsr.Problem(w["vertices"], w["p"], kappa=w["kappa"], relax_fp32=relax_fp32, seed=0, autotune=autotune,
                       share_factors=share_factors, coarse_solver=coarse_solver)
    n = prob.n
    f = torch.tensor(w["f"], dtype=torch.float64, device="cuda")
    b = torch.zeros(n, dtype=torch.float64, device="cuda")
    prob.load_vector(f, b)
    x = torch.zeros_like(b)
    info = None
    for _ in range(warmup):
        info = prob.pcg_solve(b, x, rtol=1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for _ in range(steps):
        info = prob.pcg_solve(b, x, rtol=1e-8)
        iters.append(info["iterations"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = None
    if profile:
        # one more solve with HIP events around every patch-solve launch (host-driven, so
        # every recorded launch belongs to an iteration that did work)
        prob.set_profiling(True)
        prob.kernel_stats()
        prob.pcg_solve(b, x, rtol=1e-8)
        stats = prob.kernel_stats()
        prob.set_profiling(False)
    npatch, nentries = prob.factor_info()
    torch.cuda.synchronize()
    out = dict(n=n, seconds=dt, iterations=iters[-1], info=info, stats=stats, setup_s=info["setup_seconds"],
               patches=npatch, factor_entries=nentries, shapes=list(prob.tuning()), x=x.cpu().numpy())
    prob.close()
    return out


def batch_timed(vsr, torch, W, steps, warmup, share_factors=False):
    """Batched solve of the members of W (FP32 relaxation, autotuned shapes): seconds per
    batch solve, and per member the iterations; then the members solved one after another."""
    t0 = time.perf_counter()
    def progress(i, m):
        log(f"[bench] member {i}: {W[i]['n']}^3 cells p={W[i]['p']} n={m.n} set up, "
            f"{time.perf_counter() - t0:.1f} s")

    B = vsr.Batch([dict(vertices=w["vertices"], p=w["p"], kappa=w["kappa"]) for w in W], progress=progress,
                  relax_fp32=True, seed=0, autotune=True, share_factors=share_factors)
    setup_s = time.perf_counter() - t0
    log(f"[bench] batch setup {setup_s:.1f} s")
    bs, xs = [], []
    for m, w in zip(B.members, W):
        b = torch.zeros(m.n, dtype=torch.float64, device="cuda")
        m.load_vector(torch.tensor(w["f"], dtype=torch.float64, device="cuda"), b)
        bs.append(b)
        xs.append(torch.zeros_like(b))
    for _ in range(warmup):
        infos = B.pcg_solve(bs, xs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos = B.pcg_solve(bs, xs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    log(f"[bench] batched: {1e3 * dt:.1f} ms per batch solve")
    # the same members one after another (single solves, same shapes)
    for m, b, x in zip(B.members, bs, xs):
        m.pcg_solve(b, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for m, b, x in zip(B.members, bs, xs):
        m.pcg_solve(b, x)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    log(f"[bench] sequential single solves: {1e3 * seq:.1f} ms")
    # each member alone (synchronised around it): where the sequential time goes
    member_s = []
    for m, b, x in zip(B.members, bs, xs):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        m.pcg_solve(b, x)
        torch.cuda.synchronize()
        member_s.append(time.perf_counter() - t1)
    # dominant kernel: the patch solve of the largest member, profiled in a single solve
    big = max(range(len(W)), key=lambda i: B.members[i].n)
    m = B.members[big]
    m.set_profiling(True)
    m.kernel_stats()
    m.pcg_solve(bs[big], xs[big])
    stats = m.kernel_stats()
    m.set_profiling(False)
    out = dict(seconds=dt, sequential_seconds=seq, member_seconds=member_s, infos=infos, setup_s=setup_s, stats=stats, big=big,
               shapes={f"p{W[i]['p']}-{'jittered' if W[i]['jitter'] else 'cartesian'}": B.members[i].tuning()
                       for i in range(len(W))})
    B.close()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, cells=6, seed=0, workload=WORKLOAD):
    """The FP64 oracle (untuned) on a bounded sample of the workload: a cells^3 Cartesian mesh
    at the same degree, with the same right-hand side distribution, preconditioner and
    tolerance (a full solve of the 16^3 Q7 workload takes the oracle minutes of setup and
    solve).  The PCG solve is timed (setup excluded) twice: with numpy's BLAS pool held to one
    thread, which is the headline (the oracle's patch loops are single-threaded Python, so one
    thread is what it uses), and with the pool at its default size."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle.fdm1d import setup_1d
    from oracle.operator import Discretization
    from oracle.solver import Solver
    from paper_2107_14758_amd import inputs
    w = inputs.make_problem(cells, p, seed=seed)
    d = Discretization(w["vertices"], p)
    b = d.load_vector(w["f"])
    s = Solver(d, setup_1d(p), seed=0)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        _, it = s.pcg(b)
        dt1 = time.perf_counter() - t0
    pool = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    t0 = time.perf_counter()
    _, it2 = s.pcg(b)
    dtn = time.perf_counter() - t0
    return {"value": d.n / dt1, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "sample": f"{workload}: the oracle's PCG solve (setup excluded) on a {cells}x{cells}x{cells}-cell "
                      f"Cartesian mesh at p={p} ({d.n} DOFs, {it} iterations, {dt1:.1f} s) with the same degree, "
                      f"right-hand side distribution, preconditioner and tolerance",
            "threads": 1, "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "blas_pool": {"value": d.n / dtn, "threads": int(pool), "seconds": dtn, "iterations": it2,
                          "note": "numpy BLAS pool at its default size; the patch loops stay single-threaded"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-table", action="store_true", help="elasticity: skip the iteration table over p and lambda")
    ap.add_argument("--workload", default=WORKLOAD, choices=sorted(list(WORKLOADS) + ["batch64", "elasticity_8x8x8"]))
    ap.add_argument("--autotune", action="store_true", help="single-problem workloads: autotune launch shapes")
    ap.add_argument("--share-factors", action="store_true",
                    help="batch64: stars with equal scalings share one stored factor")
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
    if args.workload == "batch64":
        return main_batch(args, torch, inputs, vsr)
    if args.workload == "elasticity_8x8x8":
        return main_elasticity(args, torch, inputs, vsr)
    wname = args.workload
    w = inputs.workload(wname, seed=0)
    p = int(w["p"])
    ncell = len(w["f"])
    log(f"[bench] workload {wname}: {ncell} cells, p={p}")
    r32 = solve_timed(vsr, torch, w, True, args.steps, args.warmup, profile=True, autotune=args.autotune)
    log(f"[bench] fp32-relaxation: {r32['iterations']} iterations, {1e3 * r32['seconds'] / args.steps:.2f} ms/solve")
    r64 = None
    if not args.no_fp64:
        r64 = solve_timed(vsr, torch, w, False, max(3, args.steps // 4), 1, profile=False, autotune=args.autotune)
        log(f"[bench] fp64 plain: {r64['iterations']} iterations, "
            f"{1e3 * r64['seconds'] / max(3, args.steps // 4):.2f} ms/solve")
    n = r32["n"]
    ms = 1e3 * r32["seconds"] / args.steps
    value = n / (ms * 1e-3)
    roofline = patch_roofline(r32["stats"], p, measured_traffic() if wname == WORKLOAD and not args.autotune else None)
    nc = round(ncell ** (1 / 3))
    out = {
        "metric": "PCG DOF/s to 1e-8 rel. residual, FP32-precond vs FP64 plain; iters at p=7,15",
        "value": value, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (PCG, outer operator) + f32 (relaxation, coarse, inner operator)",
        "data": "synthetic (seeded U[-1,1] RHS at quadrature points)",
        "config": {"workload": wname, "cells": [nc, nc, nc], "p": p, "dofs": n, "rtol": 1e-8,
                   "preconditioner": "hybrid V(1,1), vertex-star patches at all vertices, Q1 coarse",
                   "autotune": bool(args.autotune), "launch_shapes": r32["shapes"], "parallelism": "single GPU"},
        f"iterations_p{p}": r32["iterations"],
        "true_rel_residual": r32["info"]["true_rel_residual"],
        "kappa_estimate": r32["info"]["kappa_estimate"],
        "setup_seconds": r32["setup_s"],
        "patches": r32["patches"], "factor_entries": r32["factor_entries"],
        "roofline": roofline,
    }
    out["fp32_err_vs_oracle"] = error_vs_oracle(wname, r32["x"])
    if r64:
        ms64 = 1e3 * r64["seconds"] / max(3, args.steps // 4)
        out["fp64_plain"] = {"value": n / (ms64 * 1e-3), "unit": "DOF/s", "ms_per_step": ms64,
                             "iterations": r64["iterations"], "true_rel_residual": r64["info"]["true_rel_residual"],
                             "err_vs_oracle": error_vs_oracle(wname, r64["x"])}
    if wname == WORKLOAD and not args.no_fp64:
        # iterations and rates at p = 15 on the 8^3 jittered log-normal workload
        w15 = inputs.workload("poisson_jitter_8x8x8_q15_lognormal", seed=0)
        a = solve_timed(vsr, torch, w15, True, 2, 1, profile=False)
        b = solve_timed(vsr, torch, w15, False, 2, 1, profile=False)
        out["iterations_p15"] = a["iterations"]
        out["p15"] = {"workload": "poisson_jitter_8x8x8_q15_lognormal", "dofs": a["n"],
                      "value": a["n"] / (a["seconds"] / 2), "fp64_plain_value": b["n"] / (b["seconds"] / 2),
                      "iterations": a["iterations"], "iterations_fp64": b["iterations"], "unit": "DOF/s",
                      "true_rel_residual": a["info"]["true_rel_residual"], "kappa_estimate": a["info"]["kappa_estimate"]}
        log(f"[bench] p=15: {a['iterations']} iterations, {1e3 * a['seconds'] / 2:.1f} ms/solve FP32-relaxation, "
            f"{1e3 * b['seconds'] / 2:.1f} ms FP64")
        # every interior star of this mesh is the same: one stored factor shared by all (an option,
        # not the headline; the factor then stays in cache instead of streaming from HBM)
        rs = solve_timed(vsr, torch, w, True, args.steps, 1, profile=True, autotune=args.autotune, share_factors=True)
        ms_s = 1e3 * rs["seconds"] / args.steps
        launches, total_ms, _ = rs["stats"]
        out["shared_factors"] = {"value": rs["n"] / (ms_s * 1e-3), "unit": "DOF/s", "ms_per_step": ms_s,
                                 "iterations": rs["iterations"], "true_rel_residual": rs["info"]["true_rel_residual"],
                                 "patch_kernel_ms": total_ms / max(launches, 1), "factor_entries": rs["factor_entries"]}
        log(f"[bench] shared factors: {rs['iterations']} iterations, {ms_s:.2f} ms/solve")
        # the coarse problem by geometric multigrid instead of the dense inverse (Sec. 2.8)
        rg = solve_timed(vsr, torch, w, True, args.steps, 1, profile=False, coarse_solver="gmg")
        ms_g = 1e3 * rg["seconds"] / args.steps
        out["gmg_coarse"] = {"value": rg["n"] / (ms_g * 1e-3), "unit": "DOF/s", "ms_per_step": ms_g,
                             "iterations": rg["iterations"], "true_rel_residual": rg["info"]["true_rel_residual"]}
        log(f"[bench] multigrid coarse solve: {rg['iterations']} iterations, {ms_g:.2f} ms/solve")
        # h-scaling: 32^3 cells at p = 7 (11.1M DOFs), coarse problem by multigrid (29,791 Q1
        # unknowns: the dense inverse would hold 7 GB and take hours to form)
        w32 = inputs.workload("poisson_cart_32x32x32_q7", seed=0)
        r32h = solve_timed(vsr, torch, w32, True, 3, 1, profile=False)
        ms_h = 1e3 * r32h["seconds"] / 3
        out["h_scaling"] = {"workload": "poisson_cart_32x32x32_q7", "dofs": r32h["n"], "coarse_solver": "gmg",
                            "value": r32h["n"] / (ms_h * 1e-3), "unit": "DOF/s", "ms_per_step": ms_h,
                            "iterations": r32h["iterations"], "setup_seconds": r32h["setup_s"],
                            "true_rel_residual": r32h["info"]["true_rel_residual"]}
        log(f"[bench] 32^3 Q7: {r32h['iterations']} iterations, {ms_h:.1f} ms/solve, setup {r32h['setup_s']:.1f} s")
        del w32, r32h
        # primal linear elasticity with the SDC relaxation (Sec. 3.1): 8^3 boxes, Q7, mu = lam = 1
        ge, _, _, ie, dte = elasticity_solve_timed(vsr, torch, 8, 7, 1.0, 1.0, True, args.steps, 2)
        out["elasticity"] = {"workload": "elasticity_8x8x8_q7", "dofs": ge.n, "value": ge.n / dte, "unit": "DOF/s",
                             "ms_per_step": 1e3 * dte, "iterations": ie["iterations"],
                             "kappa_estimate": ie["kappa_estimate"], "true_rel_residual": ie["true_rel_residual"]}
        ge.close()
        log(f"[bench] elasticity 8^3 Q7: {ie['iterations']} iterations, {1e3 * dte:.2f} ms/solve")
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(p, cells=8 if p <= 7 else 3, workload=wname)
    print(json.dumps(out), flush=True)


def patch_roofline(stats, p, traffic):
    launches, total_ms, bytes_per_launch = stats
    avg_ms = total_ms / max(launches, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "kernel": f"k_patch_all<float,{p}>",
            "avg_launch_ms": avg_ms, "launches": launches, "algorithmic_bytes_per_launch": bytes_per_launch}


def elasticity_problem(n, p, seed=0):
    """Primal elasticity workload: the unit cube in n^3 boxes, a seeded U[-1, 1] body force
    sampled at every quadrature point of every cell, per component."""
    rng = np.random.default_rng(seed)
    q = inputs_mod().quadrature_points_per_dir(p)
    f = np.stack([inputs_mod().rhs_samples(n ** 3, q ** 3, rng) for _ in range(3)])
    return inputs_mod().cube_vertices(n, n, n), f


def inputs_mod():
    from paper_2107_14758_amd import inputs
    return inputs


def elasticity_solve_timed(vsr, torch, n, p, mu, lam, relax_fp32, steps, warmup):
    V, f = elasticity_problem(n, p)
    g = vsr.Elasticity(V, p, mu, lam, relax_fp32=relax_fp32, seed=0)
    b = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    g.load_vector(torch.tensor(f, device="cuda"), b)
    x = torch.zeros_like(b)
    info = None
    for _ in range(warmup):
        info = g.pcg_solve(b, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        info = g.pcg_solve(b, x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(steps, 1)
    return g, b, x, info, dt


def main_elasticity(args, torch, inputs, vsr):
    """Primal linear elasticity with the SDC relaxation (Sec. 3.1) on the paper's mesh (8^3
    boxes of the unit cube), mu = 1: the headline rate at p = 7, lam = 1, the iteration table
    over p and lam of Table tab:primal_elasticity, the operator kernel's rate, and the oracle on
    a bounded sample."""
    n, p, lam = 8, 7, 1.0
    g, b, x, info, dt = elasticity_solve_timed(vsr, torch, n, p, 1.0, lam, True, args.steps, args.warmup)
    log(f"[bench] elasticity 8^3 p=7 lam=1: {info['iterations']} iterations, {1e3 * dt:.2f} ms/solve, setup {info['setup_seconds']:.1f} s")
    # operator: kernel + three gathers, timed over 20 applies
    y = torch.zeros_like(b)
    for _ in range(3):
        g.apply_operator(x, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        g.apply_operator(x, y)
    e1.record()
    torch.cuda.synchronize()
    op_us = 1e3 * e0.elapsed_time(e1) / 20
    n1 = p + 1
    op_flops = n ** 3 * 21 * 3 * 2 * n1 ** 4          # 21 Kronecker terms, three 1-D passes each
    out = {
        "metric": "PCG DOF/s to 1e-8 rel. residual, SDC-relaxation elasticity", "value": g.n / dt, "unit": "DOF/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 (PCG, outer operator) + f32 (V-cycle: component relaxations, inner operators, coarse solve)",
        "data": "synthetic (seeded U[-1,1] body force at quadrature points)",
        "config": {"workload": "elasticity_8x8x8_q7", "cells": [n, n, n], "p": p, "mu": 1.0, "lambda": lam, "dofs": g.n,
                   "rtol": 1e-8, "preconditioner": "hybrid V(1,1), SDC vertex-star FDM relaxation, vector Q1 coarse",
                   "boundary": "homogeneous Dirichlet on the whole boundary", "parallelism": "single GPU"},
        "iterations": info["iterations"], "kappa_estimate": info["kappa_estimate"],
        "true_rel_residual": info["true_rel_residual"], "setup_seconds": info["setup_seconds"],
        # the FP64 operator apply (kernel and the one gather launch, HIP events around 20 applies
        # on the library's stream): flops of the 21 Kronecker terms against the FP64 vector peak
        "roofline": {"bound": "alu", "achieved": op_flops / (op_us * 1e-6) / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                     "frac": op_flops / (op_us * 1e-6) / 78.6e12, "traffic": None,
                     "kernel": "k_op_elastic_box<double,7> + k_gather", "avg_launch_us": op_us,
                     "flops_per_launch": op_flops},
    }
    g.close()
    if not args.no_fp64:
        g64, _, _, info64, dt64 = elasticity_solve_timed(vsr, torch, n, p, 1.0, lam, False, max(3, args.steps // 4), 1)
        out["fp64_plain"] = {"value": g64.n / dt64, "ms_per_step": 1e3 * dt64, "iterations": info64["iterations"]}
        g64.close()
    table = {}
    for pp in (() if args.no_table else (3, 7, 15)):
        row = {}
        for lm in (0.0, 1.0, 10.0, 100.0, 1000.0):
            gg, _, _, ii, dtt = elasticity_solve_timed(vsr, torch, n, pp, 1.0, lm, True, 1, 0)
            row[str(lm)] = {"iterations": ii["iterations"], "kappa_estimate": round(ii["kappa_estimate"], 3),
                            "ms": round(1e3 * dtt, 2)}
            log(f"[bench] p={pp} lam={lm}: {ii['iterations']} iterations, kappa {ii['kappa_estimate']:.2f}")
            gg.close()
        table[f"p{pp}"] = row
    if table:
        out["iterations_table"] = table
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = elasticity_cpu_baseline(vsr, torch)
    print(json.dumps(out), flush=True)


def elasticity_cpu_baseline(vsr, torch, n=4, p=7):
    """The oracle's SDC PCG solve (setup excluded) on a 4^3-box sample at p = 7, lam = 1, and
    the GPU solution's error against it."""
    import threadpoolctl
    from oracle.elasticity import Elasticity as OE, SDCSolver
    from oracle.fdm1d import setup_1d
    from oracle.operator import Discretization
    V, f = elasticity_problem(n, p)
    with threadpoolctl.threadpool_limits(1):
        d = Discretization(V, p)
        el = OE(d, 1.0, 1.0)
        s = SDCSolver(el, setup_1d(p), seed=0)
        bo = el.load_vector(f)
        t0 = time.perf_counter()
        xo, it, _ = s.pcg(bo)
        dt = time.perf_counter() - t0
    g = vsr.Elasticity(V, p, 1.0, 1.0, relax_fp32=True, seed=0)
    b = torch.tensor(bo, device="cuda")
    x = torch.zeros_like(b)
    info = g.pcg_solve(b, x)
    xg = x.cpu().numpy()
    g.close()
    return {"value": el.n / dt, "unit": "DOF/s", "cores": 1, "kind": "oracle", "threads": 1,
            "sample": f"elasticity {n}^3 boxes, p={p}, lam=1: the oracle's PCG solve (setup excluded), "
                      f"{el.n} DOFs, {it} iterations, {dt:.1f} s",
            "gpu_fp32_err_vs_oracle": float(np.abs(xg - xo).max() / np.abs(xo).max()),
            "gpu_iterations": info["iterations"], "oracle_iterations": it}


def main_batch(args, torch, inputs, vsr):
    W = inputs.batch_workload(64, seed=0)
    n_total = sum((int(w["p"]) * int(w["n"]) - 1) ** 3 for w in W)
    log(f"[bench] batch of {len(W)} problems, {n_total} DOFs in total")
    steps, warmup = max(1, min(args.steps, 5)), max(1, min(args.warmup, 1))
    r = batch_timed(vsr, torch, W, steps, warmup, share_factors=args.share_factors)
    infos = r["infos"]
    big = r["big"]
    out = {
        "metric": "PCG DOF/s to 1e-8 rel. residual, batch of 64 uneven problems",
        "value": n_total / r["seconds"], "unit": "DOF/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": 1e3 * r["seconds"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (PCG, outer operator) + f32 (relaxation, coarse, inner operator)",
        "data": "synthetic (seeded U[-1,1] RHS at quadrature points; seeded sizes, degrees and jitter)",
        "config": {"workload": "batch64_uneven_p4-15", "problems": len(W), "dofs": n_total, "rtol": 1e-8,
                   "cells_per_axis": sorted(set(int(w["n"]) for w in W)), "degrees": sorted(set(int(w["p"]) for w in W)),
                   "launch": "lockstep iteration replayed from one hipGraph over 4 streams",
                   "share_factors": bool(args.share_factors),
                   "autotuned_shapes": {str(k): list(v) for k, v in sorted(r["shapes"].items())},
                   "parallelism": "single GPU"},
        "iterations_min_max": [min(i["iterations"] for i in infos), max(i["iterations"] for i in infos)],
        "max_true_rel_residual": max(i["true_rel_residual"] for i in infos),
        "setup_seconds": r["setup_s"],
        "sequential": {"value": n_total / r["sequential_seconds"], "unit": "DOF/s",
                       "ms": 1e3 * r["sequential_seconds"]},
        "roofline": patch_roofline(r["stats"], int(W[big]["p"]), None),
    }
    # the members of at least 1M DOFs fill the GPU on their own; overlap in the batch can only
    # hide the time of the others
    ms = r["member_seconds"]
    dofs = [(int(w["p"]) * int(w["n"]) - 1) ** 3 for w in W]
    large = [i for i in range(len(W)) if dofs[i] >= 1_000_000]
    out["members"] = {"ms_each": [round(1e3 * t, 3) for t in ms], "dofs_each": dofs,
                      "large_count": len(large), "large_ms": 1e3 * sum(ms[i] for i in large),
                      "small_ms": 1e3 * sum(ms[i] for i in range(len(W)) if i not in large)}
    out["roofline"]["member"] = f"{W[big]['n']}^3 cells p={W[big]['p']} (largest), single solve"
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(4, cells=4, workload="batch64_uneven_p4-15")
        out["cpu_baseline"]["sample"] += " (the smallest member class of the batch)"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
