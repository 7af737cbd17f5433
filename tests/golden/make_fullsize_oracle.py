"""Write the oracle's PCG solutions of the full-size workloads as sampled fixtures.

Calls only the FP64 oracle (``oracle/``) and the seeded input generators
(``paper_2107_14758_amd/inputs.py``, which draw numbers and hold none of the
method's arithmetic).  For each workload it solves A x = b (b from the oracle's
load vector of the seeded right-hand side samples) by the oracle's PCG with the
hybrid V(1,1) vertex-star preconditioner (Sec. 2.5, 2.8: x0 = 0, stop at
||r||_2 <= 1e-8 ||b||_2, Lanczos damping from seed 0), and writes

  oracle_pcg_<workload>.json

with the iteration count, the damping and its Lanczos estimates, the extreme
Ritz values of the solve's own Lanczos tridiagonal (condition estimate, Table
tab:poisson-cond), the final recursive residual, ||x||_2, max |x|, and x at
SAMPLES entries drawn uniformly
without replacement by numpy's PCG64 generator seeded with SAMPLE_SEED (values
as exact hexadecimal floats).  A full solve of the 16^3 Q7 workload takes the
oracle about half an hour on 8 cores, so the GPU tests compare against these
stored samples instead of re-solving.

Usage: python tests/golden/make_fullsize_oracle.py [workload ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.fdm1d import setup_1d  # noqa: E402
from oracle.operator import Discretization  # noqa: E402
from oracle.solver import Solver  # noqa: E402
from paper_2107_14758_amd import inputs  # noqa: E402

SAMPLES = 2048
SAMPLE_SEED = 20260
WORKLOADS = ("poisson_cart_16x16x16_q7", "poisson_jitter_8x8x8_q15_lognormal",
             "poisson_jitter_12x12x12_q11_lognormal")


def sample_indices(n):
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.sort(rng.choice(n, size=min(SAMPLES, n), replace=False))


def main(names):
    for name in names:
        t0 = time.time()
        w = inputs.workload(name, seed=0)
        p = w["p"]
        d = Discretization(w["vertices"], p, w["kappa"])
        b = d.load_vector(w["f"])
        s = Solver(d, setup_1d(p), seed=0)
        print(f"{name}: n={d.n}, omega={s.omega:.6f}, setup {time.time() - t0:.0f} s", flush=True)
        x, it, hist, (rmin, rmax) = s.pcg(b, rtol=1e-8, history=True, lanczos=True)
        idx = sample_indices(d.n)
        out = {
            "workload": name, "seed": 0, "p": p, "n": int(d.n), "rtol": 1e-8,
            "solver": "oracle.solver.Solver(seed=0).pcg, FP64, hybrid V(1,1), patches at all vertices",
            "iterations": int(it), "omega": s.omega, "lambda_min": s.lanczos[0], "lambda_max": s.lanczos[1],
            "ritz_min": rmin, "ritz_max": rmax, "final_rel_residual": hist[-1] / hist[0], "b_norm2": float(np.linalg.norm(b)),
            "x_norm2": float(np.linalg.norm(x)), "x_maxabs": float(np.abs(x).max()),
            "sample_seed": SAMPLE_SEED, "indices": [int(i) for i in idx],
            "x_sample_hex": [float(v).hex() for v in x[idx]],
        }
        path = os.path.join(HERE, f"oracle_pcg_{name}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=0)
        print(f"{name}: {it} iterations, {time.time() - t0:.0f} s -> {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or WORKLOADS)
