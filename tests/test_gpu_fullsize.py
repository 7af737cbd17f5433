"""GPU parity at the full workload sizes, in the configuration bench.py times.

The oracle cannot solve these sizes within a test, so each check uses what it can
compute: the full operator apply and load vector (sum factorization is cheap), the
relaxation on sampled cells (the values on a cell's nodes depend only on the patches
of the cell's eight vertices), the true residual recomputed by the oracle's operator,
and the oracle's own PCG solution, stored at 2048 sampled entries (with its iteration
count, damping and norms) by tests/golden/make_fullsize_oracle.py, which calls only
the oracle.  The FP64 solve must match it to 1e-10 and the FP32-relaxation solve
(the benchmarked form) to 1e-6, entry by entry (max-abs over the sample) and in the
2-norm over the sample.
"""
import json
import os

import numpy as np
import pytest

from oracle import transfer
from oracle.fdm1d import setup_1d
from oracle.operator import Discretization, kron3
from oracle.patches import Patches
from paper_2107_14758_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WORKLOADS = [
    ("poisson_cart_16x16x16_q7", [(0, 0, 0), (7, 8, 9), (15, 3, 15)]),
    ("poisson_jitter_8x8x8_q15_lognormal", [(0, 0, 0), (3, 4, 2), (0, 3, 7)]),
    ("poisson_jitter_12x12x12_q11_lognormal", [(11, 11, 11), (5, 6, 7), (0, 11, 4)]),
]


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)


def golden(name):
    path = os.path.join(GOLDEN, f"oracle_pcg_{name}.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    g["idx"] = np.array(g["indices"], dtype=np.int64)
    g["xs"] = np.array([float.fromhex(v) for v in g["x_sample_hex"]])
    return g


def sampled_errors(x, g):
    """(max-abs error / max |x_oracle|, 2-norm error / 2-norm of x_oracle), over the sample."""
    e = x[g["idx"]] - g["xs"]
    return float(np.abs(e).max() / np.abs(g["xs"]).max()), float(np.linalg.norm(e) / np.linalg.norm(g["xs"]))


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def cell_free_nodes(d, cell):
    """Free-DOF indices and the mask of free nodes of one cell, local order x fastest."""
    ez, ey, ex = cell
    p = d.p
    k = np.arange(p + 1)
    K, J, I = np.meshgrid(p * ez + k, p * ey + k, p * ex + k, indexing="ij")
    Fz, Fy, Fx = d.full_shape
    free = (K > 0) & (K < Fz - 1) & (J > 0) & (J < Fy - 1) & (I > 0) & (I < Fx - 1)
    Lz, Ly, Lx = d.free_shape
    idx = ((K - 1) * Ly + (J - 1)) * Lx + (I - 1)
    return idx.reshape(-1), free.reshape(-1)


def oracle_relax_on_cell(d, od, pt, rF, cell):
    """z = T sum_j Rbar_j^T A_j^{-1} Rbar_j T^T r restricted to one cell's nodes."""
    ez, ey, ex = cell
    uF = np.zeros(d.n)
    for vz in (ez, ez + 1):
        for vy in (ey, ey + 1):
            for vx in (ex, ex + 1):
                v = (vz, vy, vx)
                idx = pt.dofs(v)
                uF[idx] += pt.solve(v, rF[idx], cache=False)
    idx, free = cell_free_nodes(d, cell)
    uc = np.where(free, uF[np.where(free, idx, 0)], 0.0)
    return kron3(od["T"], od["T"], od["T"]) @ uc


@pytest.fixture(scope="module")
def vsr():
    from paper_2107_14758_amd import vsr as v
    v.lib()
    return v


@pytest.mark.parametrize("name,cells", WORKLOADS)
def test_fullsize(vsr, name, cells):
    say("case", name)
    w = inputs.workload(name, seed=0)
    p = w["p"]
    d = Discretization(w["vertices"], p, w["kappa"])
    od = setup_1d(p)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    host = lambda t: (torch.cuda.synchronize(), t.cpu().numpy())[1]
    prob64 = vsr.Problem(w["vertices"], p, kappa=w["kappa"], seed=0)
    assert prob64.n == d.n
    # operator and load vector, every entry
    x = np.random.default_rng(1).uniform(-1, 1, d.n)
    y = torch.zeros(d.n, dtype=torch.float64, device="cuda")
    prob64.apply_operator(dev(x), y)
    assert rel(host(y), d.apply(x)) < 1e-12
    b = torch.zeros_like(y)
    prob64.load_vector(dev(w["f"]), b)
    b_o = d.load_vector(w["f"])
    assert rel(host(b), b_o) < 1e-12
    # relaxation on sampled cells
    r = np.random.default_rng(2).uniform(-1, 1, d.n)
    z = torch.zeros_like(y)
    prob64.apply_relaxation(dev(r), z, 1)
    zh = host(z)
    rF = transfer.fdm_restrict(d, od["T"], r)
    pt = Patches(d, od)
    for cell in cells:
        idx, free = cell_free_nodes(d, cell)
        zo = oracle_relax_on_cell(d, od, pt, rF, cell)[free]
        assert rel(zh[idx[free]], zo) < 1e-11, cell
    # FP64 and FP32-relaxation solves: true residual by the oracle's operator
    x64 = torch.zeros_like(y)
    info64 = prob64.pcg_solve(b, x64)
    damping64 = prob64.damping()
    prob64.close()
    prob32 = vsr.Problem(w["vertices"], p, kappa=w["kappa"], seed=0, relax_fp32=True)
    x32 = torch.zeros_like(y)
    info32 = prob32.pcg_solve(b, x32)
    prob32.close()
    xh64, xh32 = host(x64), host(x32)
    res64 = np.linalg.norm(b_o - d.apply(xh64)) / np.linalg.norm(b_o)
    res32 = np.linalg.norm(b_o - d.apply(xh32)) / np.linalg.norm(b_o)
    say(f"  iterations fp64 {info64['iterations']} fp32 {info32['iterations']} res {res64:.2e} {res32:.2e}")
    assert info64["converged"] and info32["converged"]
    assert res64 <= 1.0001e-8 and res32 <= 1.0001e-8
    assert info32["iterations"] <= info64["iterations"] + 2
    assert rel(xh32, xh64) < 1e-6
    # the oracle's own solution (stored samples)
    g = golden(name)
    if g is None:
        pytest.skip(f"no stored oracle solution for {name} (tests/golden/make_fullsize_oracle.py writes it)")
    assert g["n"] == d.n and abs(np.linalg.norm(b_o) - g["b_norm2"]) <= 1e-12 * g["b_norm2"]
    e64 = sampled_errors(xh64, g)
    e32 = sampled_errors(xh32, g)
    say(f"  vs oracle x: fp64 max {e64[0]:.2e} 2-norm {e64[1]:.2e}; fp32 max {e32[0]:.2e} 2-norm {e32[1]:.2e}; "
        f"oracle iterations {g['iterations']}")
    om, lmin, lmax = damping64
    assert abs(om - g["omega"]) < 1e-9 * g["omega"] and abs(lmax - g["lambda_max"]) < 1e-9 * g["lambda_max"]
    assert info64["iterations"] == g["iterations"]
    assert info32["iterations"] <= g["iterations"] + 2
    assert max(e64) <= 1e-10
    assert max(e32) <= 1e-6
    # condition estimate of the solve (CG-Lanczos on its own coefficients, Table
    # tab:poisson-cond): the FP64 run takes the oracle's steps (1e-8).  The FP32 relaxation's
    # preconditioner differs from the oracle's by ~1e-7 per apply; the extreme Ritz values of
    # a 12- to 20-step run are not converged eigenvalues and move more than the coefficients
    # do (1.1e-4 relative observed for ritz_min at 16^3 Q7), hence 1e-3
    if "ritz_min" in g:
        say(f"  kappa fp64 {info64['kappa_estimate']:.6f} fp32 {info32['kappa_estimate']:.6f} "
            f"oracle {g['ritz_max'] / g['ritz_min']:.6f}")
        for key in ("ritz_min", "ritz_max"):
            assert abs(info64[key] - g[key]) <= 1e-8 * g[key]
            assert abs(info32[key] - g[key]) <= 1e-3 * g[key]
