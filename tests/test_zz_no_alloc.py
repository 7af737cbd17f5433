"""GPU test of the allocation-free operator entry point (vsr_apply_operator_noalloc).

It must give the same y as vsr_apply_operator (same kernels, same summation order: bit for
bit) and match the FP64 oracle's operator to 1e-12, on two calls in a row through the C ABI,
the second on a smaller problem (the static workspace keeps the first call's contents).
"""
import numpy as np
import pytest

from oracle.operator import Discretization
from paper_2107_14758_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# (cells, p, jitter, log-normal kappa): the first is the general operator at p = 15 (two
# element-vector slots per cell in FP64), the second a smaller Cartesian (Kronecker) problem.
CALLS = [((3, 3, 2), 15, 0.15, True), ((3, 2, 2), 5, 0.0, False)]


def say(*a):
    print(*a, flush=True)


def test_noalloc_operator_matches_allocating_entry_point():
    from paper_2107_14758_amd import vsr
    vsr.lib()
    sizes = []
    for call, (shape, p, jit, logn) in enumerate(CALLS):
        say(f"call {call}: cells {shape} p={p} jitter={jit} lognormal={logn}")
        nx, ny, nz = shape
        rng = np.random.default_rng(10 + call)
        V = inputs.cube_vertices(nx, ny, nz)
        if jit:
            V = inputs.jitter_vertices(V, jit, rng)
        kappa = inputs.lognormal_kappa(nx, ny, nz, rng) if logn else None
        prob = vsr.Problem(V, p, kappa=kappa, seed=0)
        n = prob.n
        sizes.append(n)
        x = rng.uniform(-1.0, 1.0, n)
        xd = torch.tensor(x, dtype=torch.float64, device="cuda")
        y_ref = torch.zeros(n, dtype=torch.float64, device="cuda")
        y_na = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        prob.apply_operator(xd, y_ref)
        prob.apply_operator_noalloc(xd, y_na)
        torch.cuda.synchronize()
        a, b = y_na.cpu().numpy(), y_ref.cpu().numpy()
        assert np.array_equal(a, b), f"call {call}: max |diff| {np.abs(a - b).max()}"
        yo = Discretization(V, p, kappa).apply(x)
        err = np.abs(a - yo).max() / np.abs(yo).max()
        say(f"  n={n}: noalloc == allocating bit for bit; max-abs error vs oracle {err:.2e}")
        assert err <= 1e-12
        assert np.linalg.norm(a - yo) <= 1e-12 * np.linalg.norm(yo)
        prob.close()
    assert sizes[1] < sizes[0]
