"""The library on a caller's stream (options.stream): a solve issued on a non-default torch
stream gives bit for bit the solve on the default stream (deterministic mode), for the scalar
problem (graph-replayed iterations over the library's streams) and for elasticity (its
iterations on the library's stream, forked from and joined back to the caller's)."""
import numpy as np
import pytest

from paper_2107_14758_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vsr():
    from paper_2107_14758_amd import vsr as v
    v.lib()
    return v


def test_scalar_solve_on_a_caller_stream(vsr):
    w = inputs.make_problem(3, 4, seed=2, jitter=0.15, lognormal=True)
    f = torch.tensor(w["f"], dtype=torch.float64, device="cuda")
    ref = vsr.Problem(w["vertices"], 4, kappa=w["kappa"], seed=0, relax_fp32=True, deterministic=True)
    b = torch.zeros(ref.n, dtype=torch.float64, device="cuda")
    ref.load_vector(f, b)
    x0 = torch.zeros_like(b)
    i0 = ref.pcg_solve(b, x0)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        prob = vsr.Problem(w["vertices"], 4, kappa=w["kappa"], seed=0, relax_fp32=True, deterministic=True,
                           stream=s.cuda_stream)
        b1 = torch.zeros_like(b)
        prob.load_vector(f, b1)
        x1 = torch.zeros_like(b)
        i1 = prob.pcg_solve(b1, x1)
    s.synchronize()
    assert torch.equal(b1, b) and i1["iterations"] == i0["iterations"] and torch.equal(x1, x0)
    prob.close()
    ref.close()


def test_elasticity_solve_on_a_caller_stream(vsr):
    V = inputs.cube_vertices(3, 2, 2)
    rng = np.random.default_rng(3)
    q = inputs.quadrature_points_per_dir(3)
    f = torch.tensor(rng.uniform(-1, 1, (3, 12, q, q, q)), dtype=torch.float64, device="cuda")
    ref = vsr.Elasticity(V, 3, 1.0, 2.0, relax_fp32=True, deterministic=True)
    b = torch.zeros(ref.n, dtype=torch.float64, device="cuda")
    ref.load_vector(f, b)
    x0 = torch.zeros_like(b)
    i0 = ref.pcg_solve(b, x0)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = vsr.Elasticity(V, 3, 1.0, 2.0, relax_fp32=True, deterministic=True, stream=s.cuda_stream)
        b1 = torch.zeros_like(b)
        g.load_vector(f, b1)
        x1 = torch.zeros_like(b)
        i1 = g.pcg_solve(b1, x1)
        y = torch.zeros_like(b)
        g.apply_operator(x1, y)
    s.synchronize()
    assert torch.equal(b1, b) and i1["iterations"] == i0["iterations"] and torch.equal(x1, x0)
    assert float((y - b).norm() / b.norm()) <= 2e-8
    g.close()
    ref.close()
