"""Seeded synthetic workloads: meshes, coefficients and right-hand sides.

This module draws inputs only; it contains none of the solver's arithmetic.
All draws use numpy's PCG64 generator, one generator per workload, in the
fixed order: vertex jitter, coefficient field, right-hand side samples.

* Unit-cube mesh of nx x ny x nz hexahedra, vertices (nz+1, ny+1, nx+1, 3),
  x fastest.  Optional jitter moves every interior vertex by an independent
  uniform offset in [-a h, a h] per coordinate (h = cell width on that axis).
* Log-normal coefficient kappa = exp(g) per cell, with g a Gaussian random
  field sampled at the cell centroids (of the unjittered mesh), squared
  exponential covariance var * exp(-r^2 / (2 ell^2)), drawn as
  chol(C + 1e-10 I) z with z standard normal.
* Right-hand side samples f i.i.d. uniform on [-1, 1] at each cell's
  quadrature points (ncell, npts), with npts given by the caller.
"""
import numpy as np


def cube_vertices(nx, ny=None, nz=None):
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    z, y, x = np.meshgrid(np.linspace(0, 1, nz + 1), np.linspace(0, 1, ny + 1),
                          np.linspace(0, 1, nx + 1), indexing="ij")
    return np.stack([x, y, z], axis=-1)


def jitter_vertices(vertices, amplitude, rng):
    V = np.array(vertices, dtype=np.float64, copy=True)
    nz, ny, nx = V.shape[0] - 1, V.shape[1] - 1, V.shape[2] - 1
    h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
    shape = (max(nz - 1, 0), max(ny - 1, 0), max(nx - 1, 0), 3)
    d = rng.uniform(-1.0, 1.0, size=shape) * amplitude * h
    V[1:-1, 1:-1, 1:-1, :] += d
    return V


def lognormal_kappa(nx, ny, nz, rng, ell=0.25, var=1.0):
    cz, cy, cx = np.meshgrid((np.arange(nz) + 0.5) / nz, (np.arange(ny) + 0.5) / ny,
                             (np.arange(nx) + 0.5) / nx, indexing="ij")
    c = np.stack([cx.reshape(-1), cy.reshape(-1), cz.reshape(-1)], axis=-1)
    d2 = ((c[:, None, :] - c[None, :, :]) ** 2).sum(-1)
    C = var * np.exp(-d2 / (2.0 * ell * ell)) + 1e-10 * np.eye(len(c))
    g = np.linalg.cholesky(C) @ rng.standard_normal(len(c))
    return np.exp(g)


def rhs_samples(ncell, npts, rng):
    return rng.uniform(-1.0, 1.0, size=(ncell, npts))


def quadrature_points_per_dir(p):
    """Points per direction at which the right-hand side is sampled, ceil(3(p+1)/2)."""
    return (3 * (p + 1) + 1) // 2


def make_problem(n, p, seed=0, jitter=0.0, lognormal=False, ell=0.25, var=1.0):
    """Return dict(vertices, kappa or None, f (ncell, q^3), p, q, n, seed) for an n^3 mesh."""
    nx = ny = nz = n
    rng = np.random.default_rng(seed)
    V = cube_vertices(nx, ny, nz)
    if jitter:
        V = jitter_vertices(V, jitter, rng)
    kappa = lognormal_kappa(nx, ny, nz, rng, ell, var) if lognormal else None
    q = quadrature_points_per_dir(p)
    f = rhs_samples(nx * ny * nz, q ** 3, rng)
    return dict(vertices=V, kappa=kappa, f=f, p=p, q=q, n=n, seed=seed, jitter=jitter)


# The workloads: (cells per axis, degree, jitter, log-normal coefficient).
WORKLOADS = {
    "poisson_cart_2x2x2_q3": dict(n=2, p=3, jitter=0.0, lognormal=False),
    "poisson_cart_16x16x16_q7": dict(n=16, p=7, jitter=0.0, lognormal=False),
    "poisson_jitter_8x8x8_q15_lognormal": dict(n=8, p=15, jitter=0.15, lognormal=True),
    "poisson_jitter_12x12x12_q11_lognormal": dict(n=12, p=11, jitter=0.2, lognormal=True),
    # h-scaling of the 16^3 Q7 workload: eight times the cells, beyond the dense coarse inverse
    "poisson_cart_32x32x32_q7": dict(n=32, p=7, jitter=0.0, lognormal=False),
}


BATCH_CELLS = (4, 6, 8, 12)
BATCH_DEGREES = (4, 7, 11, 15)


def batch_workload(count=64, seed=0, jitter=0.15):
    """Independent problems of uneven size for a batched solve: cells per axis drawn from
    {4, 6, 8, 12}, degree from {4, 7, 11, 15}, half the meshes (a seeded coin per member)
    with interior vertices jittered by U[-jitter h, jitter h], kappa = 1, RHS U[-1, 1] at the
    quadrature points.  Returns a list of make_problem dicts."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(BATCH_CELLS, count)
    ps = rng.choice(BATCH_DEGREES, count)
    jit = rng.random(count) < 0.5
    seeds = rng.integers(0, 2 ** 31, count)
    return [make_problem(int(n), int(p), seed=int(sd), jitter=jitter if j else 0.0)
            for n, p, j, sd in zip(ns, ps, jit, seeds)]


def workload(name, seed=0):
    w = WORKLOADS[name]
    return make_problem(w["n"], w["p"], seed=seed, jitter=w["jitter"], lognormal=w["lognormal"])


def random_cells(n, amplitude, rng, h=1.0):
    """n independent trilinear cells: the cube [0,h]^3 with each of its 8 corners moved by an
    independent U[-amplitude h, amplitude h] offset per coordinate; (n, 2, 2, 2, 3) [cell, c, b, a, coord]."""
    base = np.array([[[[a, b, c] for a in range(2)] for b in range(2)] for c in range(2)], dtype=np.float64) * h
    return base[None] + rng.uniform(-1.0, 1.0, size=(n, 2, 2, 2, 3)) * amplitude * h


def mlp_init(rng, nin=74, nh=64, nout=3):
    """Initial MLP parameters (float32, packed W1, b1, W2, b2, W3, b3): uniform(+-1/sqrt(fan_in)), zero biases."""
    parts = []
    for fan_in, fan_out in ((nin, nh), (nh, nh), (nh, nout)):
        lim = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)
