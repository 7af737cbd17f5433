"""Pins for the oracle's geometric multigrid on the Q1 coarse problem (Sec. 2.8):
Galerkin identities, the nested-space identity on Cartesian hierarchies, the
single-level case (the direct solve), symmetry and definiteness of the V-cycle,
and an h-independent convergence factor."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import gmg, transfer
from oracle.fdm1d import setup_1d
from oracle.operator import Discretization
from oracle.solver import Solver
from paper_2107_14758_amd import inputs


def disc(n, p=2, jitter=0.0, kappa=False, seed=4, shape=None):
    if shape is None:
        w = inputs.make_problem(n, p, seed=seed, jitter=jitter, lognormal=kappa)
        return Discretization(w["vertices"], p, w["kappa"])
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    V = inputs.cube_vertices(nx, ny, nz)
    if jitter:
        V = inputs.jitter_vertices(V, jitter, rng)
    k = inputs.lognormal_kappa(nx, ny, nz, rng) if kappa else None
    return Discretization(V, p, k)


def test_q1_matrix_is_the_galerkin_coarse_matrix():
    # the sparse Q1 matrix equals P^T A P with P the Q1 -> Q_p interpolation and A the Q_p operator
    d = disc(0, p=3, jitter=0.15, kappa=True, shape=(3, 2, 4))
    A = d.assemble().toarray()
    nc = 2 * 1 * 3
    P = np.stack([transfer.coarse_prolong(d, e) for e in np.eye(nc)], axis=1)
    np.testing.assert_allclose(gmg.q1_matrix(d).toarray(), P.T @ A @ P, atol=1e-12 * np.abs(A).max())


def test_interpolation_reproduces_linear_functions():
    # 1D factor of the trilinear interpolation: every column is the coarse hat function, and
    # piecewise-linear coarse data (zero on the Dirichlet ends) is reproduced exactly
    P1 = gmg.interpolation_1d(8)
    assert P1.shape == (7, 3)
    # column I is the coarse hat at fine index 2I: values 1/2, 1, 1/2 at 2I-1, 2I, 2I+1
    for I in range(1, 4):
        col = np.zeros(7)
        col[2 * I - 2], col[2 * I - 1], col[2 * I] = 0.5, 1.0, 0.5
        np.testing.assert_array_equal(P1[:, I - 1], col)
    # a piecewise-linear function on the coarse grid is reproduced exactly on the fine grid
    xc = np.array([0.3, -1.2, 2.0])                       # interior coarse values, 0 on the boundary
    full_c = np.concatenate([[0.0], xc, [0.0]])
    fine = np.interp(np.arange(1, 8) / 2.0, np.arange(5), full_c)
    np.testing.assert_allclose(P1 @ xc, fine, atol=1e-15)


@pytest.mark.parametrize("n", [4, 8])
def test_galerkin_equals_rediscretization_on_cartesian_hierarchy(n):
    # nested Q1 spaces, exact quadrature: P^T A_h P = A_2h on a uniform Cartesian mesh
    mg = gmg.Q1Multigrid.for_discretization(disc(n))
    assert mg.levels == int(np.log2(n))
    for l in range(1, mg.levels):
        coarse = gmg.q1_matrix(disc(n >> l))
        np.testing.assert_allclose(mg.A[l].toarray(), coarse.toarray(), atol=1e-13 * abs(coarse).max())


@pytest.mark.parametrize("shape", [(3, 3, 3), (2, 2, 2), (4, 3, 4), (6, 6, 5)])
def test_single_level_is_the_direct_solve(shape):
    d = disc(0, jitter=0.15, kappa=True, shape=shape)
    mg = gmg.Q1Multigrid.for_discretization(d)
    assert mg.levels == 1
    A = gmg.q1_matrix(d).toarray()
    b = np.random.default_rng(1).standard_normal(A.shape[0])
    np.testing.assert_allclose(mg.vcycle(b), np.linalg.solve(A, b), rtol=0, atol=1e-13 * np.abs(np.linalg.solve(A, b)).max())


@pytest.mark.parametrize("shape,jit", [((8, 4, 4), 0.15), ((8, 8, 8), 0.0)])
def test_vcycle_is_symmetric_positive_definite(shape, jit):
    d = disc(0, jitter=jit, kappa=jit > 0, shape=shape)
    mg = gmg.Q1Multigrid.for_discretization(d)
    assert mg.levels >= 2
    n = mg.A[0].shape[0]
    B = np.stack([mg.vcycle(e) for e in np.eye(n)], axis=1)
    assert np.abs(B - B.T).max() <= 1e-13 * np.abs(B).max()
    ev = np.linalg.eigvalsh(0.5 * (B + B.T))
    assert ev.min() > 0
    # B A has its spectrum in (0, 1]: the cycle is a convergent stationary iteration
    lam = sla.eigvals(B @ mg.A[0].toarray()).real
    assert lam.min() > 0 and lam.max() <= 1 + 1e-12


def test_jacobi_weight_is_inside_the_stability_bound():
    # 2/3 lambda_max(D^-1 A) < 2 on every level (Gershgorin bound of the Q1 stencil)
    mg = gmg.Q1Multigrid.for_discretization(disc(8, jitter=0.2, kappa=True))
    for A, dinv in zip(mg.A, mg.dinv):
        gersh = (np.abs(A).sum(axis=1).A1 * dinv).max()
        assert mg.omega * gersh < 2


def convergence_factor(mg, iters=25):
    A = mg.A[0]
    e = np.random.default_rng(0).standard_normal(A.shape[0])
    rho = 0.0
    for _ in range(iters):
        e_new = e - mg.vcycle(A @ e)
        rho = np.linalg.norm(e_new) / np.linalg.norm(e)
        e = e_new / np.linalg.norm(e_new)
    return rho


def test_convergence_factor_is_independent_of_h():
    # two-grid (4 cells per axis) down to four levels (16): the factor settles near 0.4
    rhos = [convergence_factor(gmg.Q1Multigrid.for_discretization(disc(n))) for n in (4, 8, 16)]
    assert max(rhos) < 0.5
    assert abs(rhos[2] - rhos[1]) < 0.05


def test_pcg_with_gmg_coarse_solve_converges_like_the_direct_one():
    w = inputs.make_problem(4, 3, seed=0, jitter=0.15, lognormal=True)
    d = Discretization(w["vertices"], 3, w["kappa"])
    b = d.load_vector(w["f"])
    xd, itd = Solver(d, setup_1d(3), seed=0).pcg(b)
    s = Solver(d, setup_1d(3), seed=0, coarse="gmg")
    assert s.mg.levels == 2
    xg, itg = s.pcg(b)
    assert abs(itg - itd) <= 1
    x = sla.solve(d.assemble().toarray(), b, assume_a="pos")
    assert np.linalg.norm(xg - x) <= 1e-7 * np.linalg.norm(x)
