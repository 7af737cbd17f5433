"""Pins for the elasticity oracle (Sec. 3.1): closed-form strain energy of linear fields,
rigid rotations in the kernel of the element operators, the diagonal blocks against the
scalar operator with the tensor coefficient K_j, the Q1 coarse matrix against the operator
itself, the SDC scalings' closed form on boxes, the single-patch SDC relaxation against the
exact block-diagonal solve, PCG against a direct solve, and the growth of the preconditioned
condition number with lambda that eq. SDC predicts."""
import numpy as np
import pytest

from oracle import mesh as omesh
from oracle import transfer
from oracle.elasticity import Elasticity, SDCSolver
from oracle.fdm1d import setup_1d
from oracle.operator import Discretization
from paper_2107_14758_amd import inputs

MU, LAM = 1.3, 2.9


def lattice_coords(d):
    """Physical coordinates of every lattice node (Fz, Fy, Fx, 3): the trilinear map of each
    cell evaluated at its GLL nodes (shared nodes agree: the map is continuous)."""
    X = omesh.cell_corners(d.vertices)
    N, _ = omesh.hat_1d(d.ref["nodes"])                       # (p+1, 2)
    xc = np.einsum("kc,jb,ia,ncbad->nkjid", N, N, N, X)
    K, J, I = d.cell_index()
    out = np.zeros(d.full_shape + (3,))
    out[K, J, I] = xc
    return out


def mesh(n, p, jitter, seed=3):
    rng = np.random.default_rng(seed)
    V = inputs.cube_vertices(*n)
    if jitter:
        V = inputs.jitter_vertices(V, jitter, rng)
    return Discretization(V, p), rng


@pytest.mark.parametrize("p,jit", [(2, 0.0), (3, 0.2)])
def test_linear_field_energy_and_rigid_rotations(p, jit):
    d, _ = mesh((2, 2, 3), p, jit)
    el = Elasticity(d, MU, LAM)
    x = lattice_coords(d)
    vol = np.sum(el.wdet)                                     # the mesh volume (exact rule)
    assert abs(vol - 1.0) < 1e-12
    G = np.array([[0.3, -1.1, 0.4], [0.7, 0.2, -0.5], [1.3, 0.6, -0.9]])
    u = np.moveaxis(x @ G.T, -1, 0)                           # u = G x, (3, Fz, Fy, Fx)
    E = np.sum(u * el.apply_full(u))
    sym = 0.5 * (G + G.T)
    exact = vol * (2 * MU * np.sum(sym * sym) + LAM * np.trace(G) ** 2)
    assert abs(E - exact) < 1e-11 * exact
    # a rigid rotation (skew G) has no strain: every element operator annihilates it
    W = np.array([[0.0, 0.8, -0.3], [-0.8, 0.0, 1.1], [0.3, -1.1, 0.0]])
    r = np.moveaxis(x @ W.T + np.array([0.2, -0.4, 0.9]), -1, 0)
    assert np.abs(el.apply_full(r)).max() < 1e-12 * np.abs(el.apply_full(u)).max()


def test_operator_symmetric_positive_definite():
    d, rng = mesh((2, 2, 2), 2, 0.15)
    el = Elasticity(d, MU, LAM)
    A = np.stack([el.apply(e) for e in np.eye(el.n)], axis=1)
    assert np.abs(A - A.T).max() < 1e-12 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0


def test_diagonal_blocks_are_the_scalar_operator_with_coefficient_K_j():
    # A_jj = int grad v . K_j grad u, K_j = mu I + (mu + lam) e_j e_j^T (any cell shape)
    d, rng = mesh((2, 3, 2), 3, 0.2)
    el = Elasticity(d, MU, LAM)
    w = rng.standard_normal(d.n)
    J = omesh.jacobians(d.vertices, d.ref["xq"])
    Ji = np.linalg.inv(J)
    det = np.abs(np.linalg.det(J))
    for j in range(3):
        u = np.zeros(el.n)
        u[j * d.n:(j + 1) * d.n] = w
        y = el.apply(u)[j * d.n:(j + 1) * d.n]
        K = MU * np.eye(3)
        K[j, j] += MU + LAM
        Gw = (det[..., None, None] * (Ji @ K @ np.swapaxes(Ji, -1, -2))) * d.w3[None, ..., None, None]
        ref = d.apply(w, G=Gw)
        assert np.abs(y - ref).max() < 1e-12 * np.abs(ref).max()


def test_coarse_matrix_is_the_galerkin_product():
    d, _ = mesh((2, 2, 3), 3, 0.15)
    el = Elasticity(d, MU, LAM)
    A0 = el.coarse_matrix()
    nc = A0.shape[0] // 3
    cols = []
    for k in range(3 * nc):
        e = np.zeros(3 * nc)
        e[k] = 1.0
        Pe = np.concatenate([transfer.coarse_prolong(d, e[c * nc:(c + 1) * nc]) for c in range(3)])
        y = el.apply(Pe)
        cols.append(np.concatenate([transfer.coarse_restrict(d, yc) for yc in el.split(y)]))
    ref = np.stack(cols, axis=1)
    assert np.abs(A0 - ref).max() < 1e-12 * np.abs(ref).max()


def test_sdc_scalings_on_boxes():
    # axis-aligned cells: mu_a^(j) = (mu + (mu + lam) delta_aj) * prod_i (L_i / 2) / (L_a / 2)^2
    nx, ny, nz = 3, 2, 2
    d = Discretization(inputs.cube_vertices(nx, ny, nz), 3)
    el = Elasticity(d, MU, LAM)
    base = omesh.cartesian_mu([1.0 / nx, 1.0 / ny, 1.0 / nz])
    for j, m in enumerate(el.sdc_mu()):
        k = np.full(3, MU)
        k[j] += MU + LAM
        assert np.abs(m - k * base).max() < 1e-13 * np.abs(m).max()


def test_single_patch_sdc_is_the_exact_block_diagonal_solve():
    # 2^3 Cartesian cells, the centre star only: it holds every DOF, its FDM surrogate is
    # exact, so S r = diag(A_11, A_22, A_33)^{-1} r
    d = Discretization(inputs.cube_vertices(2, 2, 2), 3)
    el = Elasticity(d, MU, LAM)
    s = SDCSolver(el, setup_1d(3), omega=1.0, interior_only=True)
    A = np.stack([el.apply(e) for e in np.eye(el.n)], axis=1)
    r = np.random.default_rng(5).standard_normal(el.n)
    z = s.relax(r)
    n = d.n
    ref = np.concatenate([np.linalg.solve(A[j * n:(j + 1) * n, j * n:(j + 1) * n], r[j * n:(j + 1) * n]) for j in range(3)])
    assert np.abs(z - ref).max() < 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("lam", [0.0, 10.0])
def test_pcg_matches_direct_solve(lam):
    d = Discretization(inputs.cube_vertices(3, 2, 2), 3)
    el = Elasticity(d, 1.0, lam)
    rng = np.random.default_rng(8)
    f = rng.uniform(-1, 1, (3, d.ncell, d.q, d.q, d.q))
    b = el.load_vector(f)
    s = SDCSolver(el, setup_1d(3), seed=0)
    x, it, (lmin, lmax) = s.pcg(b)
    A = np.stack([el.apply(e) for e in np.eye(el.n)], axis=1)
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(b - A @ x) <= 1.0000001e-8 * np.linalg.norm(b)
    assert np.linalg.norm(x - xd) <= 1e-6 * np.linalg.norm(xd)
    assert 0 < lmin < lmax and it < 40
    # the preconditioned operator's spectrum contains the Ritz values
    M = np.stack([s.precondition(e) for e in np.eye(el.n)], axis=1)
    ev = np.sort(np.linalg.eigvals(M @ A).real)
    assert ev[0] - 1e-9 <= lmin and lmax <= ev[-1] + 1e-9


def test_sdc_conditioning_degrades_with_lambda():
    # eq. SDC: the SDC-preconditioned condition number grows like (1 - nu) / (1 - 2 nu), i.e.
    # without bound as lambda / mu grows (nearly incompressible); the two-level method inherits
    # it.  Dense spectrum of M A on a small mesh for lambda = 0, 10, 100.
    d = Discretization(inputs.cube_vertices(3, 2, 2), 2)
    kappas = []
    for lam in (0.0, 10.0, 100.0):
        el = Elasticity(d, 1.0, lam)
        s = SDCSolver(el, setup_1d(2), seed=0)
        A = np.stack([el.apply(e) for e in np.eye(el.n)], axis=1)
        M = np.stack([s.precondition(e) for e in np.eye(el.n)], axis=1)
        ev = np.sort(np.linalg.eigvals(M @ A).real)
        assert ev[0] > 0
        kappas.append(ev[-1] / ev[0])
    assert kappas[0] < kappas[1] < kappas[2] and kappas[2] > 3 * kappas[0]
