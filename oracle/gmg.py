"""Geometric multigrid for the p-coarse (Q1) problem (Sec. 2.8, Fig. solver_pcg).

Test infrastructure only (see ``oracle/__init__``).

The paper solves the low-order coarse problem of its hybrid p-multigrid/Schwarz
cycle (the Q1 space on the same mesh, one unknown per interior vertex) by
geometric multigrid over a hierarchy of uniformly refined meshes, with damped
point-Jacobi relaxation on every level and a Cholesky factorization on the
coarsest one.

Readings (the paper gives the structure, not these details):

* Hierarchy.  The given mesh is the finest level.  A level with nx x ny x nz
  cells is coarsened by merging 2 x 2 x 2 cells while every axis has an even
  number of at least 4 cells; the last level reached is the coarsest.  A mesh
  that cannot be coarsened is a single level, solved directly.
* Transfers.  P_l interpolates coarse vertex values to the fine vertices
  trilinearly in index space (fine vertex 2I takes coarse vertex I, fine
  vertex 2I +- 1 takes half of I and half of its neighbour), with zero
  Dirichlet values on the boundary; restriction is P_l^T.  On a uniform
  Cartesian hierarchy this is exactly the interpolation of nested Q1 spaces.
* Coarse operators.  Galerkin, A_{l-1} = P_l^T A_l P_l, starting from the Q1
  matrix of the fine mesh (the same A_0 = P^T A P as the direct coarse solve;
  on a uniform Cartesian hierarchy the Galerkin products equal the Q1
  rediscretizations).
* Cycle.  One V(1,1) cycle from a zero initial guess: one damped point-Jacobi
  step before and one after the coarse-grid correction, weight 2/3, and the
  coarsest level solved exactly by dense Cholesky.  With Jacobi before and
  after, the cycle is a symmetric positive definite operator, so the whole
  preconditioner stays symmetric.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .mesh import hat_1d

JACOBI_WEIGHT = 2.0 / 3.0


def q1_matrix(disc):
    """Sparse Q1 stiffness matrix over the interior vertices, from the Q1 element
    matrices integrated with the operator's quadrature (the A_0 of the coarse space)."""
    xq = disc.ref["xq"]
    N, dN = hat_1d(xq)
    g1 = np.einsum("zc,yb,xa->zyxcba", N, N, dN).reshape(disc.q ** 3, 8)
    g2 = np.einsum("zc,yb,xa->zyxcba", N, dN, N).reshape(disc.q ** 3, 8)
    g3 = np.einsum("zc,yb,xa->zyxcba", dN, N, N).reshape(disc.q ** 3, 8)
    grad = np.stack([g1, g2, g3], axis=-1)                       # (q^3, 8, 3)
    Gq = disc.Gw.reshape(disc.ncell, -1, 3, 3)
    Ae = np.einsum("qai,nqij,qbj->nab", grad, Gq, grad, optimize=True)
    nvz, nvy, nvx = disc.nz + 1, disc.ny + 1, disc.nx + 1
    ez, ey, ex = np.meshgrid(np.arange(disc.nz), np.arange(disc.ny), np.arange(disc.nx), indexing="ij")
    vid = np.stack([((ez + c) * nvy + (ey + b)) * nvx + (ex + a)
                    for c in range(2) for b in range(2) for a in range(2)], axis=-1).reshape(disc.ncell, 8)
    rows = np.repeat(vid, 8, axis=1).reshape(-1)
    cols = np.tile(vid, (1, 8)).reshape(-1)
    nv = nvz * nvy * nvx
    Afull = sp.coo_matrix((Ae.reshape(-1), (rows, cols)), shape=(nv, nv)).tocsr()
    inner = np.zeros((nvz, nvy, nvx), dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    fid = np.flatnonzero(inner.reshape(-1))
    return Afull[fid][:, fid].tocsr()


def interpolation_1d(nf):
    """(nf - 1) x (nf/2 - 1) index-space linear interpolation between interior vertices of
    a line of nf cells and of its nf/2-cell coarsening."""
    nc = nf // 2
    P = np.zeros((nf - 1, nc - 1))
    for I in range(1, nc):
        P[2 * I - 1, I - 1] = 1.0
        P[2 * I - 2, I - 1] = 0.5
        P[2 * I, I - 1] = 0.5
    return P


def interpolation(cells):
    """Trilinear index-space interpolation for a level of cells = (nx, ny, nz) cells
    (x fastest, as every vector here): P = P_z x P_y x P_x."""
    nx, ny, nz = cells
    return sp.csr_matrix(np.kron(interpolation_1d(nz), np.kron(interpolation_1d(ny), interpolation_1d(nx))))


def coarsenable(cells):
    return all(n % 2 == 0 and n >= 4 for n in cells)


class Q1Multigrid:
    """Levels 0 (finest) .. L (coarsest) of the Q1 problem and its V(1,1) cycle."""

    def __init__(self, A, cells, omega=JACOBI_WEIGHT):
        self.omega = omega
        self.A = [sp.csr_matrix(A)]
        self.cells = [tuple(cells)]
        self.P = []
        while coarsenable(self.cells[-1]):
            P = interpolation(self.cells[-1])
            self.P.append(P)
            self.A.append(sp.csr_matrix(P.T @ self.A[-1] @ P))
            self.cells.append(tuple(n // 2 for n in self.cells[-1]))
        self.dinv = [1.0 / A_l.diagonal() for A_l in self.A]
        Ac = self.A[-1].toarray()
        self.chol = sla.cho_factor(Ac, lower=True) if Ac.size else None

    @classmethod
    def for_discretization(cls, disc, omega=JACOBI_WEIGHT):
        return cls(q1_matrix(disc), (disc.nx, disc.ny, disc.nz), omega)

    @property
    def levels(self):
        return len(self.A)

    def vcycle(self, b, level=0):
        """One V(1,1) cycle for A_level x = b from x = 0."""
        b = np.asarray(b, dtype=np.float64)
        if level == self.levels - 1:
            return sla.cho_solve(self.chol, b) if self.chol is not None else np.zeros_like(b)
        A, dinv, P, w = self.A[level], self.dinv[level], self.P[level], self.omega
        x = w * dinv * b                                   # pre-smoothing from zero
        rc = P.T @ (b - A @ x)                              # restricted residual
        x = x + P @ self.vcycle(rc, level + 1)              # coarse-grid correction
        return x + w * dinv * (b - A @ x)                   # post-smoothing
