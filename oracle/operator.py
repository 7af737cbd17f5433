"""Galerkin stiffness operator and load vector for Q_p on hexahedra (Sec. 2.1, 2.7).

Test infrastructure only (see ``oracle/__init__``).

Discrete space: continuous Q_p with the GLL Lagrange basis on every cell,
homogeneous Dirichlet conditions on the whole boundary.  The global nodes form
the lattice (p nz + 1) x (p ny + 1) x (p nx + 1); the free DOFs are its
interior points in lexicographic order with x fastest.

A = sum_K R_K^T A^K R_K (direct stiffness summation, Sec. 2.1), where
A^K_ab = sum_q w_q grad_hat phi_a(x_q) . G_hat(x_q) grad_hat phi_b(x_q)
with the q^3-point tensor GLL rule (Sec. 2.8) and G_hat from ``mesh``.

Two evaluations are provided: ``assemble`` builds A^K as dense element
matrices and sums them into a sparse matrix (definition mode, tiny sizes), and
``apply`` evaluates the same sums by one-dimensional contractions per
direction (sum factorization, the matrix-free form of Sec. 1 and 2.7).
"""
import numpy as np
import scipy.sparse as sp

from . import mesh as _mesh
from .fdm1d import reference_matrices


class Discretization:
    """Everything the operator needs for one mesh and degree (float64)."""

    def __init__(self, vertices, p, kappa=None, q=None):
        V = np.asarray(vertices, dtype=np.float64)
        self.vertices = V
        self.nz, self.ny, self.nx = V.shape[0] - 1, V.shape[1] - 1, V.shape[2] - 1
        self.p = p
        self.ref = reference_matrices(p, q)
        self.q = self.ref["q"]
        self.ncell = self.nx * self.ny * self.nz
        self.kappa = None if kappa is None else np.asarray(kappa, dtype=np.float64).reshape(-1)
        J = _mesh.jacobians(V, self.ref["xq"])
        self.G, self.detJ = _mesh.inverse_metric(J, self.kappa)
        wq = self.ref["wq"]
        self.w3 = np.einsum("c,b,a->cba", wq, wq, wq)
        self.Gw = self.G * self.w3[None, :, :, :, None, None]
        self.mu = _mesh.surrogate_mu(self.G, wq)
        self.full_shape = (p * self.nz + 1, p * self.ny + 1, p * self.nx + 1)
        self.free_shape = tuple(s - 2 for s in self.full_shape)
        self.n = int(np.prod(self.free_shape))

    # ---- lattice <-> cell views -------------------------------------------------
    def to_full(self, x):
        full = np.zeros(self.full_shape)
        full[1:-1, 1:-1, 1:-1] = np.asarray(x).reshape(self.free_shape)
        return full

    def from_full(self, full):
        return full[1:-1, 1:-1, 1:-1].reshape(-1).copy()

    def cell_index(self):
        """Fancy-index triple selecting (ncell, p+1, p+1, p+1) cell views of the lattice."""
        p = self.p
        ez, ey, ex = np.meshgrid(np.arange(self.nz), np.arange(self.ny), np.arange(self.nx), indexing="ij")
        ez, ey, ex = ez.reshape(-1), ey.reshape(-1), ex.reshape(-1)
        k = np.arange(p + 1)
        K = p * ez[:, None, None, None] + k[None, :, None, None]
        J = p * ey[:, None, None, None] + k[None, None, :, None]
        I = p * ex[:, None, None, None] + k[None, None, None, :]
        K, J, I = np.broadcast_arrays(K, J, I)
        return K, J, I

    def gather(self, x):
        K, J, I = self.cell_index()
        return self.to_full(x)[K, J, I]

    def scatter_add(self, ycells):
        K, J, I = self.cell_index()
        full = np.zeros(self.full_shape)
        np.add.at(full, (K, J, I), ycells)
        return self.from_full(full)

    # ---- matrix-free operator (sum factorization) ------------------------------
    def apply(self, x, G=None):
        """y = A x over the free DOFs; G (weighted metric per point) defaults to the true one."""
        Gw = self.Gw if G is None else G
        Iq, Dq = self.ref["Iq"], self.ref["Dq"]
        xc = self.gather(x)                                # [n, k, j, i]
        # gradient in reference coordinates at the q^3 points
        u1 = np.einsum("ck,bj,ai,nkji->ncba", Iq, Iq, Dq, xc, optimize=True)
        u2 = np.einsum("ck,bj,ai,nkji->ncba", Iq, Dq, Iq, xc, optimize=True)
        u3 = np.einsum("ck,bj,ai,nkji->ncba", Dq, Iq, Iq, xc, optimize=True)
        u = np.stack([u1, u2, u3], axis=-1)
        v = np.einsum("ncbaij,ncbaj->ncbai", Gw, u)
        yc = (np.einsum("ck,bj,ai,ncba->nkji", Iq, Iq, Dq, v[..., 0], optimize=True)
              + np.einsum("ck,bj,ai,ncba->nkji", Iq, Dq, Iq, v[..., 1], optimize=True)
              + np.einsum("ck,bj,ai,ncba->nkji", Dq, Iq, Iq, v[..., 2], optimize=True))
        return self.scatter_add(yc)

    # ---- definition mode --------------------------------------------------------
    def reference_gradients(self):
        """grad_hat phi_a at every point: (q^3, (p+1)^3, 3), a = i + (p+1)(j + (p+1)k)."""
        Iq, Dq = self.ref["Iq"], self.ref["Dq"]
        g1 = np.einsum("ck,bj,ai->cbakji", Iq, Iq, Dq)
        g2 = np.einsum("ck,bj,ai->cbakji", Iq, Dq, Iq)
        g3 = np.einsum("ck,bj,ai->cbakji", Dq, Iq, Iq)
        nq, nb = self.q ** 3, (self.p + 1) ** 3
        return np.stack([g1.reshape(nq, nb), g2.reshape(nq, nb), g3.reshape(nq, nb)], axis=-1)

    def element_matrices(self, Gw=None):
        Gw = self.Gw if Gw is None else Gw
        grad = self.reference_gradients()                     # (q^3, nb, 3)
        Gq = Gw.reshape(self.ncell, -1, 3, 3)
        gT = np.transpose(grad, (0, 2, 1)).reshape(-1, grad.shape[1])     # (3 q^3, nb), rows (q, i)
        out = np.empty((self.ncell, grad.shape[1], grad.shape[1]))
        for e in range(self.ncell):
            H = np.einsum("qij,qbj->qib", Gq[e], grad).reshape(-1, grad.shape[1])
            out[e] = gT.T @ H                                  # sum_{q,i} g[q,a,i] (G g)[q,i,b]
        return out

    def assemble(self, element=None):
        """Sparse A over the free DOFs from dense element matrices (tiny sizes)."""
        Ae = self.element_matrices() if element is None else element
        K, J, I = self.cell_index()
        Fz, Fy, Fx = self.full_shape
        gid = (K * Fy + J) * Fx + I                           # full-lattice id per cell node
        gid = gid.reshape(self.ncell, -1)
        rows = np.repeat(gid, gid.shape[1], axis=1).reshape(-1)
        cols = np.tile(gid, (1, gid.shape[1])).reshape(-1)
        Afull = sp.coo_matrix((Ae.reshape(-1), (rows, cols)), shape=(Fz * Fy * Fx,) * 2).tocsr()
        free = np.zeros(self.full_shape, dtype=bool)
        free[1:-1, 1:-1, 1:-1] = True
        fid = np.flatnonzero(free.reshape(-1))
        return Afull[fid][:, fid].tocsr()

    # ---- load vector -----------------------------------------------------------
    def load_vector(self, f):
        """b_a = sum_K sum_q w_q |det J| phi_a(x_q) f_{K,q}; f has shape (ncell, q, q, q)."""
        Iq = self.ref["Iq"]
        fq = np.asarray(f, dtype=np.float64).reshape(self.ncell, self.q, self.q, self.q)
        g = fq * self.w3[None] * np.abs(self.detJ)
        bc = np.einsum("ck,bj,ai,ncba->nkji", Iq, Iq, Iq, g, optimize=True)
        return self.scatter_add(bc)


def kron3(M3, M2, M1):
    """M3 (z) x M2 (y) x M1 (x), x fastest, as in the Kronecker form of Sec. 2.2."""
    return np.kron(M3, np.kron(M2, M1))


def separable_cell_matrix(mu, A1, B1):
    """mu_1 B x B x A + mu_2 B x A x B + mu_3 A x B x B (Sec. 2.2)."""
    return mu[0] * kron3(B1, B1, A1) + mu[1] * kron3(B1, A1, B1) + mu[2] * kron3(A1, B1, B1)
