"""Vertex-star patches and their exact solves (Sec. 2.5, 2.6).

Test infrastructure only (see ``oracle/__init__``).

One patch per mesh vertex v (Sec. 2.5: the DOFs of v and of every cell, face
and edge around it).  On the structured hex mesh the star of v is the block
of the (up to) 2 x 2 x 2 cells around it; the patch DOFs are the free lattice
nodes strictly inside that block.  Along an axis where v is interior this is
2p-1 positions (two cells and the central plane); where v lies on the
boundary it is the p-1 interior positions of the single adjacent cell.  With
``interior_only=True`` only interior vertices get patches (the alternative
reading; every free DOF is still covered).

Patch matrices are those of the separable surrogate form (Sec. 2.7):
each cell contributes mu_1 B x B x A + mu_2 B x A x B + mu_3 A x B x B in the
chosen one-dimensional basis.  In the FDM basis (Sec. 2.4) the 1D blocks are
A_F = [[a00, a0I, a0p], [aI0, diag(lam), aIp], [ap0, apI, app]] and
B_F = [[b00, 0, b0p], [0, I, 0], [bp0, 0, bpp]] exactly; the FDM matrices are
built in that form (the computed T^T A T differs from it only by rounding).

``solve`` follows Sec. 2.6 (block LDL^T, interior DOFs first): the interior
block A_II (nodes on no central plane of the star) is diagonal, so the
interface Schur complement S = A_GG - A_GI A_II^{-1} A_IG is formed densely
and factored by dense Cholesky; u_G = S^{-1}(r_G - A_GI A_II^{-1} r_I),
u_I = A_II^{-1}(r_I - A_IG u_G).  ``solve_dense_gll`` is the definition: the
dense GLL-basis patch matrix of the surrogate, solved directly (small p only).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .operator import separable_cell_matrix


def exact_fdm_1d(od):
    """1D FDM matrices with their structural zeros imposed (see module doc)."""
    p = od["p"]
    AF = od["AF"].copy()
    BF = od["BF"].copy()
    I = slice(1, p)
    AF[I, I] = np.diag(od["lam"])
    BF[I, I] = np.eye(p - 1)
    BF[I, 0] = BF[I, p] = 0.0
    BF[0, I] = BF[p, I] = 0.0
    return AF, BF


class Patches:
    def __init__(self, disc, od, mu=None, interior_only=False):
        self.disc = disc
        self.od = od
        self.p = disc.p
        self.mu = (disc.mu if mu is None else np.asarray(mu, dtype=np.float64)).reshape(
            disc.nz, disc.ny, disc.nx, 3)
        self.AF, self.BF = exact_fdm_1d(od)
        lo = 1 if interior_only else 0
        self.vertices = [(vz, vy, vx) for vz in range(lo, disc.nz + 1 - lo)
                         for vy in range(lo, disc.ny + 1 - lo) for vx in range(lo, disc.nx + 1 - lo)]
        self._cache = {}

    def _axis(self, v, ncell):
        """Free lattice positions strictly inside the star along one axis, and the
        central-plane flag for each (only an interior vertex has a central plane)."""
        p = self.p
        lo, hi = max(p * (v - 1) + 1, 1), min(p * (v + 1) - 1, p * ncell - 1)
        pos = np.arange(lo, hi + 1)
        return pos, pos == p * v

    def layout(self, v):
        """(free-DOF indices, interface mask) of the patch of v, local order x fastest."""
        vz, vy, vx = v
        d = self.disc
        Lz, Ly, Lx = d.free_shape
        (pz, cz), (py, cy), (px, cx) = self._axis(vz, d.nz), self._axis(vy, d.ny), self._axis(vx, d.nx)
        idx = (((pz[:, None, None] - 1) * Ly + (py[None, :, None] - 1)) * Lx + (px[None, None, :] - 1))
        face = cz[:, None, None] | cy[None, :, None] | cx[None, None, :]
        return idx.reshape(-1), face.reshape(-1)

    def dofs(self, v):
        return self.layout(v)[0]

    def _assemble(self, v, A1, B1, sparse):
        """Patch matrix from the star's cells' separable matrices in the given 1D basis.

        Works in the star's local box of (2p+1)^3 lattice positions, whose
        origin is the global position p (v - 1) on every axis."""
        p, d = self.p, self.disc
        m = 2 * p + 1
        rows, cols, vals = [], [], []
        k = np.arange(p + 1)
        vz, vy, vx = v
        for ez in (vz - 1, vz):
            for ey in (vy - 1, vy):
                for ex in (vx - 1, vx):
                    if not (0 <= ez < d.nz and 0 <= ey < d.ny and 0 <= ex < d.nx):
                        continue
                    mu = self.mu[ez, ey, ex]
                    if sparse:
                        A1s, B1s = sp.csr_matrix(A1), sp.csr_matrix(B1)
                        Ak = (mu[0] * sp.kron(B1s, sp.kron(B1s, A1s)) + mu[1] * sp.kron(B1s, sp.kron(A1s, B1s))
                              + mu[2] * sp.kron(A1s, sp.kron(B1s, B1s))).tocoo()
                    else:
                        Ak = sp.coo_matrix(separable_cell_matrix(mu, A1, B1))
                    gz = p * (ez - vz + 1) + k
                    gy = p * (ey - vy + 1) + k
                    gx = p * (ex - vx + 1) + k
                    gid = ((gz[:, None, None] * m + gy[None, :, None]) * m + gx[None, None, :]).reshape(-1)
                    rows.append(gid[Ak.row])
                    cols.append(gid[Ak.col])
                    vals.append(Ak.data)
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(m ** 3, m ** 3)).tocsr()
        (pz, _), (py, _), (px, _) = self._axis(vz, d.nz), self._axis(vy, d.ny), self._axis(vx, d.nx)
        lz, ly, lx = pz - p * (vz - 1), py - p * (vy - 1), px - p * (vx - 1)
        local = ((lz[:, None, None] * m + ly[None, :, None]) * m + lx[None, None, :]).reshape(-1)
        return A[local][:, local]

    def fdm_matrix(self, v):
        """Sparse FDM-basis patch matrix A_j (surrogate form)."""
        A = self._assemble(v, self.AF, self.BF, sparse=True)
        A.eliminate_zeros()
        return A.tocsr()

    def gll_matrix(self, v):
        """Dense GLL-basis patch matrix of the surrogate (definition mode)."""
        return self._assemble(v, self.od["A"], self.od["B"], sparse=False).toarray()

    def factor(self, v):
        if v in self._cache:
            return self._cache[v]
        A = self.fdm_matrix(v)
        _, face = self.layout(v)
        I, G = np.flatnonzero(~face), np.flatnonzero(face)
        AII = A[I][:, I]
        D = AII.diagonal()
        off = AII - sp.diags(D)
        if off.nnz and np.max(np.abs(off.data)) != 0.0:
            raise AssertionError("interior block is not diagonal")
        AGI = A[G][:, I].tocsr()
        S = A[G][:, G].toarray() - (AGI @ sp.diags(1.0 / D) @ AGI.T).toarray()
        chol = sla.cho_factor(S, lower=True) if len(G) else None
        f = (I, G, D, AGI, chol)
        self._cache[v] = f
        return f

    def solve(self, v, r, cache=True):
        """u = A_j^{-1} r for one patch (FDM basis), by interior-first elimination."""
        I, G, D, AGI, chol = self.factor(v)
        if not cache:
            self._cache.pop(v, None)
        rI, rG = r[I], r[G]
        u = np.empty_like(r)
        if len(G):
            uG = sla.cho_solve(chol, rG - AGI @ (rI / D))
            u[G] = uG
            u[I] = (rI - AGI.T @ uG) / D
        else:
            u[I] = rI / D
        return u

    def solve_dense_gll(self, v, r):
        return np.linalg.solve(self.gll_matrix(v), r)

    def relax_fdm(self, rF, cache=True, vertices=None):
        """sum_j Rbar_j^T A_j^{-1} Rbar_j rF over the chosen patches (FDM covector -> coefficients)."""
        out = np.zeros_like(rF)
        for v in (self.vertices if vertices is None else vertices):
            idx = self.dofs(v)
            out[idx] += self.solve(v, rF[idx], cache=cache)
        return out

    def relax_gll_dense(self, r, vertices=None):
        """Definition of the relaxation: sum_j Rbar_j^T Atilde_j^{-1} Rbar_j r in the GLL basis."""
        out = np.zeros_like(r)
        for v in (self.vertices if vertices is None else vertices):
            idx = self.dofs(v)
            out[idx] += self.solve_dense_gll(v, r[idx])
        return out
