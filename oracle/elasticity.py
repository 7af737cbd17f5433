"""Primal linear elasticity with the SDC/FDM/sparse relaxation (Sec. 3.1).

Test infrastructure only (see ``oracle/__init__``).

* Form (Sec. 3.1): a(v, u) = int 2 mu eps(v) : eps(u) + lam div v div u, with Lame
  parameters mu, lam constant over the mesh, Q_p in every displacement component and
  homogeneous Dirichlet conditions on the whole boundary (reading: the paper clamps one
  face only; this build's lattice of free DOFs has no Neumann faces).  A displacement
  vector is stored component after component, [u_1; u_2; u_3], each in the scalar
  lattice order of ``operator.Discretization``.
* Operator: matrix-free with the q^3 GLL rule of the scalar operator (Sec. 2.8):
  F = grad u at every point (reference gradients mapped by J^{-1}), sigma = mu (F + F^T)
  + lam tr(F) I, and the weak form integrates sigma : grad v.
* SDC (Sec. 3.1): the block diagonal diag(A_11, A_22, A_33) of the component blocks.  A_jj
  is the scalar form int grad v . K_j grad u with K_j = mu I + (mu + lam) e_j e_j^T, so its
  separable surrogate on a cell has the scalings of Sec. 2.7 with the metric
  |det J| J^{-1} K_j J^{-T}; on axis-aligned cells the surrogate is exact.  The SDC
  relaxation applies the scalar vertex-star FDM relaxation (Sec. 2.4-2.6) to each
  component with that component's scalings.
* Coarse space (Sec. 2.5): Q1 in every component, A_0 = P^T A P assembled from Q1 element
  matrices under the same quadrature, solved exactly.
* Preconditioner and solver: the hybrid V(1,1) cycle, damping by CG-Lanczos and PCG of
  ``solver`` (Sec. 2.5, 2.8), with the SDC relaxation in place of the scalar one.
"""
import numpy as np
import scipy.linalg as sla

from . import mesh as _mesh
from . import transfer
from .patches import Patches
from .solver import ALPHA, lanczos_extremes, uniform_pm1


class Elasticity:
    """The vector operator on the mesh of a scalar ``Discretization`` (float64)."""

    def __init__(self, disc, mu, lam):
        self.d = disc
        self.mu, self.lam = float(mu), float(lam)
        self.n = 3 * disc.n
        J = _mesh.jacobians(disc.vertices, disc.ref["xq"])          # (ncell, q, q, q, 3, 3)
        self.Jinv = np.linalg.inv(J)
        self.wdet = disc.w3[None] * np.abs(np.linalg.det(J))       # w_q |det J|

    def split(self, u):
        u = np.asarray(u, dtype=np.float64)
        return u[:self.d.n], u[self.d.n:2 * self.d.n], u[2 * self.d.n:]

    # ---- operator ---------------------------------------------------------------
    def ref_grad(self, uc):
        """Reference gradient of one component at every point: (ncell, q, q, q, 3)."""
        Iq, Dq = self.d.ref["Iq"], self.d.ref["Dq"]
        x = self.d.gather(uc)
        g1 = np.einsum("ck,bj,ai,nkji->ncba", Iq, Iq, Dq, x, optimize=True)
        g2 = np.einsum("ck,bj,ai,nkji->ncba", Iq, Dq, Iq, x, optimize=True)
        g3 = np.einsum("ck,bj,ai,nkji->ncba", Dq, Iq, Iq, x, optimize=True)
        return np.stack([g1, g2, g3], axis=-1)

    def ref_grad_T(self, W):
        """Transpose of ref_grad: W (ncell, q, q, q, 3) -> free-DOF vector."""
        Iq, Dq = self.d.ref["Iq"], self.d.ref["Dq"]
        yc = (np.einsum("ck,bj,ai,ncba->nkji", Iq, Iq, Dq, W[..., 0], optimize=True)
              + np.einsum("ck,bj,ai,ncba->nkji", Iq, Dq, Iq, W[..., 1], optimize=True)
              + np.einsum("ck,bj,ai,ncba->nkji", Dq, Iq, Iq, W[..., 2], optimize=True))
        return self.d.scatter_add(yc)

    def stress(self, F):
        """sigma = mu (F + F^T) + lam tr(F) I at every point; F[..., c, j] = du_c / dx_j."""
        tr = F[..., 0, 0] + F[..., 1, 1] + F[..., 2, 2]
        S = self.mu * (F + np.swapaxes(F, -1, -2))
        for c in range(3):
            S[..., c, c] += self.lam * tr
        return S

    def apply_full(self, ufull):
        """The unassembled-boundary form: ufull (3, Fz, Fy, Fx) on the whole lattice (no
        Dirichlet rows removed) -> the same shape; the sum over cells of the element operators."""
        d = self.d
        K, J, I = d.cell_index()
        Iq, Dq = d.ref["Iq"], d.ref["Dq"]

        def grad(full):
            x = full[K, J, I]
            return np.stack([np.einsum("ck,bj,ai,nkji->ncba", Iq, Iq, Dq, x, optimize=True),
                             np.einsum("ck,bj,ai,nkji->ncba", Iq, Dq, Iq, x, optimize=True),
                             np.einsum("ck,bj,ai,nkji->ncba", Dq, Iq, Iq, x, optimize=True)], axis=-1)

        F = np.stack([np.einsum("...r,...rj->...j", grad(ufull[c]), self.Jinv) for c in range(3)], axis=-2)
        S = self.stress(F)
        out = np.zeros_like(ufull)
        for c in range(3):
            W = np.einsum("...j,...rj->...r", S[..., c, :], self.Jinv) * self.wdet[..., None]
            yc = (np.einsum("ck,bj,ai,ncba->nkji", Iq, Iq, Dq, W[..., 0], optimize=True)
                  + np.einsum("ck,bj,ai,ncba->nkji", Iq, Dq, Iq, W[..., 1], optimize=True)
                  + np.einsum("ck,bj,ai,ncba->nkji", Dq, Iq, Iq, W[..., 2], optimize=True))
            np.add.at(out[c], (K, J, I), yc)
        return out

    def apply(self, u):
        """y = A u: F_cj = sum_r (du_c/dxi_r) (J^{-1})_rj; the test gradient of component c
        along xi_r is weighted by w |det J| sum_j sigma_cj (J^{-1})_rj."""
        F = np.stack([np.einsum("...r,...rj->...j", self.ref_grad(uc), self.Jinv) for uc in self.split(u)], axis=-2)
        S = self.stress(F)
        out = []
        for c in range(3):
            W = np.einsum("...j,...rj->...r", S[..., c, :], self.Jinv) * self.wdet[..., None]
            out.append(self.ref_grad_T(W))
        return np.concatenate(out)

    def load_vector(self, f):
        """b = [b_1; b_2; b_3], b_c the scalar load vector of the body-force component f[c]
        (each of shape (ncell, q, q, q))."""
        return np.concatenate([self.d.load_vector(f[c]) for c in range(3)])

    # ---- SDC scalings ----------------------------------------------------------
    def sdc_mu(self):
        """Per component j the surrogate scalings (ncell, 3) of A_jj: the cell average (Sec.
        2.7) of the diagonal of |det J| J^{-1} K_j J^{-T}, K_j = mu I + (mu + lam) e_j e_j^T."""
        det = np.abs(np.linalg.det(np.linalg.inv(self.Jinv)))
        out = []
        for j in range(3):
            K = self.mu * np.eye(3)
            K[j, j] += self.mu + self.lam
            G = det[..., None, None] * (self.Jinv @ K @ np.swapaxes(self.Jinv, -1, -2))
            out.append(_mesh.surrogate_mu(G, self.d.ref["wq"]))
        return out

    # ---- coarse space ----------------------------------------------------------
    def coarse_matrix(self):
        """A_0 = P^T A P for Q1 in every component, from Q1 element matrices (24 x 24, nodes
        within a component, component-major) under the operator's quadrature; rows and
        columns ordered [component][interior vertex]."""
        d = self.d
        N, dN = _mesh.hat_1d(d.ref["xq"])
        g1 = np.einsum("zc,yb,xa->zyxcba", N, N, dN).reshape(d.q ** 3, 8)
        g2 = np.einsum("zc,yb,xa->zyxcba", N, dN, N).reshape(d.q ** 3, 8)
        g3 = np.einsum("zc,yb,xa->zyxcba", dN, N, N).reshape(d.q ** 3, 8)
        gref = np.stack([g1, g2, g3], axis=-1)                       # (q^3, 8, r)
        Ji = self.Jinv.reshape(d.ncell, -1, 3, 3)
        wd = self.wdet.reshape(d.ncell, -1)
        gx = np.einsum("qar,nqrj->nqaj", gref, Ji)                   # physical gradients
        # a(v, u) for v = e_c phi_a, u = e_e phi_b: mu (grad_a . grad_b delta_ce + d_e phi_a d_c phi_b)
        # + lam d_c phi_a d_e phi_b
        Ae = np.zeros((d.ncell, 3, 8, 3, 8))
        lap = np.einsum("nq,nqaj,nqbj->nab", wd, gx, gx)
        for c in range(3):
            Ae[:, c, :, c, :] += self.mu * lap
            for e in range(3):
                Ae[:, c, :, e, :] += self.mu * np.einsum("nq,nqa,nqb->nab", wd, gx[..., e], gx[..., c])
                Ae[:, c, :, e, :] += self.lam * np.einsum("nq,nqa,nqb->nab", wd, gx[..., c], gx[..., e])
        nvz, nvy, nvx = d.nz + 1, d.ny + 1, d.nx + 1
        nv = nvz * nvy * nvx
        ez, ey, ex = np.meshgrid(np.arange(d.nz), np.arange(d.ny), np.arange(d.nx), indexing="ij")
        vid = np.stack([((ez + c) * nvy + (ey + b)) * nvx + (ex + a)
                        for c in range(2) for b in range(2) for a in range(2)], axis=-1).reshape(d.ncell, 8)
        A0full = np.zeros((3 * nv, 3 * nv))
        for e in range(d.ncell):
            idx = np.concatenate([c * nv + vid[e] for c in range(3)])
            A0full[np.ix_(idx, idx)] += Ae[e].reshape(24, 24)
        inner = np.zeros((nvz, nvy, nvx), dtype=bool)
        inner[1:-1, 1:-1, 1:-1] = True
        fid = np.flatnonzero(inner.reshape(-1))
        keep = np.concatenate([c * nv + fid for c in range(3)])
        return A0full[np.ix_(keep, keep)]


class SDCSolver:
    """Hybrid V(1,1) with the SDC/FDM/sparse relaxation and the vector Q1 coarse space."""

    def __init__(self, el, od, omega=None, lanczos_steps=20, seed=0, interior_only=False):
        self.el = el
        d = el.d
        self.T = od["T"]
        self.patches = [Patches(d, od, mu=m, interior_only=interior_only) for m in el.sdc_mu()]
        self.nc = transfer.coarse_shape(d)
        self.chol = sla.cho_factor(el.coarse_matrix(), lower=True)
        if omega is None:
            self.lanczos = self.estimate_extremes(lanczos_steps, seed)
            lmin, lmax = self.lanczos
            omega = 2.0 / ((1 + ALPHA) * lmax + (1 - ALPHA) * lmin)
        self.omega = omega

    def relax(self, r):
        """S r: per component, the scalar FDM vertex-star relaxation with its scalings."""
        d = self.el.d
        return np.concatenate([transfer.fdm_prolong(d, self.T, P.relax_fdm(transfer.fdm_restrict(d, self.T, rc)))
                               for P, rc in zip(self.patches, self.el.split(r))])

    def coarse(self, r):
        d = self.el.d
        rc = np.concatenate([transfer.coarse_restrict(d, x) for x in self.el.split(r)])
        ec = sla.cho_solve(self.chol, rc)
        m = rc.size // 3
        return np.concatenate([transfer.coarse_prolong(d, ec[c * m:(c + 1) * m]) for c in range(3)])

    def precondition(self, r):
        w = self.omega
        z1 = w * self.relax(r)
        z2 = z1 + self.coarse(r - self.el.apply(z1))
        return z2 + w * self.relax(r - self.el.apply(z2))

    def estimate_extremes(self, steps, seed):
        """Extreme eigenvalues of S A by CG-Lanczos from the seeded start vector (as the
        scalar solver, over the 3n vector)."""
        r = uniform_pm1(seed, self.el.n)
        z = self.relax(r)
        rz0 = rz = float(r @ z)
        p = z.copy()
        alphas, betas = [], []
        for _ in range(steps):
            q = self.el.apply(p)
            alpha = rz / float(p @ q)
            r = r - alpha * q
            z = self.relax(r)
            rz_new = float(r @ z)
            beta = rz_new / rz
            alphas.append(alpha)
            betas.append(beta)
            if rz_new <= 1e-28 * rz0:
                break
            p = z + beta * p
            rz = rz_new
        return lanczos_extremes(alphas, betas)

    def pcg(self, b, rtol=1e-8, maxit=1000):
        """x, iterations, (lmin, lmax) of the run's Lanczos tridiagonal."""
        b = np.asarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        r = b.copy()
        bn = float(np.linalg.norm(b))
        alphas, betas = [], []
        it = 0
        if bn > 0:
            z = self.precondition(r)
            p = z.copy()
            rz = float(r @ z)
            while it < maxit:
                q = self.el.apply(p)
                alpha = rz / float(p @ q)
                alphas.append(alpha)
                x += alpha * p
                r -= alpha * q
                it += 1
                if np.linalg.norm(r) <= rtol * bn:
                    break
                z = self.precondition(r)
                rz_new = float(r @ z)
                betas.append(rz_new / rz)
                p = z + betas[-1] * p
                rz = rz_new
        return x, it, (lanczos_extremes(alphas, betas) if alphas else (0.0, 0.0))
