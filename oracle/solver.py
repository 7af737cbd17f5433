"""Relaxation, hybrid two-level preconditioner, damping and PCG (Sec. 2.5, 2.8).

Test infrastructure only (see ``oracle/__init__``).

* Relaxation (Sec. 2.5): S r = sum_j Rbar_j^T A_j^{-1} Rbar_j r with the
  surrogate patch matrices, applied in the FDM basis through the change of
  basis of Sec. 2.4:  S r = T (sum_j Rbar_j^T A_F,j^{-1} Rbar_j) T^T r.
* Coarse correction (Sec. 2.5): C r = P A_0^{-1} P^T r, dense Cholesky of A_0
  (coarse="direct"), or C r = P B P^T r with B one V(1,1) cycle of geometric
  multigrid for A_0 (coarse="gmg", Sec. 2.8 and ``gmg``).
* Hybrid V(1,1) (Sec. 2.5, multiplicative between the two levels, additive
  among patches):  z1 = w S r;  z2 = z1 + C (r - A z1);  z = z2 + w S (r - A z2).
  The fully additive variant is z = S r + C r.
* Damping (Sec. 2.5): w = 2 / ((1 + a) lmax + (1 - a) lmin), a = 1/4, with the
  extreme eigenvalues of S A estimated by CG-Lanczos: k steps of CG
  preconditioned by S from a pseudo-random start vector, the Lanczos
  tridiagonal built from the CG coefficients, its extreme eigenvalues taken.
  Reading: k = 20 steps; early stop once r^T S r has dropped below 1e-28 of
  its initial value; the start vector is entry i -> splitmix64 output i of the
  stream seeded with ``seed``, mapped to [-1, 1).
* PCG (Sec. 2.8): x0 = 0, stop when the Euclidean norm of the recursively
  updated residual is at most rtol ||b||_2; the iteration count is the number
  of updates of x.
* Condition estimate (Sec. 4, Table tab:poisson-cond): kappa(P^{-1} A) by
  CG-Lanczos on the solve itself, i.e. the extreme eigenvalues of the Lanczos
  tridiagonal built from the k step lengths and the k - 1 direction updates
  of the PCG run.
"""
import numpy as np
import scipy.linalg as sla

from . import transfer
from .gmg import Q1Multigrid
from .patches import Patches

ALPHA = 0.25
_M64 = (1 << 64) - 1


def splitmix64(seed, n):
    """Outputs 0..n-1 of the splitmix64 generator (Steele, Lea & Flood 2014)."""
    gamma = 0x9E3779B97F4A7C15
    out = np.empty(n, dtype=np.uint64)
    state = seed & _M64
    for i in range(n):
        state = (state + gamma) & _M64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        out[i] = z ^ (z >> 31)
    return out


def uniform_pm1(seed, n):
    """splitmix64 outputs mapped to [-1, 1) through their top 53 bits."""
    z = splitmix64(seed, n)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0


def lanczos_extremes(alphas, betas):
    """Extreme eigenvalues of the Lanczos tridiagonal of k (P)CG steps with step lengths
    alpha_0..alpha_{k-1} and direction updates beta_0..beta_{k-2} (a k-th beta is ignored):
    diagonal 1/alpha_j + beta_{j-1}/alpha_{j-1}, off-diagonal sqrt(beta_j)/alpha_j (the CG-Lanczos
    relation, Saad, Iterative Methods for Sparse Linear Systems, Sec. 6.7.3)."""
    k = len(alphas)
    Tk = np.zeros((k, k))
    for j in range(k):
        Tk[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            Tk[j, j + 1] = Tk[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    ev = np.linalg.eigvalsh(Tk)
    return float(ev[0]), float(ev[-1])


class Solver:
    def __init__(self, disc, od, mu=None, omega=None, lanczos_steps=20, seed=0, cycle="hybrid",
                 interior_only=False, coarse="direct"):
        self.disc = disc
        self.od = od
        self.patches = Patches(disc, od, mu, interior_only)
        self.T = od["T"]
        has_coarse = disc.nx > 1 and disc.ny > 1 and disc.nz > 1
        self.mg = None
        self.A0 = self.A0chol = None
        if coarse == "gmg":
            self.mg = Q1Multigrid.for_discretization(disc) if has_coarse else None
        elif coarse == "direct":
            self.A0 = transfer.coarse_matrix(disc) if has_coarse else None
            self.A0chol = sla.cho_factor(self.A0, lower=True) if self.A0 is not None and self.A0.size else None
        else:
            raise ValueError("coarse must be 'direct' or 'gmg'")
        self.cycle = cycle
        self.lanczos = None
        if omega is None:
            self.lanczos = self.estimate_extremes(lanczos_steps, seed)
            lmin, lmax = self.lanczos
            omega = 2.0 / ((1 + ALPHA) * lmax + (1 - ALPHA) * lmin)
        self.omega = omega

    # ---- building blocks ---------------------------------------------------------
    def A(self, x):
        return self.disc.apply(x)

    def relax(self, r):
        rF = transfer.fdm_restrict(self.disc, self.T, r)
        uF = self.patches.relax_fdm(rF)
        return transfer.fdm_prolong(self.disc, self.T, uF)

    def coarse(self, r):
        if self.mg is not None:
            rc = transfer.coarse_restrict(self.disc, r)
            return transfer.coarse_prolong(self.disc, self.mg.vcycle(rc))
        if self.A0chol is None:
            return np.zeros_like(r)
        rc = transfer.coarse_restrict(self.disc, r)
        ec = sla.cho_solve(self.A0chol, rc)
        return transfer.coarse_prolong(self.disc, ec)

    def precondition(self, r):
        if self.cycle == "additive":
            return self.relax(r) + self.coarse(r)
        w = self.omega
        z1 = w * self.relax(r)
        z2 = z1 + self.coarse(r - self.A(z1))
        return z2 + w * self.relax(r - self.A(z2))

    # ---- damping -----------------------------------------------------------------
    def estimate_extremes(self, steps, seed):
        """Extreme eigenvalues of S A from `steps` CG steps preconditioned by S."""
        r = uniform_pm1(seed, self.disc.n)
        z = self.relax(r)
        rz0 = rz = float(r @ z)
        p = z.copy()
        alphas, betas = [], []
        for _ in range(steps):
            q = self.A(p)
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

    # ---- Krylov solve --------------------------------------------------------------
    def pcg(self, b, rtol=1e-8, maxit=1000, history=False, lanczos=False):
        """x, iterations [, residual norms] [, (lmin, lmax) of the run's Lanczos tridiagonal]."""
        b = np.asarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        r = b.copy()
        bn = float(np.linalg.norm(b))
        hist = [bn]
        alphas, betas = [], []
        it = 0
        if bn > 0.0:
            z = self.precondition(r)
            p = z.copy()
            rz = float(r @ z)
            while it < maxit:
                q = self.A(p)
                alpha = rz / float(p @ q)
                alphas.append(alpha)
                x += alpha * p
                r -= alpha * q
                it += 1
                rn = float(np.linalg.norm(r))
                hist.append(rn)
                if rn <= rtol * bn:
                    break
                z = self.precondition(r)
                rz_new = float(r @ z)
                beta = rz_new / rz
                betas.append(beta)
                p = z + beta * p
                rz = rz_new
        out = (x, it)
        if history:
            out += (hist,)
        if lanczos:
            out += (lanczos_extremes(alphas, betas) if alphas else (0.0, 0.0),)
        return out
