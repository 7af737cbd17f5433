"""Reference-interval matrices and the FDM basis (Sec. 2.2-2.4).

Test infrastructure only (see ``oracle/__init__``).

* A_hat[i,j] = int l_i' l_j',  B_hat[i,j] = int l_i l_j  on [-1, 1], in the GLL
  Lagrange basis, integrated with the q-point GLL rule used by the operator,
  q = ceil(3(p+1)/2) (Sec. 2.8 states 3(p+1)/2 points per direction; the
  ceiling is this implementation's reading for even p).  q >= p + 2, so both
  integrals are exact.
* The interior generalized eigenproblem A_II S = B_II S Lambda with
  S^T B_II S = I (Sec. 2.3) is solved through the Cholesky factor of B_II and a
  symmetric eigensolver; eigenvalues ascend and each eigenvector is signed so
  that its value at the first interior node is positive (the continuous
  eigenfunctions sin(j pi (1+x)/2) are positive just right of x = -1).
* The FDM basis (Sec. 2.4) is dual to {point values at -1 and +1, moments
  against the interior eigenfunctions s_j}.  Its GLL coefficients are the
  columns of T_hat:  interior columns are S itself; the vertex columns are
  l_0 (resp. l_p) plus the interior correction -B_II^{-1} B_I0 (resp. B_Ip)
  that makes their moments against every s_j vanish.
  A_F = T^T A T and B_F = T^T B T are the FDM-basis matrices.
"""
import math

import numpy as np

from .gll import gll_points, lagrange


def quad_points(p):
    """Default number of GLL quadrature points per direction."""
    return int(math.ceil(3 * (p + 1) / 2))


def reference_matrices(p, q=None):
    """Return dict with nodes, quadrature, interpolation and 1D matrices."""
    if q is None:
        q = quad_points(p)
    xi, _ = gll_points(p + 1)
    xq, wq = gll_points(q)
    Iq, Dq = lagrange(xi, xq)          # q x (p+1): values / derivatives at the points
    A = Dq.T @ (wq[:, None] * Dq)
    B = Iq.T @ (wq[:, None] * Iq)
    return dict(p=p, q=q, nodes=xi, xq=xq, wq=wq, Iq=Iq, Dq=Dq, A=A, B=B)


def fdm_basis(A, B):
    """Interior eigenpairs and the FDM change of basis (Sec. 2.3, 2.4).

    Returns (lam, S, T, AF, BF):  lam ascending (p-1,), S (p-1, p-1) with
    S^T A_II S = diag(lam), S^T B_II S = I; T (p+1, p+1) the GLL coefficients
    of the FDM basis (columns); AF, BF the matrices in the FDM basis.
    """
    n = A.shape[0]
    p = n - 1
    I = slice(1, p)
    Lc = np.linalg.cholesky(B[I, I])
    Linv = np.linalg.inv(Lc)
    C = Linv @ A[I, I] @ Linv.T
    C = 0.5 * (C + C.T)
    lam, Q = np.linalg.eigh(C)
    S = Linv.T @ Q
    S = S * np.where(S[0, :] < 0, -1.0, 1.0)[None, :]
    T = np.eye(n)
    T[I, I] = S
    T[I, 0] = -np.linalg.solve(B[I, I], B[I, 0])
    T[I, p] = -np.linalg.solve(B[I, I], B[I, p])
    AF = T.T @ A @ T
    BF = T.T @ B @ T
    return lam, S, T, AF, BF


def setup_1d(p, q=None):
    """All one-dimensional data of the method for degree p."""
    d = reference_matrices(p, q)
    lam, S, T, AF, BF = fdm_basis(d["A"], d["B"])
    d.update(lam=lam, S=S, T=T, AF=AF, BF=BF)
    return d
