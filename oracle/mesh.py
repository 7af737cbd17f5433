"""Hexahedral cells, the weighted inverse metric and the separable surrogate (Sec. 2.1, 2.7).

Test infrastructure only (see ``oracle/__init__``).

A structured mesh of nx * ny * nz hexahedra is given by its vertex array
``vertices[kz, ky, kx, :]`` (shape (nz+1, ny+1, nx+1, 3)).  Cell (ez, ey, ex)
is the trilinear image F_K of the reference cube [-1, 1]^3 whose corner
(a, b, c) in {0,1}^3 (x, y, z) maps to vertices[ez+c, ey+b, ex+a].  Reference
axis 1 is x (fastest index).

For the Poisson form, a_K(v, u) = int_Khat grad v . G_hat grad u, with
G_hat = kappa_K |det DF| DF^{-1} DF^{-T}  (Sec. 2.7; kappa_K is a per-cell
constant coefficient, the reading used for the variable-coefficient
workloads).  The surrogate coefficients are the cell averages
mu_j = (1/|Khat|) int_Khat G_hat_jj  (Sec. 2.7), evaluated with the operator's
quadrature rule; |Khat| = 8.
"""
import numpy as np


def hat_1d(x):
    """Linear reference functions N_0 = (1-x)/2, N_1 = (1+x)/2 and derivatives."""
    x = np.asarray(x, dtype=np.float64)
    N = np.stack([(1 - x) / 2, (1 + x) / 2], axis=-1)
    dN = np.stack([np.full_like(x, -0.5), np.full_like(x, 0.5)], axis=-1)
    return N, dN


def cell_corners(vertices):
    """(ncell, 2, 2, 2, 3) corner coordinates indexed [cell, c(z), b(y), a(x), :].

    Cells are numbered ex + nx * (ey + ny * ez).
    """
    V = np.asarray(vertices, dtype=np.float64)
    nz, ny, nx = V.shape[0] - 1, V.shape[1] - 1, V.shape[2] - 1
    out = np.empty((nz, ny, nx, 2, 2, 2, 3))
    for c in range(2):
        for b in range(2):
            for a in range(2):
                out[:, :, :, c, b, a, :] = V[c:c + nz, b:b + ny, a:a + nx, :]
    return out.reshape(nz * ny * nx, 2, 2, 2, 3)


def jacobians(vertices, x1d):
    """DF at the tensor points x1d^3: (ncell, n, n, n, 3, 3), J[..., i, j] = dx_i/dxi_j.

    Point (i3, i2, i1) is (xi_1, xi_2, xi_3) = (x1d[i1], x1d[i2], x1d[i3]).
    """
    X = cell_corners(vertices)
    N, dN = hat_1d(x1d)               # (n, 2)
    # d/dxi_1: derivative on the a (x) corner index, values on b, c.
    J1 = np.einsum("zc,yb,xa,ncbad->nzyxd", N, N, dN, X)
    J2 = np.einsum("zc,yb,xa,ncbad->nzyxd", N, dN, N, X)
    J3 = np.einsum("zc,yb,xa,ncbad->nzyxd", dN, N, N, X)
    return np.stack([J1, J2, J3], axis=-1)


def physical_points(vertices, x1d):
    """F_K at the tensor points: (ncell, n, n, n, 3)."""
    X = cell_corners(vertices)
    N, _ = hat_1d(x1d)
    return np.einsum("zc,yb,xa,ncbad->nzyxd", N, N, N, X)


def inverse_metric(J, kappa=None):
    """G_hat = kappa |det J| J^{-1} J^{-T} at every point, and det J."""
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    G = np.abs(det)[..., None, None] * (Jinv @ np.swapaxes(Jinv, -1, -2))
    if kappa is not None:
        k = np.asarray(kappa, dtype=np.float64).reshape(-1)
        G = G * k.reshape((-1,) + (1,) * (G.ndim - 1))
    return G, det


def surrogate_mu(G, wq):
    """mu_j = (1/8) sum_q w_q G_jj (cell average of the diagonal), shape (ncell, 3)."""
    w3 = np.einsum("c,b,a->cba", wq, wq, wq)
    diag = np.stack([G[..., 0, 0], G[..., 1, 1], G[..., 2, 2]], axis=-1)
    return np.einsum("cba,ncbaj->nj", w3, diag) / 8.0


def cartesian_mu(lengths):
    """Closed form on an axis-aligned box (Sec. 2.2): mu_j = L_j^{-2} prod_i L_i,
    with L_j the box length along axis j divided by |Ihat| = 2."""
    L = np.asarray(lengths, dtype=np.float64) / 2.0
    return np.prod(L) / L ** 2
