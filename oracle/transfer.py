"""Change to the FDM basis and the low-order coarse space (Sec. 2.4, 2.5).

Test infrastructure only (see ``oracle/__init__``).

Basis change.  A function with FDM coefficients u_F has GLL coefficients
u = T u_F, evaluated cell by cell as (T_hat x T_hat x T_hat) u_F,K (Sec. 2.4:
the method is applied in another basis by interpolation and restriction).
The value at a node shared by several cells is the same from every cell,
because T_hat maps the vertex coefficients to themselves (its first and last
rows are unit vectors).  The restriction of a residual to FDM covectors is the
transpose, T^T r = sum_K R_K^T (T_hat^T)^{x3} W_K R_K r, where W_K divides each
node by the number of cells that contain it, so every (node, FDM-function)
pair is counted once.

Coarse space.  The lowest-order (Q1) space on the same mesh, with one DOF per
interior vertex (Sec. 2.5).  P interpolates Q1 functions at the GLL nodes:
per cell (N x N x N) with N the linear reference functions at the GLL nodes.
A_0 = P^T A P is the Galerkin coarse matrix; since Q1 is a subspace of Q_p and
the same quadrature is used, it equals the Q1 element matrices integrated with
that quadrature and summed, which is how it is built here.
"""
import numpy as np

from .mesh import hat_1d
from .operator import kron3


def multiplicity(disc):
    """Number of cells containing each node, per cell view: (ncell, p+1, p+1, p+1)."""
    count = np.zeros(disc.full_shape)
    K, J, I = disc.cell_index()
    np.add.at(count, (K, J, I), 1.0)
    return count[K, J, I]


def fdm_prolong(disc, T, uF):
    """u = T u_F on the free DOFs (FDM coefficients -> GLL nodal values)."""
    T3 = kron3(T, T, T)
    uc = disc.gather(uF).reshape(disc.ncell, -1)
    vc = uc @ T3.T
    K, J, I = disc.cell_index()
    full = np.zeros(disc.full_shape)
    full[K, J, I] = vc.reshape(K.shape)          # shared nodes: identical values
    return disc.from_full(full)


def fdm_restrict(disc, T, r):
    """r_F = T^T r on the free DOFs (GLL residual -> FDM covector)."""
    T3 = kron3(T, T, T)
    rc = (disc.gather(r) / multiplicity(disc)).reshape(disc.ncell, -1)
    sc = rc @ T3
    return disc.scatter_add(sc.reshape((disc.ncell,) + (disc.p + 1,) * 3))


# ---- coarse space -------------------------------------------------------------
def coarse_shape(disc):
    return (disc.nz - 1, disc.ny - 1, disc.nx - 1)


def coarse_prolong(disc, ec):
    """P e_c: interpolate interior-vertex values (Q1) at all free GLL nodes."""
    N, _ = hat_1d(disc.ref["nodes"])                     # (p+1, 2)
    P3 = kron3(N, N, N)                                  # ((p+1)^3, 8)
    vfull = np.zeros((disc.nz + 1, disc.ny + 1, disc.nx + 1))
    vfull[1:-1, 1:-1, 1:-1] = np.asarray(ec).reshape(coarse_shape(disc))
    corners = np.stack([vfull[c:c + disc.nz, b:b + disc.ny, a:a + disc.nx]
                        for c in range(2) for b in range(2) for a in range(2)], axis=-1)
    corners = corners.reshape(disc.ncell, 8)
    vals = corners @ P3.T
    K, J, I = disc.cell_index()
    full = np.zeros(disc.full_shape)
    full[K, J, I] = vals.reshape(K.shape)
    return disc.from_full(full)


def coarse_restrict(disc, r):
    """P^T r, with the same per-cell multiplicity weighting as fdm_restrict."""
    N, _ = hat_1d(disc.ref["nodes"])
    P3 = kron3(N, N, N)
    rc = (disc.gather(r) / multiplicity(disc)).reshape(disc.ncell, -1)
    cc = rc @ P3                                         # (ncell, 8) corner covectors
    vfull = np.zeros((disc.nz + 1, disc.ny + 1, disc.nx + 1))
    cc = cc.reshape(disc.nz, disc.ny, disc.nx, 2, 2, 2)
    for c in range(2):
        for b in range(2):
            for a in range(2):
                vfull[c:c + disc.nz, b:b + disc.ny, a:a + disc.nx] += cc[..., c, b, a]
    return vfull[1:-1, 1:-1, 1:-1].reshape(-1).copy()


def coarse_matrix(disc):
    """A_0 over interior vertices, from Q1 element matrices under the operator's quadrature."""
    xq = disc.ref["xq"]
    N, dN = hat_1d(xq)                                   # (q, 2)
    g1 = np.einsum("zc,yb,xa->zyxcba", N, N, dN).reshape(disc.q ** 3, 8)
    g2 = np.einsum("zc,yb,xa->zyxcba", N, dN, N).reshape(disc.q ** 3, 8)
    g3 = np.einsum("zc,yb,xa->zyxcba", dN, N, N).reshape(disc.q ** 3, 8)
    grad = np.stack([g1, g2, g3], axis=-1)               # (q^3, 8, 3)
    Gq = disc.Gw.reshape(disc.ncell, -1, 3, 3)
    Ae = np.einsum("qai,nqij,qbj->nab", grad, Gq, grad, optimize=True)
    nvz, nvy, nvx = disc.nz + 1, disc.ny + 1, disc.nx + 1
    ez, ey, ex = np.meshgrid(np.arange(disc.nz), np.arange(disc.ny), np.arange(disc.nx), indexing="ij")
    vid = np.stack([((ez + c) * nvy + (ey + b)) * nvx + (ex + a)
                    for c in range(2) for b in range(2) for a in range(2)], axis=-1).reshape(disc.ncell, 8)
    A0full = np.zeros((nvz * nvy * nvx,) * 2)
    for e in range(disc.ncell):
        A0full[np.ix_(vid[e], vid[e])] += Ae[e]
    inner = np.zeros((nvz, nvy, nvx), dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    fid = np.flatnonzero(inner.reshape(-1))
    return A0full[np.ix_(fid, fid)]
