"""Learned separable surrogate: features, Theorem-1 ratio, labels and the MLP (FP64).

Test infrastructure only (see ``oracle/__init__``).

The paper's surrogate (Sec. 2.7) replaces G_hat on each cell by the constant
diagonal mu = cell average of diag(G_hat); Theorem 1 bounds a(v,v)/a~(v,v) on
the cell by the extreme eigenvalues c_K, C_K of mu^{-1/2} G_hat mu^{-1/2} over
the cell.  The paper has no learned part; this module writes out the reading
used to build one (parity of the learned part beyond these definitions is
unpinned):

* features of a cell: DF at the 2 x 2 x 2 Gauss points (xi = +-1/sqrt 3, x
  fastest, each DF row-major), scale-free and centred on the undistorted cube:
  FEATURE_GAIN * (DF / s - I) with s = |det DF(0)|^(1/3); then log kappa and the
  within-cell variance of log kappa (0 for a per-cell kappa): 74 values.  The
  gain 8 brings the geometric entries to about unit spread for vertex jitter of
  a fifth of the mesh size;
* Theorem-1 ratio of scalings mu: C_K / c_K with the eigenvalues taken at the
  3 x 3 x 3 points xi in {-1, 0, 1}^3;
* label delta*: the log-scaling (mu = mu_avg exp(delta)) minimising that ratio.
  The ratio is invariant under delta -> delta + t(1,1,1), and can be flat in
  other directions too (a cell sheared in one plane leaves the third scaling
  free), so the minimised objective is log(C/c) + 1e-6 |delta - mean(delta)|^2,
  which keeps the minimax value and picks, among ties, the scaling closest to
  the average.  The search is over delta = (a, b, 0) on a coarse-to-fine grid:
  17 x 17 points of step 1/8 around 0, then twice 9 x 9 points with the step
  divided by 4 around the best point (first minimum in row-major (a, b)
  order); finally every component is shifted by log(c C)/2 so that the
  spectrum is centred at 1 (c C = 1);
* MLP: 74 -> 64 -> 64 -> 3, GELU (erf form) on the hidden layers, predicting
  delta; loss = mean over samples and outputs of (y - t)^2.
"""
import math

import numpy as np
from scipy.special import erf

from .mesh import hat_1d

NIN, NH, NOUT = 74, 64, 3
PARAM_SHAPES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NOUT, NH)), ("b3", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in PARAM_SHAPES)
FEATURE_GAIN = 8.0


# ---------------------------------------------------------------- geometry per cell
def jacobian_at(corners, xi):
    """DF at reference points xi (npts, 3) for cells given by corners (ncell, 2, 2, 2, 3)
    indexed [cell, c(z), b(y), a(x), coord]: returns (ncell, npts, 3, 3), J[i, j] = dx_i/dxi_j."""
    N1, dN1 = hat_1d(xi[:, 0])
    N2, dN2 = hat_1d(xi[:, 1])
    N3, dN3 = hat_1d(xi[:, 2])
    g1 = np.einsum("pa,pb,pc->pcba", dN1, N2, N3)
    g2 = np.einsum("pa,pb,pc->pcba", N1, dN2, N3)
    g3 = np.einsum("pa,pb,pc->pcba", N1, N2, dN3)
    J = np.stack([np.einsum("pcba,ncbai->npi", g, corners) for g in (g1, g2, g3)], axis=-1)
    return J


def gauss_points():
    g = 1.0 / math.sqrt(3.0)
    return np.array([[x, y, z] for z in (-g, g) for y in (-g, g) for x in (-g, g)])


def sample_points():
    return np.array([[x, y, z] for z in (-1.0, 0.0, 1.0) for y in (-1.0, 0.0, 1.0) for x in (-1.0, 0.0, 1.0)])


def features(corners, kappa=None):
    ncell = corners.shape[0]
    J = jacobian_at(corners, gauss_points())                      # (ncell, 8, 3, 3)
    J0 = jacobian_at(corners, np.zeros((1, 3)))[:, 0]
    s = np.abs(np.linalg.det(J0)) ** (1.0 / 3.0)
    F = (FEATURE_GAIN * (J / s[:, None, None, None] - np.eye(3))).reshape(ncell, 72)
    logk = np.zeros(ncell) if kappa is None else np.log(np.asarray(kappa, dtype=np.float64))
    return np.concatenate([F, logk[:, None], np.zeros((ncell, 1))], axis=1)


def metric_at(corners, xi):
    """G_hat (without kappa) at points xi: (ncell, npts, 3, 3)."""
    J = jacobian_at(corners, xi)
    det = np.linalg.det(J)
    Ji = np.linalg.inv(J)
    return np.abs(det)[..., None, None] * (Ji @ np.swapaxes(Ji, -1, -2))


def mu_average(corners, q):
    """Cell average of diag(G_hat) with the q-point GLL rule (Sec. 2.7), kappa = 1."""
    from .gll import gll_points
    x, w = gll_points(q)
    pts = np.array([[a, b, c] for c in x for b in x for a in x])
    wt = np.array([wa * wb * wc for wc in w for wb in w for wa in w])
    G = metric_at(corners, pts)
    return np.einsum("p,npjj->nj", wt, G) / 8.0


# ---------------------------------------------------------------- Theorem 1
def spectrum_bounds(G, mu):
    """c_K = min eigenvalue, C_K = max eigenvalue of mu^{-1/2} G mu^{-1/2} over the points."""
    s = 1.0 / np.sqrt(mu)
    M = G * s[:, None, :, None] * s[:, None, None, :]
    ev = np.linalg.eigvalsh(M)
    return ev[..., 0].min(axis=1), ev[..., -1].max(axis=1)


def theorem1_ratio(G, mu):
    c, C = spectrum_bounds(G, mu)
    return C / c


def labels(corners, q):
    """delta* per cell (see module doc), and the ratio it attains."""
    G = metric_at(corners, sample_points())
    mu0 = mu_average(corners, q)
    ncell = corners.shape[0]
    best = np.zeros((ncell, 2))
    step = 1.0 / 8.0
    half = 8
    for level in range(3):
        if level > 0:
            step /= 4.0
            half = 4
        offs = np.arange(-half, half + 1) * step
        best_r = np.full(ncell, np.inf)
        new = best.copy()
        for da in offs:
            for db in offs:
                a = best[:, 0] + da
                b = best[:, 1] + db
                mu = mu0 * np.exp(np.stack([a, b, np.zeros(ncell)], axis=1))
                m = (a + b) / 3.0
                r = np.log(theorem1_ratio(G, mu)) + 1e-6 * ((a - m) ** 2 + (b - m) ** 2 + m ** 2)
                better = r < best_r
                best_r = np.where(better, r, best_r)
                new[better, 0] = a[better]
                new[better, 1] = b[better]
        best = new
    delta = np.stack([best[:, 0], best[:, 1], np.zeros(ncell)], axis=1)
    c, C = spectrum_bounds(G, mu0 * np.exp(delta))
    delta = delta + 0.5 * np.log(c * C)[:, None]
    return delta, C / c


# ---------------------------------------------------------------- MLP
def unpack(theta):
    out, o = {}, 0
    for name, shape in PARAM_SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, X):
    P = unpack(theta)
    z1 = X @ P["W1"].T + P["b1"]
    h1 = gelu(z1)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = gelu(z2)
    y = h2 @ P["W3"].T + P["b3"]
    return y, (z1, h1, z2, h2)


def loss_and_grad(theta, X, T):
    """Mean squared error over samples and outputs and its gradient (backpropagation)."""
    P = unpack(theta)
    y, (z1, h1, z2, h2) = forward(theta, X)
    n = X.shape[0]
    r = y - T
    loss = float(np.mean(r * r))
    dy = 2.0 * r / (n * NOUT)
    g = {"W3": dy.T @ h2, "b3": dy.sum(0)}
    dz2 = (dy @ P["W3"]) * gelu_prime(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ P["W2"]) * gelu_prime(z1)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return loss, np.concatenate([g[name].reshape(-1) for name, _ in PARAM_SHAPES])


def bf16_round(x):
    """Round float64 values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)
