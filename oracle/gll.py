"""GLL nodes, weights and Lagrange polynomials (Sec. 2.1).

Test infrastructure only (see ``oracle/__init__``).

The p+1 GLL nodes on [-1, 1] are the roots of (1 - x^2) P'_p(x), with P_k the
Legendre polynomial of degree k.  The n-point GLL rule (n = p + 1) has weights
w_i = 2 / (n (n - 1) P_{n-1}(x_i)^2) and integrates polynomials of degree up to
2n - 3 exactly.  The Lagrange polynomials are the product formula of Sec. 2.1,
l_j(x) = prod_{k != j} (x - xi_k) / (xi_j - xi_k).
"""
import numpy as np


def legendre(n, x):
    """P_n(x) and P_n'(x) by the three-term recurrence (float64)."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if n == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for k in range(1, n):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    # P_n' = n (x P_n - P_{n-1}) / (x^2 - 1), away from the endpoints;
    # at x = +-1 it is (+-1)^{n+1} n (n + 1) / 2.
    with np.errstate(divide="ignore", invalid="ignore"):
        dp = n * (x * p1 - p0) / (x * x - 1.0)
    end = np.isclose(np.abs(x), 1.0, rtol=0.0, atol=0.0)
    dp = np.where(end, np.sign(x) ** (n + 1) * n * (n + 1) / 2.0, dp)
    return p1, dp


def gll_points(n):
    """n-point Gauss-Lobatto-Legendre rule on [-1, 1] (n >= 2).

    Interior nodes are the roots of P'_{n-1}, found by Newton's method on
    P'_{n-1} starting from the Chebyshev-Gauss-Lobatto points.
    Returns (nodes ascending, weights).
    """
    if n < 2:
        raise ValueError("GLL needs at least 2 points")
    N = n - 1
    x = -np.cos(np.pi * np.arange(n) / N)
    interior = x[1:-1].copy()
    for _ in range(100):
        # d/dx P'_N = (2x P'_N - N(N+1) P_N) / (1 - x^2)  (Legendre ODE)
        pn, dpn = legendre(N, interior)
        ddpn = (2.0 * interior * dpn - N * (N + 1) * pn) / (1.0 - interior ** 2)
        step = dpn / ddpn
        interior -= step
        if np.all(np.abs(step) < 1e-16):
            break
    nodes = np.concatenate([[-1.0], np.sort(interior), [1.0]])
    pn, _ = legendre(N, nodes)
    weights = 2.0 / (n * N * pn ** 2)
    return nodes, weights


def lagrange(nodes, x):
    """Values V[i, j] = l_j(x_i) and derivatives D[i, j] = l_j'(x_i).

    Product formula of Sec. 2.1; the derivative is the product rule
    l_j'(x) = sum_{l != j} 1/(xi_j - xi_l) prod_{k != j, l} (x - xi_k)/(xi_j - xi_k).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(x), n))
    D = np.zeros((len(x), n))
    for j in range(n):
        for k in range(n):
            if k != j:
                V[:, j] *= (x - nodes[k]) / (nodes[j] - nodes[k])
        for l in range(n):
            if l == j:
                continue
            t = np.full(len(x), 1.0 / (nodes[j] - nodes[l]))
            for k in range(n):
                if k != j and k != l:
                    t *= (x - nodes[k]) / (nodes[j] - nodes[k])
            D[:, j] += t
    return V, D
