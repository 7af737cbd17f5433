"""Pins for the oracle's one-dimensional data (Sec. 2.1-2.4) against closed forms."""
import math
import os

import numpy as np
import pytest

from oracle.fdm1d import quad_points, reference_matrices, setup_1d
from oracle.gll import gll_points, lagrange, legendre
from oracle.solver import splitmix64

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        line = line.split("--")[0].strip()
        if not line or line.startswith("#"):
            continue
        key, *vals = line.split()
        out[key] = vals
    return out


G = golden()


def fvals(key):
    return np.array([float(v) for v in G[key]])


def test_gll_closed_forms():
    x, w = gll_points(4)
    np.testing.assert_allclose(x, fvals("gll4_nodes"), atol=1e-15)
    np.testing.assert_allclose(w, fvals("gll4_weights"), atol=1e-15)
    x, w = gll_points(5)
    np.testing.assert_allclose(x, fvals("gll5_nodes"), atol=1e-15)
    np.testing.assert_allclose(w, fvals("gll5_weights"), atol=1e-15)


@pytest.mark.parametrize("n", [2, 3, 6, 9, 16, 24, 33])
def test_gll_exactness(n):
    x, w = gll_points(n)
    assert abs(w.sum() - 2.0) < 1e-14
    # nodes: +-1 and roots of P'_{n-1}
    _, dp = legendre(n - 1, x[1:-1])
    if n > 2:
        assert np.max(np.abs(dp)) < 1e-10 * max(1, n * n)
    for k in range(2 * n - 2):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(w @ x ** k - exact) < 1e-13
    # Lobatto (not Gauss): degree 2n-2 is not integrated exactly
    k = 2 * n - 2
    if n <= 9:
        assert abs(w @ x ** k - 2.0 / (k + 1)) > 1e-6


@pytest.mark.parametrize("p", [1, 3, 7, 15])
def test_lagrange(p):
    xi, _ = gll_points(p + 1)
    V, D = lagrange(xi, xi)
    np.testing.assert_allclose(V, np.eye(p + 1), atol=1e-13)
    t = np.linspace(-1, 1, 13)
    Vt, Dt = lagrange(xi, t)
    np.testing.assert_allclose(Vt.sum(1), 1.0, atol=1e-12)
    for k in range(p + 1):
        np.testing.assert_allclose(Vt @ xi ** k, t ** k, atol=1e-11)
        np.testing.assert_allclose(Dt @ xi ** k, k * t ** max(k - 1, 0) if k else 0 * t, atol=1e-9)


def test_reference_matrices_p1():
    d = reference_matrices(1)
    np.testing.assert_allclose(d["A"].reshape(-1), fvals("A_hat_p1"), atol=1e-15)
    np.testing.assert_allclose(d["B"].reshape(-1), fvals("B_hat_p1"), atol=1e-15)


@pytest.mark.parametrize("p", [2, 3, 4, 7, 11, 15])
def test_reference_matrices_exact(p):
    d = reference_matrices(p)
    assert d["q"] == quad_points(p) == math.ceil(3 * (p + 1) / 2)
    A, B, xi = d["A"], d["B"], d["nodes"]
    one = np.ones(p + 1)
    np.testing.assert_allclose(A @ one, 0, atol=1e-11)
    assert abs(one @ B @ one - 2) < 1e-13
    # integrals of monomials represented by their nodal values
    for a in range(p + 1):
        for b in range(p + 1):
            ua, ub = xi ** a, xi ** b
            mass = 2.0 / (a + b + 1) if (a + b) % 2 == 0 else 0.0
            stiff = (a * b * 2.0 / (a + b - 1)) if a and b and (a + b) % 2 == 0 else 0.0
            assert abs(ua @ B @ ub - mass) < 1e-12
            assert abs(ua @ A @ ub - stiff) < 1e-10 * max(1, a * b)


def test_eigenvalues_closed_form():
    np.testing.assert_allclose(setup_1d(2)["lam"], fvals("lambda_p2"), rtol=1e-14)
    np.testing.assert_allclose(setup_1d(3)["lam"], fvals("lambda_p3"), rtol=1e-14)
    lam4 = setup_1d(4)["lam"]
    assert np.min(np.abs(lam4 - fvals("lambda_p4_odd")[0])) < 1e-12


@pytest.mark.parametrize("p", [3, 7, 11, 15])
def test_eigen_normalization_and_limit(p):
    d = setup_1d(p)
    I = slice(1, p)
    S, lam = d["S"], d["lam"]
    np.testing.assert_allclose(S.T @ d["B"][I, I] @ S, np.eye(p - 1), atol=1e-12)
    np.testing.assert_allclose(S.T @ d["A"][I, I] @ S, np.diag(lam), atol=1e-10 * lam.max())
    assert np.all(np.diff(lam) > 0)
    # Rayleigh-Ritz: each discrete eigenvalue bounds the continuous one from above
    j = np.arange(1, p)
    assert np.all(lam >= j ** 2 * np.pi ** 2 / 4 * (1 - 1e-12))
    if p >= 15:
        assert abs(lam[0] - fvals("lambda1_limit")[0]) < 1e-11
        # first eigenvector approximates sin(pi (1 + x)/2) at the interior nodes
        s1 = np.sin(np.pi * (1 + d["nodes"][1:-1]) / 2)
        assert np.max(np.abs(S[:, 0] - s1)) < 1e-9
    assert np.all(S[0, :] > 0)


@pytest.mark.parametrize("p", [2, 3, 7, 15])
def test_fdm_basis_structure_and_duality(p):
    d = setup_1d(p)
    T, AF, BF = d["T"], d["AF"], d["BF"]
    I = slice(1, p)
    scale = np.abs(d["A"]).max()
    np.testing.assert_allclose(BF[I, I], np.eye(p - 1), atol=1e-12)
    np.testing.assert_allclose(BF[I, 0], 0, atol=1e-12)
    np.testing.assert_allclose(BF[I, p], 0, atol=1e-12)
    off = AF[I, I] - np.diag(np.diag(AF[I, I]))
    assert np.abs(off).max() <= 1e-12 * scale * p
    np.testing.assert_allclose(np.diag(AF[I, I]), d["lam"], rtol=1e-11)
    # dual basis: values at -1, +1 and moments against the interior functions s_k
    xq, wq = d["xq"], d["wq"]
    Vq, _ = lagrange(d["nodes"], xq)
    phi = Vq @ T                        # FDM functions at the quadrature points
    s = Vq[:, I] @ d["S"]               # s_k as polynomials vanishing at +-1
    np.testing.assert_allclose(T[0], np.eye(p + 1)[0], atol=0)
    np.testing.assert_allclose(T[p], np.eye(p + 1)[p], atol=0)
    moments = (phi * wq[:, None]).T @ s
    expect = np.zeros((p + 1, p - 1))
    expect[1:p] = np.eye(p - 1)
    np.testing.assert_allclose(moments, expect, atol=1e-12)


def test_splitmix64_reference_outputs():
    ref = [int(v, 16) for v in G["splitmix64_seed0"]]
    assert [int(v) for v in splitmix64(0, 3)] == ref
