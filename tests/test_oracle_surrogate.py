"""Pins for the oracle's learned-surrogate definitions (features, Theorem 1, labels, MLP)."""
import numpy as np

from oracle import surrogate as S
from paper_2107_14758_amd import inputs


def box_cell(L=(0.5, 0.7, 1.3)):
    c = np.zeros((1, 2, 2, 2, 3))
    for cc in range(2):
        for b in range(2):
            for a in range(2):
                c[0, cc, b, a] = [a * L[0], b * L[1], cc * L[2]]
    return c


def sheared_cell(theta, L1=1.0, L2=1.4, L3=0.8):
    A = np.array([[L1, L2 * np.cos(theta), 0], [0, L2 * np.sin(theta), 0], [0, 0, L3]])
    c = np.zeros((1, 2, 2, 2, 3))
    for cc in range(2):
        for b in range(2):
            for a in range(2):
                c[0, cc, b, a] = A @ np.array([a, b, cc], dtype=float)
    return c


def test_features_of_affine_cells():
    c = box_cell()
    F = S.features(c)
    J = np.diag([0.25, 0.35, 0.65])
    s = np.linalg.det(J) ** (1 / 3)
    np.testing.assert_allclose(F[0, :72].reshape(8, 3, 3), np.broadcast_to(8.0 * (J / s - np.eye(3)), (8, 3, 3)),
                               atol=1e-13)
    # a cube (any size, any translation) maps to the zero feature vector
    np.testing.assert_allclose(S.features(box_cell((0.3, 0.3, 0.3)) + 5.0)[0], 0, atol=1e-13)
    assert F.shape == (1, 74) and F[0, 72] == 0 and F[0, 73] == 0


def test_cartesian_label_is_zero_and_ratio_one():
    d, r = S.labels(box_cell(), q=8)
    np.testing.assert_allclose(d, 0, atol=1e-14)
    np.testing.assert_allclose(r, 1, atol=1e-13)


def test_sheared_cell_ratio_matches_closed_form():
    # eq. (spectralboundstheta): sigma = [1-|cos t|, 1+|cos t|]; for this 2 x 2 block the averaged
    # (Jacobi) scaling is already the minimax one, so the label only recentres the spectrum
    for theta in (0.6, 1.2, 2.0):
        c = sheared_cell(theta)
        q = 8
        G = S.metric_at(c, S.sample_points())
        mu = S.mu_average(c, q)
        cs = abs(np.cos(theta))
        np.testing.assert_allclose(S.theorem1_ratio(G, mu), (1 + cs) / (1 - cs), rtol=1e-12)
        d, r = S.labels(c, q)
        # shape unchanged; the centring c C = 1 shifts every component by log((1-cs)(1+cs))/2 = log|sin t|
        np.testing.assert_allclose(d, np.full((1, 3), np.log(abs(np.sin(theta)))), atol=1e-12)
        np.testing.assert_allclose(r, (1 + cs) / (1 - cs), rtol=1e-12)


def test_labels_are_grid_optimal_on_a_finer_search():
    rng = np.random.default_rng(3)
    cells = inputs.random_cells(6, 0.2, rng)
    q = 8
    d, r = S.labels(cells, q)
    G = S.metric_at(cells, S.sample_points())
    mu0 = S.mu_average(cells, q)
    # centring: c C = 1 at the label
    c, C = S.spectrum_bounds(G, mu0 * np.exp(d))
    np.testing.assert_allclose(c * C, 1.0, rtol=1e-12)
    # no point of a finer brute-force grid around the label does better than the grid resolution allows
    for da in np.linspace(-0.05, 0.05, 11):
        for db in np.linspace(-0.05, 0.05, 11):
            mu = mu0 * np.exp(d + np.array([da, db, 0.0]))
            assert np.all(S.theorem1_ratio(G, mu) >= r * (1 - 2e-3))
    # and the label beats (or equals) the averaged scaling
    assert np.all(r <= S.theorem1_ratio(G, mu0) * (1 + 1e-12))


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    theta = inputs.mlp_init(rng).astype(np.float64)
    theta[S.NH * S.NIN:S.NH * S.NIN + S.NH] = rng.normal(size=S.NH) * 0.1
    X = rng.normal(size=(7, S.NIN))
    T = rng.normal(size=(7, S.NOUT))
    loss, g = S.loss_and_grad(theta, X, T)
    idx = rng.choice(S.NPARAM, 40, replace=False)
    h = 1e-6
    for j in idx:
        e = np.zeros_like(theta)
        e[j] = h
        fd = (S.loss_and_grad(theta + e, X, T)[0] - S.loss_and_grad(theta - e, X, T)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j]))
    assert S.NPARAM == 64 * 74 + 64 + 64 * 64 + 64 + 3 * 64 + 3


def test_bf16_rounding():
    vals = np.array([1.0, 1 + 2 ** -7, 1 + 2 ** -9, 1 + 3 * 2 ** -9, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 0.0])
    expect = np.array([1.0, 1 + 2 ** -7, 1.0, 1 + 2 ** -7, 1.0, 1 + 2 ** -6, -2.5, 0.0])
    np.testing.assert_array_equal(S.bf16_round(vals), expect)
