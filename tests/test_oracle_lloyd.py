"""Pins for the oracle's randomized Lloyd iteration (grid optimization for the
quadratic quantization error, Sec. 2, eq. Qerr).

Pins: the optimal 2-point quantizer of N(0, 1) is +-sqrt(2/pi) with
distortion 1 - 2/pi (closed form); the optimal N-point quantizer of N(0, 1)
computed from the exact normal integrals (scipy) is a fixed point, and its
exact distortion matches the estimate; the product of two such grids is a
fixed point for N(0, I_2); one step equals cell means computed independently
in FP64 with numpy; on a fixed sample set the distortion never increases;
scaling L scales the result; the samples have covariance L L^T; a cell
without samples keeps its point.
"""
import numpy as np
import pytest
from scipy.stats import norm


def exact_lloyd_1d(N, iters=2000):
    """Optimal N-point quantizer of N(0, 1) by deterministic Lloyd steps with
    the exact conditional means E[Z | a < Z < b] = (phi(a) - phi(b)) / (Phi(b) - Phi(a))."""
    g = np.linspace(-2.0, 2.0, N)
    for _ in range(iters):
        e = np.concatenate([[-np.inf], 0.5 * (g[1:] + g[:-1]), [np.inf]])
        p = norm.cdf(e[1:]) - norm.cdf(e[:-1])
        g = (norm.pdf(e[:-1]) - norm.pdf(e[1:])) / p
    return g


def exact_distortion_1d(g):
    """E min_i (Z - g_i)^2 for a sorted 1-D grid, from the truncated moments."""
    e = np.concatenate([[-np.inf], 0.5 * (g[1:] + g[:-1]), [np.inf]])
    a, b = e[:-1], e[1:]
    p = norm.cdf(b) - norm.cdf(a)
    m1 = norm.pdf(a) - norm.pdf(b)                                     # E[Z; cell]
    ta = np.where(np.isinf(a), 0.0, a) * norm.pdf(a)                  # x phi(x) -> 0 at +-inf
    tb = np.where(np.isinf(b), 0.0, b) * norm.pdf(b)
    m2 = p + ta - tb                                                   # E[Z^2; cell]
    return float(np.sum(m2 - 2 * g * m1 + g * g * p))


def test_two_points_converge_to_the_closed_form(oracle_lib):
    g, dist = oracle_lib.lloyd(1, np.array([-0.3, 0.5]), [[1.0]], 200_000, 30, seed=7)
    assert np.allclose(g.ravel(), [-np.sqrt(2 / np.pi), np.sqrt(2 / np.pi)], atol=5e-3)
    assert dist[-1] == pytest.approx(1 - 2 / np.pi, abs=3e-3)
    assert dist[0] > dist[-1] + 0.1                     # the start is far from optimal


def test_exact_optimum_is_a_fixed_point_and_its_distortion_matches(oracle_lib):
    gopt = exact_lloyd_1d(8)
    g, dist = oracle_lib.lloyd(1, gopt, [[1.0]], 200_000, 4, seed=11)
    assert np.abs(g.ravel() - gopt).max() < 0.02
    assert dist.mean() == pytest.approx(exact_distortion_1d(gopt), rel=5e-3)
    # a grid 10 % too wide moves back towards the optimum
    g2, _ = oracle_lib.lloyd(1, 1.1 * gopt, [[1.0]], 200_000, 1, seed=11)
    assert np.all(np.abs(g2.ravel() - gopt) < np.abs(1.1 * gopt - gopt) + 1e-3)


def test_product_grid_is_a_fixed_point_in_two_dimensions(oracle_lib):
    g1 = exact_lloyd_1d(6)
    G = np.stack(np.meshgrid(g1, g1, indexing="ij"), axis=-1).reshape(-1, 2)
    g, dist = oracle_lib.lloyd(2, G, np.eye(2), 400_000, 1, seed=3)
    assert np.abs(g - G).max() < 0.04
    assert dist[0] == pytest.approx(2 * exact_distortion_1d(g1), rel=5e-3)


def test_one_step_equals_independent_cell_means(oracle_lib):
    d, M, seed = 2, 5000, 21
    L = np.array([[1.0, 0.0], [0.5, 0.8]])
    G = np.array([[-1.0, -0.5], [0.2, 0.9], [1.1, -0.3], [0.0, 0.0]], np.float32)
    g, dist = oracle_lib.lloyd(d, G, L, M, 1, seed=seed)
    X = oracle_lib.lloyd_samples(d, L, seed, 0, M).astype(np.float64)
    D = ((X[:, None, :] - G[None, :, :].astype(np.float64)) ** 2).sum(axis=2)
    cell = D.argmin(axis=1)
    for i in range(G.shape[0]):
        assert np.allclose(g[i], X[cell == i].mean(axis=0), rtol=0, atol=1e-6)
    assert dist[0] == pytest.approx(D.min(axis=1).mean(), rel=1e-6)


def test_distortion_never_increases_on_a_fixed_sample_set(oracle_lib):
    rng = np.random.default_rng(5)
    G = rng.normal(size=(40, 2)).astype(np.float32)
    _, dist = oracle_lib.lloyd(2, G, np.eye(2), 20_000, 25, seed=9, fresh=False)
    assert np.all(np.diff(dist) <= 1e-9 * dist[:-1])
    assert dist[-1] < 0.8 * dist[0]


def test_scaling_L_scales_the_grid(oracle_lib):
    g1 = exact_lloyd_1d(5)
    G = np.stack(np.meshgrid(g1, g1, indexing="ij"), axis=-1).reshape(-1, 2) * 0.9
    a, da = oracle_lib.lloyd(2, G, np.eye(2), 30_000, 3, seed=4)
    b, db = oracle_lib.lloyd(2, 2 * G, 2 * np.eye(2), 30_000, 3, seed=4)
    assert np.allclose(b, 2 * a, rtol=0, atol=1e-6)
    assert np.allclose(db, 4 * da, rtol=1e-6)


def test_samples_have_covariance_L_Lt(oracle_lib):
    L = np.array([[1.0, 0.0, 0.0], [0.8, 0.6, 0.0], [-0.3, 0.2, 0.5]])
    X = oracle_lib.lloyd_samples(3, L, 13, 2, 60_000).astype(np.float64)
    C = np.cov(X.T)
    assert np.allclose(C, L @ L.T, atol=0.02)
    assert not np.allclose(C, L.T @ L, atol=0.1)


def test_a_cell_without_samples_keeps_its_point(oracle_lib):
    G = np.array([[-0.5, 0.0], [0.5, 0.0], [40.0, 40.0]], np.float32)
    g, _ = oracle_lib.lloyd(2, G, np.eye(2), 10_000, 2, seed=1)
    assert np.array_equal(g[2], G[2])
    assert not np.array_equal(g[0], G[0])
