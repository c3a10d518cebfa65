"""Pins for the oracle's grids from samples of a marginal of any law (Sec. 2:
sub-optimal grids that match the first two moments of X_k where no optimal
grid is available; the Lloyd condition of eq. Qerr on an empirical measure).

Moment-matching grid: sample sets with exactly known moments (symmetric
lattices) give their mean, covariance and Cholesky factor exactly; random
non-Gaussian samples agree with numpy's FP64 mean / covariance and
numpy.linalg.cholesky; Gaussian samples X = L z give L times the base grid
within the Monte Carlo error; the map is affine-equivariant.
Lloyd on samples: on the samples the randomized Lloyd iteration draws, it is
the same iteration bit for bit (the generator-driven oracle has its own
closed-form pins); a single cell moves to the sample mean, relaxed steps
follow the geometric closed form; the uniform law converges to its optimal
quantizer (2i + 1) / (2N); the windows wrap around the sample set as a
rotation of the array computed by numpy; inadmissible samples are counted
and ignored; on a fixed sample set the distortion never increases, the
result is a fixed point whose points are their cells' means by a brute-force
FP64 assignment, and Lloyd improves on the moment-matching grid of a
log-normal law.
"""
import numpy as np
import pytest

import synth


def test_moments_of_symmetric_lattices_are_exact(oracle_lib):
    O = oracle_lib
    # 1-D: a +- b with a, b dyadic: mean a, variance b^2, factor b
    x = np.array([[3.25 + 0.5], [3.25 - 0.5]] * 7, np.float32)
    base = np.array([[-1.0], [0.0], [2.0]], np.float32)
    g, mean, cov, chol, cnt = O.moment_grid(1, x, base)
    assert cnt == 14
    assert mean[0] == 3.25 and cov[0, 0] == 0.25 and chol[0, 0] == 0.5
    assert np.array_equal(g.ravel(), np.float32([2.75, 3.25, 4.25]))
    # 2-D: (s, (s + t) / 2) for s, t = +-1: covariance [[1, 1/2], [1/2, 1/2]],
    # factor [[1, 0], [1/2, 1/2]]
    pts = np.array([[s, 0.5 * (s + t)] for s in (-1, 1) for t in (-1, 1)], np.float32) + \
        np.float32([1.5, -2.0])
    g, mean, cov, chol, cnt = O.moment_grid(2, pts, np.float32([[1.0, 1.0], [-2.0, 4.0]]))
    assert np.array_equal(mean, [1.5, -2.0])
    assert np.array_equal(cov, [[1.0, 0.5], [0.5, 0.5]])
    assert np.array_equal(chol, [[1.0, 0.0], [0.5, 0.5]])
    assert np.array_equal(g, np.float32([[2.5, -1.0], [-0.5, -1.0]]))


@pytest.mark.parametrize("d", [1, 2, 3])
def test_moments_agree_with_numpy_on_non_gaussian_samples(oracle_lib, d):
    rng = np.random.default_rng(synth.SEED_BASE + d)
    M = 200_000
    z = rng.standard_normal((M, d))
    mix = np.tril(rng.uniform(0.2, 0.8, (d, d))) + np.eye(d)
    x = (np.exp(0.4 * z) @ mix.T + rng.uniform(-1, 1, (M, d))).astype(np.float32)
    base = rng.standard_normal((50, d)).astype(np.float32)
    g, mean, cov, chol, cnt = oracle_lib.moment_grid(d, x, base)
    x64 = x.astype(np.float64)
    ref_mean = x64.mean(axis=0)
    ref_cov = np.cov(x64, rowvar=False, bias=True).reshape(d, d)
    assert cnt == M
    assert np.allclose(mean, ref_mean, rtol=0, atol=1e-7)
    assert np.allclose(cov, ref_cov, rtol=0, atol=1e-5 * np.abs(ref_cov).max())
    ref_chol = np.linalg.cholesky(ref_cov)
    assert np.allclose(chol, ref_chol, rtol=0, atol=1e-5)
    assert np.allclose(g, ref_mean + base.astype(np.float64) @ ref_chol.T, atol=1e-4)


def test_gaussian_samples_give_the_scaled_base_grid(oracle_lib):
    L = np.array([[0.8, 0.0], [0.3, 0.5]])
    rng = np.random.default_rng(5)
    M = 400_000
    x = (rng.standard_normal((M, 2)) @ L.T).astype(np.float32)
    base = np.stack(np.meshgrid([-1.5, 0.0, 1.5], [-1.0, 1.0], indexing="ij"), -1).reshape(-1, 2)
    g, mean, cov, chol, _ = oracle_lib.moment_grid(2, x, base.astype(np.float32))
    se = 4.0 / np.sqrt(M)
    assert np.abs(mean).max() < se
    assert np.abs(chol - L).max() < 3 * se
    assert np.abs(g - base @ L.T).max() < 6 * se


def test_moment_grid_is_affine_equivariant(oracle_lib):
    rng = np.random.default_rng(9)
    x = rng.gamma(2.0, 0.5, (100_000, 2)).astype(np.float32)
    A = np.array([[2.0, 0.0], [0.5, 1.0]])            # lower triangular, positive diagonal
    c = np.array([-1.0, 0.25])
    y = (x.astype(np.float64) @ A.T + c).astype(np.float32)
    base = rng.standard_normal((20, 2)).astype(np.float32)
    gx, mx, _, Cx, _ = oracle_lib.moment_grid(2, x, base)
    gy, my, _, Cy, _ = oracle_lib.moment_grid(2, y, base)
    assert np.allclose(my, A @ mx + c, atol=1e-5)
    assert np.allclose(Cy, A @ Cx, atol=1e-4)
    assert np.allclose(gy, (gx.astype(np.float64) - mx) @ A.T + my, atol=1e-4)


@pytest.mark.parametrize("d", [1, 2])
def test_lloyd_on_generator_samples_is_the_randomized_lloyd(oracle_lib, d):
    O = oracle_lib
    L = [[0.9]] if d == 1 else [[0.9, 0.0], [0.2, 0.7]]
    M = 20_000
    x = O.lloyd_samples(d, L, seed=77, it=0, count=M, fresh=False)
    start = (np.linspace(-1.5, 1.5, 12).reshape(-1, 1) if d == 1 else
             np.stack(np.meshgrid(np.linspace(-1, 1, 4), np.linspace(-1, 1, 3), indexing="ij"),
                      -1).reshape(-1, 2)).astype(np.float32)
    ref, rdist = O.lloyd(d, start, L, M, 6, seed=77, fresh=False)
    got, gdist, rej = O.lloyd_empirical(d, start, x, M, 6)
    assert rej == 0
    assert np.array_equal(got, ref)
    assert np.array_equal(gdist, rdist)


def test_single_cell_moves_to_the_mean_and_relaxed_steps_are_geometric(oracle_lib):
    O = oracle_lib
    x = np.array([[0.5], [1.5], [2.0], [4.0]], np.float32)        # mean 2
    g, dist, _ = O.lloyd_empirical(1, np.float32([[-3.0]]), x, 4, 1)
    assert g[0, 0] == 2.0
    assert dist[0] == pytest.approx(np.mean((x.ravel() + 3.0) ** 2))
    gamma = 0.25
    g, _, _ = O.lloyd_empirical(1, np.float32([[-3.0]]), x, 4, 10, gamma=gamma)
    assert g[0, 0] == pytest.approx(2.0 + (1 - gamma) ** 10 * (-5.0), abs=1e-5)


def test_uniform_law_converges_to_its_optimal_quantizer(oracle_lib):
    M, N = 100_000, 8
    x = ((np.arange(M) + 0.5) / M).astype(np.float32).reshape(-1, 1)
    start = np.sort(np.random.default_rng(3).uniform(0.05, 0.6, N)).astype(np.float32)
    g, dist, _ = oracle_lib.lloyd_empirical(1, start.reshape(-1, 1), x, M, 1500)
    opt = (2 * np.arange(N) + 1) / (2 * N)
    assert np.abs(g.ravel() - opt).max() < 2e-4
    assert dist[-1] == pytest.approx(1.0 / (12 * N * N), rel=1e-3)
    assert np.all(np.diff(dist) <= 1e-5 * dist[:-1])     # up to the rounding of the sums


def test_windows_wrap_around_the_sample_set(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(21)
    M, B, steps = 1000, 370, 7
    x = rng.standard_normal((M, 2)).astype(np.float32)
    start = rng.standard_normal((9, 2)).astype(np.float32)
    got, gdist, _ = O.lloyd_empirical(2, start, x, B, steps)
    g = start.copy()
    for t in range(steps):
        window = np.roll(x, -((t * B) % M), axis=0)[:B]
        g, dt, _ = O.lloyd_empirical(2, g, window, B, 1)
        assert dt[0] == gdist[t]
    assert np.array_equal(g, got)


def test_inadmissible_samples_are_counted_and_ignored(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(4)
    good = rng.standard_normal((500, 2)).astype(np.float32)
    bad = np.float32([[np.nan, 0.0], [0.0, np.inf], [65.0, 0.0], [0.0, -64.5]])
    x = np.concatenate([good[:200], bad, good[200:]])
    start = rng.standard_normal((6, 2)).astype(np.float32)
    got, gdist, rej = O.lloyd_empirical(2, start, x, x.shape[0], 3)
    ref, rdist, rej0 = O.lloyd_empirical(2, start, good, good.shape[0], 3)
    assert rej == 3 * 4 and rej0 == 0
    assert np.array_equal(got, ref) and np.array_equal(gdist, rdist)
    cnt, _, _ = O.sample_moments(2, x)
    assert cnt == 500
    # the edge itself is admissible
    assert O.sample_moments(1, np.float32([[64.0], [-64.0]]))[0] == 2


def test_fixed_sample_set_gives_a_stationary_grid_better_than_moment_matching(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(8)
    M = 20_000
    x = np.exp(0.5 * rng.standard_normal((M, 2)) @ np.array([[1.0, 0.0], [0.6, 0.8]]).T)
    x = x.astype(np.float32)
    b1 = np.linspace(-1.6, 1.6, 5)
    base = np.stack(np.meshgrid(b1, b1, indexing="ij"), -1).reshape(-1, 2).astype(np.float32)
    gm, mean, _, _, _ = O.moment_grid(2, x, base)
    g, dist, _ = O.lloyd_empirical(2, gm, x, M, 300)
    assert np.all(np.diff(dist) <= 1e-5 * dist[:-1])     # up to the rounding of the sums
    assert dist[-1] < 0.8 * dist[0]          # the moment grid is sub-optimal for this law
    # a fixed point: each point is the FP64 mean of its brute-force cell
    x64, g64 = x.astype(np.float64), g.astype(np.float64)
    cell = np.argmin(((x64[:, None, :] - g64[None]) ** 2).sum(-1), axis=1)
    for i in range(g.shape[0]):
        sel = cell == i
        if sel.sum() > 0:
            assert np.allclose(x64[sel].mean(axis=0), g64[i], atol=2e-6)
