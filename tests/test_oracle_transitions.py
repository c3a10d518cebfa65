"""Pins for the oracle's transition counts (Sec. 3 Algorithm I, Sec. 4
Algorithm III).

The law of the counts is fixed by the mathematics: for an AR(1) chain with
Gaussian marginals, P(X_k in C_i, X_{k+1} in C_j) is a one-dimensional
integral of normal distribution functions over the Voronoi intervals
(computed here by quadrature), the Brownian and Ornstein-Uhlenbeck
covariances are closed forms, and the counting itself obeys exact
invariants (totals, pathwise flow conservation, additivity over sample
chunks, independence from the thread split).
"""
import numpy as np
import pytest
from scipy import stats

import synth
from tests import _exact


def _model(oracle_lib, spec):
    return oracle_lib.Model(spec["d"], spec["n"], spec["A"], spec["b"], spec["T"],
                            spec["mu"], spec["L"], spec["x0"])


def _layer_grid(grid, N, k, d):
    off = np.concatenate([[0], np.cumsum(N)])
    return grid[off[k]:off[k + 1]].reshape(-1, d)


@pytest.mark.parametrize("mode", [0, 1])
def test_1d_counts_follow_exact_transition_law(oracle_lib, mode):
    """Counts of every layer against M * P_ij from exact integration over
    the 1-D Voronoi intervals (chi-square, Bonferroni max |z|)."""
    n, M = 5, 200_000
    spec = synth.bm_model(1, n, T=1.0)
    Ns = [1] + [9, 12, 15, 10, 14]
    grid, N = synth.layer_grids(spec, Ns)
    mdl = _model(oracle_lib, spec)
    counts = oracle_lib.transitions(mdl, grid, N, M, seed=0x5EED0001, mode=mode, nthreads=4)
    for k in range(n):
        ck = oracle_lib.layer_counts(counts, N, k)
        assert ck.sum() == M
        g0 = _layer_grid(grid, N, k, 1)[:, 0]
        g1 = _layer_grid(grid, N, k + 1, 1)[:, 0]
        s = float(spec["L"][k, 0, 0])
        P = _exact.transition_probs_1d(g0, g1, float(spec["mu"][k, 0]), s,
                                       float(spec["A"][k, 0, 0]), float(spec["b"][k, 0]),
                                       float(spec["T"][k, 0, 0]))
        assert abs(P.sum() - 1.0) < 1e-9
        stat, dof, zmax = _exact.chi2_check(ck, P)
        assert stats.chi2.sf(stat, dof) > 1e-5, (k, stat, dof)
        assert zmax < 5.5


def test_2d_product_grid_counts_factorise(oracle_lib):
    """Independent components on a product grid: the 2-D cells are products
    of 1-D intervals, so P((i1,i2) -> (j1,j2)) = P1(i1 -> j1) P2(i2 -> j2)."""
    n, M = 3, 300_000
    spec = synth.bm_model(2, n, T=1.0, rho=0.0)
    shapes = [1, (4, 5), (5, 4), (6, 3)]
    grid, N = synth.layer_grids(spec, shapes)
    mdl = _model(oracle_lib, spec)
    for mode in (0, 1):
        counts = oracle_lib.transitions(mdl, grid, N, M, seed=0x5EED0002, mode=mode,
                                        nthreads=4)
        for k in range(n):
            ck = oracle_lib.layer_counts(counts, N, k)
            assert ck.sum() == M
            sh0 = (1, 1) if k == 0 else shapes[k]
            sh1 = shapes[k + 1]
            g0 = _layer_grid(grid, N, k, 2)
            g1 = _layer_grid(grid, N, k + 1, 2)
            Ps = []
            for a in range(2):
                ax0 = np.unique(g0[:, a])
                ax1 = np.unique(g1[:, a])
                assert len(ax0) == sh0[a] and len(ax1) == sh1[a]
                s = float(spec["L"][k, a, a])
                Ps.append(_exact.transition_probs_1d(ax0, ax1, 0.0, s, 1.0, 0.0,
                                                     float(spec["T"][k, a, a])))
            # grid index = i_a * n_b + i_b (meshgrid 'ij' order)
            P = np.einsum("ac,bd->abcd", Ps[0], Ps[1]).reshape(N[k], N[k + 1])
            stat, dof, zmax = _exact.chi2_check(ck, P)
            assert stats.chi2.sf(stat, dof) > 1e-5, (mode, k, stat, dof)
            assert zmax < 5.5


def _cov_check(X, Y, Sxx, Sxy, Syy, M):
    Z = np.concatenate([X, Y], axis=1).astype(np.float64)
    S = np.block([[Sxx, Sxy.T], [Sxy, Syy]])
    emp = np.cov(Z, rowvar=False, bias=True)
    mean = Z.mean(axis=0)
    se_mean = np.sqrt(np.diag(S) / M)
    assert np.all(np.abs(mean) < 5.5 * se_mean), mean
    se = np.sqrt((np.outer(np.diag(S), np.diag(S)) + S * S) / M)
    z = np.abs(emp - S) / se
    assert z.max() < 5.5, (emp, S)


@pytest.mark.parametrize("d,rho", [(2, 0.3), (3, -0.4), (2, 0.9)])
def test_layer_pairs_have_brownian_covariance(oracle_lib, d, rho):
    """(X_k, X_{k+1}) of the correlated Brownian state: Cov(X_k) = t_k R,
    Cov(X_{k+1}, X_k) = t_k R, Cov(X_{k+1}) = t_{k+1} R."""
    n, M = 4, 200_000
    spec = synth.bm_model(d, n, T=2.0, rho=rho)
    mdl = _model(oracle_lib, spec)
    R = synth.corr_matrix(d, rho)
    for k in (1, 3):
        X, Y = oracle_lib.layer_pairs(mdl, k, 0, M, seed=0x5EED0003 + k)
        tk, tk1 = 2.0 * k / n, 2.0 * (k + 1) / n
        _cov_check(X, Y, tk * R, tk * R, tk1 * R, M)


def test_layer_pairs_have_ou_covariance(oracle_lib):
    """Two-factor Ornstein-Uhlenbeck state (Sec. 3): Cov(X_k)_ab =
    s_a s_b rho_ab (1 - e^{-(a_a + a_b) t}) / (a_a + a_b) and
    Cov(X_{k+1}, X_k) = diag(e^{-a dt}) Cov(X_k)."""
    n, M = 6, 200_000
    alpha, sig, rho = (0.5, 8.0), (0.7, 1.3), -0.6
    spec = synth.ou_model(n, alpha=alpha, sig=sig, rho=rho, T=1.0)
    mdl = _model(oracle_lib, spec)
    a, s = np.array(alpha), np.array(sig)
    R = synth.corr_matrix(2, rho)

    def cov(t):
        lam = a[:, None] + a[None, :]
        return np.outer(s, s) * R * (1 - np.exp(-lam * t)) / lam

    k = 3
    X, Y = oracle_lib.layer_pairs(mdl, k, 0, M, seed=0x5EED0004)
    dt = 1.0 / n
    Sxx, Syy = cov(k * dt), cov((k + 1) * dt)
    Sxy = np.diag(np.exp(-a * dt)) @ Sxx
    _cov_check(X, Y, Sxx, Sxy, Syy, M)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_path_noise_is_iid_standard(oracle_lib, d):
    m_count, n = 20_000, 8
    E = np.array([[oracle_lib.path_noise(d, k, m, 0x5EED0005) for k in range(n)]
                  for m in range(m_count)])          # [m][k][d]
    flat = E.reshape(-1, d)
    assert np.all(np.abs(flat.mean(axis=0)) < 5.5 / np.sqrt(flat.shape[0]))
    C = np.cov(flat, rowvar=False).reshape(d, d)
    assert np.all(np.abs(C - np.eye(d)) < 5.5 * np.sqrt(2.0 / flat.shape[0]))
    # consecutive steps of one path are uncorrelated (they share Philox blocks)
    for k in range(n - 1):
        c = np.corrcoef(E[:, k, 0], E[:, k + 1, 0])[0, 1]
        assert abs(c) < 5.5 / np.sqrt(m_count)


def test_pathwise_flow_conservation_and_totals(oracle_lib):
    n, M = 6, 50_000
    for d in (1, 2):
        spec = synth.bm_model(d, n, T=1.0, rho=0.2)
        Ns = [1] + ([20, 30, 25, 40, 22, 31] if d == 1 else [(4, 5), (5, 6), (5, 5), (8, 5),
                                                           (2, 11), (1, 31)])
        grid, N = synth.layer_grids(spec, Ns)
        mdl = _model(oracle_lib, spec)
        counts = oracle_lib.transitions(mdl, grid, N, M, seed=9, mode=1, nthreads=3)
        for k in range(n):
            ck = oracle_lib.layer_counts(counts, N, k)
            assert ck.sum() == M
            if k + 1 < n:
                nxt = oracle_lib.layer_counts(counts, N, k + 1)
                assert np.array_equal(ck.sum(axis=0), nxt.sum(axis=1))


@pytest.mark.parametrize("mode", [0, 1])
def test_chunk_additivity_and_thread_independence(oracle_lib, mode):
    n = 4
    for d in (1, 2, 3):
        spec = synth.bm_model(d, n, T=1.0, rho=0.1)
        Ns = [1] + ([11, 13, 17, 19] if d == 1 else [(3,) * d if d == 3 else (3, 4)] * n)
        grid, N = synth.layer_grids(spec, Ns)
        mdl = _model(oracle_lib, spec)
        full = oracle_lib.transitions(mdl, grid, N, 20_001, seed=77, mode=mode, nthreads=1)
        a = oracle_lib.transitions(mdl, grid, N, 7_777, seed=77, mode=mode, m0=0, nthreads=2)
        b = oracle_lib.transitions(mdl, grid, N, 12_224, seed=77, mode=mode, m0=7_777,
                                   nthreads=3)
        assert np.array_equal(full, a + b)
        other = oracle_lib.transitions(mdl, grid, N, 20_001, seed=77, mode=mode, contract=1,
                                       nthreads=4)
        assert not np.array_equal(full, other)
        assert other.sum() == full.sum() == 20_001 * n


def test_invalid_arguments_rejected(oracle_lib):
    spec = synth.bm_model(1, 2)
    grid, N = synth.layer_grids(spec, [1, 5, 5])
    mdl = _model(oracle_lib, spec)
    with pytest.raises(ValueError):
        oracle_lib.transitions(mdl, grid, N, 2**31, seed=1)
    bad = N.copy()
    bad[0] = 2
    with pytest.raises(ValueError):
        oracle_lib.transitions(mdl, grid, bad, 10, seed=1)
