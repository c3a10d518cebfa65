"""Pins for the oracle's stratified time-layer estimate (d = 1; not in the
paper: the samples of X_k are drawn cell by cell from the marginal
conditioned on the cell, M per cell or max(1, rint(M p_i)), so row i of the
counts sums to its sample count).

Pins: the normal quantile (AS 241) against scipy's; the FP64 logarithm
against numpy's; the cell-edge probabilities against scipy's normal CDF;
every stratified sample lies in its own cell; the stratum means equal the
truncated-normal means; the counts estimate the exact transition
probabilities obtained by numerical integration; the plain estimator agrees;
proportional allocation lowers the spread of the estimated next-layer
marginal below the plain estimator's at the same budget.
"""
import numpy as np
import pytest
from scipy import integrate
from scipy.stats import norm

import synth


def _model(oracle_lib, n=3, T=1.0):
    spec = synth.bm_model(1, n, T=T)
    mdl = oracle_lib.Model(1, n, spec["A"], spec["b"], spec["T"], spec["mu"], spec["L"],
                           spec["x0"])
    return spec, mdl


def test_quantile_matches_scipy(oracle_lib):
    ps = np.concatenate([np.logspace(-300, -1, 300), np.linspace(0.005, 0.995, 2001),
                         1 - np.logspace(-16, -1, 150)])
    got = np.array([oracle_lib.ppnd16(p) for p in ps])
    ref = norm.ppf(ps)
    assert np.all(np.abs(got - ref) <= 1e-14 * np.maximum(1.0, np.abs(ref)))
    assert oracle_lib.ppnd16(0.5) == 0.0
    assert oracle_lib.ppnd16(0.0) == -np.inf and oracle_lib.ppnd16(1.0) == np.inf
    # symmetry of the central and the tail branches
    for p in (1e-3, 0.07, 0.2, 0.4):
        assert oracle_lib.ppnd16(p) == -oracle_lib.ppnd16(1.0 - p) or \
            abs(oracle_lib.ppnd16(p) + oracle_lib.ppnd16(1.0 - p)) < 1e-12


def test_log_matches_numpy(oracle_lib):
    xs = np.concatenate([np.logspace(-310, 300, 700), np.linspace(0.3, 3.0, 3001), [1.0, 2.0]])
    for x in xs:
        ref = np.log(x)
        got = oracle_lib.ln64(x)
        assert abs(got - ref) <= 4 * np.spacing(abs(ref)) + 1e-300, x


def test_cell_edges_match_the_normal_cdf(oracle_lib):
    g = np.array([-3.1, -1.2, -0.4, 0.0, 0.3, 1.7, 2.2], np.float32)
    e = oracle_lib.strat_edges(g, 0.25, 1.3)
    m = 0.5 * (g[1:] + g[:-1])
    ref = norm.cdf((m.astype(np.float64) - 0.25) / np.float64(np.float32(1.3)))
    assert e[0] == 0.0 and e[-1] == 1.0
    assert np.allclose(e[1:-1], ref, rtol=1e-14, atol=1e-300)
    assert np.all(np.diff(e) > 0)


def test_every_sample_lies_in_its_cell_and_strata_have_the_truncated_means(oracle_lib):
    spec, mdl = _model(oracle_lib)
    grid, N = synth.layer_grids(spec, [1, 9, 11, 13])
    k, Ms = 2, 4000
    off = int(N[:k].sum())
    gk = grid[off:off + N[k], 0]
    e = oracle_lib.strat_edges(gk, spec["mu"][k, 0], spec["L"][k, 0, 0])
    x = np.concatenate([oracle_lib.strat_pairs(mdl, k, e, i, 0, Ms, seed=17)[0]
                        for i in range(N[k])])
    mids = 0.5 * (gk[1:] + gk[:-1])
    cells = np.searchsorted(mids, x, side="left")          # midpoints strictly below
    rows = np.arange(N[k] * Ms) // Ms
    # a sample rounded onto an edge may land in the neighbour: at most a few
    assert np.mean(cells == rows) > 0.999
    Lk = float(spec["L"][k, 0, 0])
    for i in range(N[k]):
        a = -np.inf if i == 0 else (float(mids[i - 1])) / Lk
        b = np.inf if i == N[k] - 1 else (float(mids[i])) / Lk
        p = norm.cdf(b) - norm.cdf(a)
        mean = Lk * (norm.pdf(a) - norm.pdf(b)) / p
        xi = x[rows == i].astype(np.float64)
        assert abs(xi.mean() - mean) < 5 * xi.std() / np.sqrt(Ms) + 1e-9, i


def test_counts_estimate_the_exact_transition_probabilities(oracle_lib):
    spec, mdl = _model(oracle_lib, n=2)
    grid, N = synth.layer_grids(spec, [1, 6, 7])
    Ms = 200_000
    c = oracle_lib.transitions_stratified(mdl, grid, N, Ms, seed=5, alloc=0)
    k = 1
    off0, off1 = 1, 1 + 6
    gk, gk1 = grid[off0:off0 + 6, 0], grid[off1:off1 + 7, 0]
    ck = c[6:].reshape(6, 7)
    assert np.all(ck.sum(axis=1) == Ms)
    assert np.all(c[:6] .sum() == Ms)                      # layer 0: one stratum
    Lk = float(spec["L"][k, 0, 0])
    Tk = float(spec["T"][k, 0, 0])
    mk = np.concatenate([[-np.inf], 0.5 * (gk[1:] + gk[:-1]).astype(np.float64), [np.inf]])
    mk1 = np.concatenate([[-np.inf], 0.5 * (gk1[1:] + gk1[:-1]).astype(np.float64), [np.inf]])
    for i in range(6):
        pi = norm.cdf(mk[i + 1] / Lk) - norm.cdf(mk[i] / Lk)
        for j in range(7):
            f = lambda z: norm.pdf(z) * (norm.cdf((mk1[j + 1] - Lk * z) / Tk)
                                         - norm.cdf((mk1[j] - Lk * z) / Tk))
            exact = integrate.quad(f, mk[i] / Lk, mk[i + 1] / Lk, epsabs=1e-12)[0] / pi
            est = ck[i, j] / Ms
            assert abs(est - exact) <= 5 * np.sqrt(max(exact * (1 - exact), 1e-12) / Ms) + 1e-6


def test_plain_and_stratified_estimators_agree(oracle_lib):
    spec, mdl = _model(oracle_lib, n=3)
    grid, N = synth.layer_grids(spec, [1, 8, 8, 8])
    plain = oracle_lib.transitions(mdl, grid, N, 400_000, seed=3).astype(np.float64)
    strat = oracle_lib.transitions_stratified(mdl, grid, N, 400_000, seed=3,
                                              alloc=1).astype(np.float64)
    off = 8
    for k in (1, 2):
        P = plain[off:off + 64].reshape(8, 8)
        S = strat[off:off + 64].reshape(8, 8)
        pr = P / np.maximum(P.sum(axis=1, keepdims=True), 1)
        sr = S / S.sum(axis=1, keepdims=True)
        rows = P.sum(axis=1) > 2000
        assert np.abs(pr[rows] - sr[rows]).max() < 0.02
        off += 64


def test_proportional_rows_and_lower_spread(oracle_lib):
    spec, mdl = _model(oracle_lib, n=2)
    grid, N = synth.layer_grids(spec, [1, 12, 12])
    k, M = 1, 6000
    gk = grid[1:13, 0]
    e = oracle_lib.strat_edges(gk, spec["mu"][k, 0], spec["L"][k, 0, 0])
    rows = oracle_lib.strat_rows(e, M, 1)
    assert np.all(rows >= 1) and abs(rows.sum() - M) <= N[k]
    assert np.array_equal(rows, np.maximum(1, np.rint(M * np.diff(e)).astype(np.int64)))
    assert np.all(oracle_lib.strat_rows(e, M, 0) == M)
    # estimated probability of the central cells of layer 2: sum_i p_i c_ij / rows_i
    p = np.diff(e)
    est_s, est_p = [], []
    for r in range(12):
        cs = oracle_lib.transitions_stratified(mdl, grid, N, M, seed=100 + r, alloc=1)
        cp = oracle_lib.transitions(mdl, grid, N, M, seed=100 + r)
        S = cs[12:].reshape(12, 12).astype(np.float64)
        P = cp[12:].reshape(12, 12).astype(np.float64)
        assert np.array_equal(S.sum(axis=1), rows)
        est_s.append((p[:, None] * S / S.sum(axis=1, keepdims=True))[:, 5:7].sum())
        est_p.append(P[:, 5:7].sum() / M)
    assert np.std(est_s) < 0.8 * np.std(est_p)
