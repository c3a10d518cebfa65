"""Pins for the oracle's backward dynamic programming (Sec. 2, quantized BDP)
and payoffs.

Pins: a tree small enough to solve by hand; the identity that a European
claim on a tree whose transition weights are the exact cell probabilities
prices E phi(X^_n) (law of total probability); convergence of that price to
Black-Scholes as N grows; American >= European (exact); the Bermudan put
against a Cox-Ross-Rubinstein tree with the same exercise dates; the
two-asset max-call, whose early-exercise premium vanishes without
dividends, against brute-force quadrature.
"""
import math

import numpy as np
import pytest

import synth
from oracle.quantizer import gauss_quantizer
from tests import _exact


def test_bdp_hand_example(oracle_lib):
    # n = 2, N = [1, 2, 2]
    N = np.array([1, 2, 2], np.int32)
    counts = np.array([3, 1,            # layer 0 -> 1: pi = (3/4, 1/4)
                       2, 2,            # layer 1 row 0: (1/2, 1/2)
                       0, 5], np.int32)  # layer 1 row 1: (0, 1)
    phi = np.array([0.1,      # layer 0
                    0.5, 2.0,  # layer 1
                    1.0, 3.0])  # layer 2
    V0, V, empty = oracle_lib.bdp(counts, N, phi, want_all=True)
    # layer 1: row 0 cont = 0.5*1 + 0.5*3 = 2 -> max(0.5, 2) = 2; row 1 cont = 3 -> 3
    # layer 0: cont = 0.75*2 + 0.25*3 = 2.25 -> max(0.1, 2.25)
    assert np.allclose(V[0], [2.25, 2.0, 3.0, 1.0, 3.0], rtol=0, atol=1e-15)
    assert V0[0] == pytest.approx(2.25, abs=1e-15)
    assert empty == 0
    # an empty source row has continuation value 0 (and is reported)
    counts2 = counts.copy()
    counts2[4:6] = 0
    V0b, Vb, empty_b = oracle_lib.bdp(counts2, N, phi, want_all=True)
    assert Vb[0][2] == 2.0 and empty_b == 1
    assert V0b[0] == pytest.approx(0.75 * 2.0 + 0.25 * 2.0)


def _exact_counts_bm(spec, grid, N, scale=2.0e9):
    """Integer weights proportional to the exact joint cell probabilities."""
    n = spec["n"]
    off = np.concatenate([[0], np.cumsum(N)])
    blocks = []
    for k in range(n):
        g0 = grid[off[k]:off[k + 1], 0]
        g1 = grid[off[k + 1]:off[k + 2], 0]
        P = _exact.transition_probs_1d(g0, g1, float(spec["mu"][k, 0]), float(spec["L"][k, 0, 0]),
                                       1.0, 0.0, float(spec["T"][k, 0, 0]))
        blocks.append(np.rint(P / P.sum() * scale).astype(np.int64).reshape(-1))
    c = np.concatenate(blocks)
    assert c.max() < 2**31
    return c.astype(np.int32)


def _lloyd_grids(spec, Nn):
    base = {}

    def q(N):
        if N not in base:
            base[N] = gauss_quantizer(N)
        return base[N]
    return synth.layer_grids(spec, [1] + [Nn] * spec["n"], base=q)


S0, K, R, SIG, TM = 100.0, 100.0, 0.05, 0.2, 1.0


def test_brownian_scaling_mix_prices_maturity_T_on_the_unit_grid(oracle_lib):
    """The log-price factor y = mix x: with mix = sqrt(T) the tree of the
    unit-time Brownian motion prices maturity T (W_{sT} has the law of
    sqrt(T) W_s), the same as the tree built on the maturity-T grid up to the
    FP32 rounding of the two grids, and both converge to Black-Scholes."""
    n, Nn, T = 4, 200, 1.7
    unit = synth.bm_model(1, n, T=1.0)
    direct = synth.bm_model(1, n, T=T)
    gu, N = _lloyd_grids(unit, Nn)
    gd, _ = _lloyd_grids(direct, Nn)
    kind = oracle_lib.PUT | oracle_lib.EUROPEAN
    v_unit = oracle_lib.bdp(_exact_counts_bm(unit, gu, N), N,
                            oracle_lib.payoff(kind, 1, N, gu, S0, K, R, T, SIG,
                                              mix=[[math.sqrt(T)]]))[0][0]
    v_direct = oracle_lib.bdp(_exact_counts_bm(direct, gd, N), N,
                              oracle_lib.payoff(kind, 1, N, gd, S0, K, R, T, SIG))[0][0]
    assert v_unit == pytest.approx(v_direct, rel=2e-6)
    bs = _exact.black_scholes_put(S0, K, R, SIG, T)
    assert abs(v_unit - bs) < 1e-4 * bs
    # a wrong scale (mix = 1, i.e. maturity 1 paths with maturity-T discounting) is far off
    v_wrong = oracle_lib.bdp(_exact_counts_bm(unit, gu, N), N,
                             oracle_lib.payoff(kind, 1, N, gu, S0, K, R, T, SIG))[0][0]
    assert abs(v_wrong - bs) > 1e-2 * bs


def test_mix_correlates_independent_factors(oracle_lib):
    """2-D: mix = chol(R) on a grid of independent factors gives the payoff
    of the grid C g of correlated factors (pointwise, up to FP32 rounding of
    the correlated grid)."""
    rho = 0.6
    C = np.linalg.cholesky(np.array([[1.0, rho], [rho, 1.0]]))
    indep = synth.bm_model(2, 3)
    g, N = synth.layer_grids(indep, [1, (4, 5), (5, 6), (6, 7)])
    gc = (g.astype(np.float64) @ C.T).astype(np.float32)
    for kind in (oracle_lib.MAX_CALL, oracle_lib.PUT):
        a = oracle_lib.payoff(kind, 2, N, g, S0, K, R, TM, [0.2, 0.3], mix=C)
        b = oracle_lib.payoff(kind, 2, N, gc, S0, K, R, TM, [0.2, 0.3])
        assert np.allclose(a, b, rtol=1e-6, atol=1e-9)
    # the max-call sees the correlation (the put, on factor 0 = x_0, does not)
    a = oracle_lib.payoff(oracle_lib.MAX_CALL, 2, N, g, S0, K, R, TM, [0.2, 0.3], mix=C)
    assert not np.allclose(a, oracle_lib.payoff(oracle_lib.MAX_CALL, 2, N, g, S0, K, R, TM,
                                                [0.2, 0.3]), rtol=1e-3, atol=1e-3)


def test_european_put_exact_tree_is_quantized_expectation_and_converges(oracle_lib):
    n = 4
    spec = synth.bm_model(1, n, T=TM)
    bs = _exact.black_scholes_put(S0, K, R, SIG, TM)
    errs = []
    for Nn in (10, 25, 100, 200):
        grid, N = _lloyd_grids(spec, Nn)
        counts = _exact_counts_bm(spec, grid, N)
        phi = oracle_lib.payoff(oracle_lib.PUT | oracle_lib.EUROPEAN, 1, N, grid, S0, K, R, TM,
                                SIG)
        V0, _, _ = oracle_lib.bdp(counts, N, phi)
        # law of total probability: the forced-Markov chain with exact weights
        # has the exact marginal of X^_n, so V0 = sum_j P(X_n in C_j) phi_n(x_j)
        gn = grid[-Nn:, 0]
        e = _exact.edges_from_grid(gn)
        s = math.sqrt(TM)
        Pn = _exact._mass(e[:-1] / s, e[1:] / s)
        direct = float(np.sum(Pn * phi[-Nn:]))
        # tolerance: the model's sqrt(t_k), sqrt(dt) are FP32, so the chained
        # variance of X_n differs from t_n by ~1e-7 relative; counts are
        # rounded to integers at scale 2e9
        assert V0[0] == pytest.approx(direct, rel=3e-7)
        errs.append(abs(V0[0] - bs))
    # quantization error of E phi(X^) shrinks at least like N^-2 (the kink
    # of the put makes it oscillate between neighbouring N, hence the spread
    # of sizes); at N = 200 it is below 1e-4 of the price
    assert errs[-1] < 1e-4 * bs
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[0] / errs[-1] > (200 / 10) ** 2


def test_monte_carlo_tree_tracks_exact_tree(oracle_lib):
    n, Nn, M = 4, 40, 400_000
    spec = synth.bm_model(1, n, T=TM)
    grid, N = _lloyd_grids(spec, Nn)
    mdl = oracle_lib.Model(spec["d"], spec["n"], spec["A"], spec["b"], spec["T"], spec["mu"],
                           spec["L"], spec["x0"])
    phi_am = oracle_lib.payoff(oracle_lib.PUT, 1, N, grid, S0, K, R, TM, SIG)
    phi_eu = oracle_lib.payoff(oracle_lib.PUT | oracle_lib.EUROPEAN, 1, N, grid, S0, K, R, TM,
                               SIG)
    exact = _exact_counts_bm(spec, grid, N)
    ex_am = oracle_lib.bdp(exact, N, phi_am)[0][0]
    ex_eu = oracle_lib.bdp(exact, N, phi_eu)[0][0]
    am, eu = [], []
    for r in range(6):
        for mode in (0, 1):
            c = oracle_lib.transitions(mdl, grid, N, M, seed=0x5EED0000 + r, mode=mode,
                                       nthreads=4)
            V0, V_am, _ = oracle_lib.bdp(c, N, np.stack([phi_am, phi_eu]), want_all=True)
            am.append(V0[0])
            eu.append(V0[1])
            # American >= European pointwise on every node (exact)
            assert np.all(V_am[0] >= V_am[1] - 1e-12)
    am, eu = np.array(am), np.array(eu)
    for est, ref in ((am, ex_am), (eu, ex_eu)):
        se = est.std(ddof=1) / math.sqrt(est.size)
        assert abs(est.mean() - ref) < 5 * se + 1e-3 * ref


def test_bermudan_put_matches_crr_with_same_exercise_dates(oracle_lib):
    n, Nn = 10, 200
    spec = synth.bm_model(1, n, T=TM)
    grid, N = _lloyd_grids(spec, Nn)
    counts = _exact_counts_bm(spec, grid, N)
    phi = oracle_lib.payoff(oracle_lib.PUT, 1, N, grid, S0, K, R, TM, SIG)
    V0 = oracle_lib.bdp(counts, N, phi)[0][0]
    steps = 20_000
    berm = _exact.crr_put(S0, K, R, SIG, TM, steps, exercise_every=steps // n)
    amer = _exact.crr_put(S0, K, R, SIG, TM, steps)
    euro = _exact.black_scholes_put(S0, K, R, SIG, TM)
    assert euro < berm < amer
    # the tree's error is the quantization error, a few 1e-3 relative at N = 200
    assert abs(V0 - berm) < 5e-3 * berm, (V0, berm, amer, euro)


def test_max_call_american_equals_european(oracle_lib):
    """Two assets, no dividends: the discounted max-call payoff is a
    submartingale, so the American and European prices coincide; both tree
    prices must sit next to brute-force quadrature of the European price."""
    n, M = 6, 400_000
    rho, sig = 0.3, (0.2, 0.3)
    spec = synth.bm_model(2, n, T=TM, rho=rho)
    base = {}

    def q(N):
        if N not in base:
            base[N] = gauss_quantizer(N)
        return base[N]
    grid, N = synth.layer_grids(spec, [1] + [(20, 20)] * n, base=q)
    mdl = oracle_lib.Model(2, n, spec["A"], spec["b"], spec["T"], spec["mu"], spec["L"],
                           spec["x0"])
    c = oracle_lib.transitions(mdl, grid, N, M, seed=0x5EED0042, mode=0, nthreads=6)
    phi_am = oracle_lib.payoff(oracle_lib.MAX_CALL, 2, N, grid, S0, K, R, TM, sig)
    phi_eu = oracle_lib.payoff(oracle_lib.MAX_CALL | oracle_lib.EUROPEAN, 2, N, grid, S0, K,
                               R, TM, sig)
    V0, _, _ = oracle_lib.bdp(c, N, np.stack([phi_am, phi_eu]))
    ref = _exact.max_call_european_quadrature(S0, K, R, sig, rho, TM)
    assert V0[0] >= V0[1]
    assert (V0[0] - V0[1]) < 0.02 * ref
    assert abs(V0[1] - ref) < 0.02 * ref, (V0, ref)
