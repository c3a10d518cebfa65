"""Pins for the oracle's swing option (Sec. 2, stochastic control with a
bang-bang control) and the forward obstacle of the 2-factor model (Sec. 3).

Pins: a tree solved by hand; one right (Q = (0, 1)) is the American option on
v^+ priced by the (separately pinned) optimal-stopping BDP; free exercise
(Q = (0, n)) and forced exercise (Q = (n, n)) are sums over the tree's
marginal law, obtained by pushing the cell probabilities forward through
the counts; the price is monotone in Qmin and Qmax.  The forward obstacle
equals call - put at r = 0 and has E S_k = S0 under the marginal law.
"""
import numpy as np
import pytest

import synth


def _tree(oracle_lib, n=6, side=(4, 5), M=40_000, seed=3):
    spec = synth.ou_model(n, alpha=(1.0, 5.0), sig=(1.0, 1.0), rho=-0.4)
    grid, N = synth.layer_grids(spec, [1] + [side] * n)
    mdl = oracle_lib.Model(2, n, spec["A"], spec["b"], spec["T"], spec["mu"], spec["L"],
                           spec["x0"])
    counts = oracle_lib.transitions(mdl, grid, N, M, seed=seed, nthreads=8)
    return spec, grid, N, counts


def _marginals(counts, N):
    """Cell probabilities of every layer, pushed forward through pi = c / p."""
    n = N.size - 1
    m = [np.ones(1)]
    off = 0
    for k in range(n):
        c = counts[off:off + N[k] * N[k + 1]].reshape(N[k], N[k + 1]).astype(np.float64)
        off += N[k] * N[k + 1]
        p = c.sum(axis=1)
        pi = np.divide(c, p[:, None], out=np.zeros_like(c), where=p[:, None] > 0)
        m.append(m[-1] @ pi)
    return m


def test_swing_hand_example(oracle_lib):
    # n = 2, N = [1, 2, 2]; layer 0 -> 1: pi = (3/4, 1/4); layer 1 row 0: (1/2, 1/2),
    # row 1: (0, 1).  v_0 = 1, v_1 = (2, -1).  Exactly one right (Q = (1, 1)):
    #   k = 1: c = 0 must exercise now or never reach Qmin=1 -> P_1(i, 0) = v_1(i)
    #          c = 1: no more rights -> P_1(i, 1) = 0
    #   k = 0: x = 1 -> 1 + E P_1(., 1) = 1;  x = 0 -> E P_1(., 0) = 3/4*2 + 1/4*(-1) = 1.25
    N = np.array([1, 2, 2], np.int32)
    counts = np.array([3, 1, 2, 2, 0, 5], np.int32)
    v = np.array([1.0, 2.0, -1.0, 7.0, 7.0])              # layer 2 is not a date
    P0, Pall = oracle_lib.swing(counts, N, v, 1, 1, want_all=True)
    assert P0 == pytest.approx(1.25, abs=1e-15)
    assert np.allclose(Pall[0, 1:3], [2.0, -1.0]) and np.allclose(Pall[1, 1:3], [0.0, 0.0])
    # at most one right (Q = (0, 1)): row 1 may skip -> P_1(1, 0) = 0, so
    # x = 0 gives 3/4*2 + 1/4*0 = 1.5 > 1
    assert oracle_lib.swing(counts, N, v, 0, 1)[0] == pytest.approx(1.5, abs=1e-15)
    # two rights forced (Q = (2, 2)): 1 + 3/4*2 + 1/4*(-1) = 2.25
    assert oracle_lib.swing(counts, N, v, 2, 2)[0] == pytest.approx(2.25, abs=1e-15)


def test_one_right_is_the_american_option(oracle_lib):
    spec, grid, N, counts = _tree(oracle_lib)
    v = oracle_lib.forward_payoff(spec, N, grid, 20.0, 20.0, 0.0, 1.0, [0.7, 1.4])
    n = N.size - 1
    phi = np.maximum(v, 0.0)
    phi[-N[n]:] = 0.0                                      # no date at layer n
    V0, _, _ = oracle_lib.bdp(counts, N, phi)
    assert oracle_lib.swing(counts, N, v, 0, 1)[0] == pytest.approx(V0[0], rel=1e-13)


def test_free_and_forced_exercise_are_marginal_sums(oracle_lib):
    spec, grid, N, counts = _tree(oracle_lib)
    v = oracle_lib.forward_payoff(spec, N, grid, 20.0, 19.0, 0.02, 1.0, [0.7, 1.4])
    n = N.size - 1
    m = _marginals(counts, N)
    off = np.concatenate([[0], np.cumsum(N)])
    free = sum(float(m[k] @ np.maximum(v[off[k]:off[k + 1]], 0.0)) for k in range(n))
    forced = sum(float(m[k] @ v[off[k]:off[k + 1]]) for k in range(n))
    assert oracle_lib.swing(counts, N, v, 0, n)[0] == pytest.approx(free, rel=1e-12)
    assert oracle_lib.swing(counts, N, v, n, n)[0] == pytest.approx(forced, rel=1e-12)
    # a dropped discount or a transposed pi would break one of the two sums
    assert abs(free - forced) > 1e-3


def test_swing_is_monotone_in_the_constraints(oracle_lib):
    spec, grid, N, counts = _tree(oracle_lib)
    v = oracle_lib.forward_payoff(spec, N, grid, 20.0, 20.0, 0.0, 1.0, [0.7, 1.4])
    n = N.size - 1
    prices = {(a, b): oracle_lib.swing(counts, N, v, a, b)[0]
              for a in range(n + 1) for b in range(a, n + 1)}
    for (a, b), p in prices.items():
        if b + 1 <= n:
            assert prices[(a, b + 1)] >= p - 1e-12          # more room: worth more
        if a + 1 <= b:
            assert prices[(a + 1, b)] <= p + 1e-12          # more obligation: worth less


def test_forward_payoff_is_call_minus_put_at_zero_rate(oracle_lib):
    spec = synth.bm_model(1, 5, T=1.3)
    grid, N = synth.layer_grids(spec, [1, 20, 30, 40, 50, 60])
    sig = 0.3
    v = oracle_lib.forward_payoff(spec, N, grid, 100.0, 95.0, 0.0, 1.3, [sig])
    call = oracle_lib.payoff(oracle_lib.MAX_CALL, 1, N, grid, 100.0, 95.0, 0.0, 1.3, sig)
    put = oracle_lib.payoff(oracle_lib.PUT, 1, N, grid, 100.0, 95.0, 0.0, 1.3, sig)
    # the forward takes var_k from the FP32 model factor L_k = sqrt(t_k) (relative
    # rounding ~6e-8), the call and put use sigma^2 t_k in FP64: the error scales
    # with S (~S0), not with S - K
    assert np.allclose(v, call - put, rtol=0, atol=2e-7 * 100.0)
    # the discount: v(r) = e^{-r t_k} (S - K) with the same S (no drift r in S)
    vr = oracle_lib.forward_payoff(spec, N, grid, 100.0, 95.0, 0.05, 1.3, [sig])
    t = np.repeat(1.3 * np.arange(6) / 5, N)
    assert np.allclose(vr, np.exp(-0.05 * t) * v, rtol=1e-12, atol=1e-12)


def test_forward_payoff_is_a_martingale_under_the_marginal_law(oracle_lib):
    """E S_k = S0: the payoff evaluated on samples X_k = mu_k + L_k z (passed
    as the 'grid' of each layer) averages to S0 - K within Monte Carlo error
    (a missing 1/2, a transposed L or a dropped correlation fails)."""
    n, Ms = 4, 400_000
    spec = synth.ou_model(n, alpha=(1.0, 5.0), sig=(1.0, 1.0), rho=-0.6)
    rng = np.random.default_rng(11)
    parts = [spec["x0"].reshape(1, 2).astype(np.float64)]
    for k in range(1, n + 1):
        z = rng.standard_normal((Ms, 2))
        parts.append(spec["mu"][k].astype(np.float64) + z @ spec["L"][k].astype(np.float64).T)
    grid = np.concatenate(parts).astype(np.float32)
    N = np.array([1] + [Ms] * n, np.int32)
    sig = [0.7, 1.4]
    v = oracle_lib.forward_payoff(spec, N, grid, 1.0, 0.0, 0.0, 1.0, sig)
    off = np.concatenate([[0], np.cumsum(N)])
    for k in range(1, n + 1):
        s = v[off[k]:off[k + 1]]
        assert abs(s.mean() - 1.0) < 5 * s.std() / np.sqrt(Ms), k
    # with the correlation dropped from L the mean is off by many standard errors
    L0 = spec["L"].copy()
    L0[:, 1, 0] = 0.0
    wrong = oracle_lib.forward_payoff(dict(spec, L=L0), N, grid, 1.0, 0.0, 0.0, 1.0, sig)
    s = wrong[off[n]:off[n + 1]]
    assert abs(s.mean() - 1.0) > 20 * s.std() / np.sqrt(Ms)
