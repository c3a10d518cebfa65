"""Closed forms and brute-force integrals used to pin the oracle (test helpers).

Nothing here calls the oracle or the GPU library.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ndtr
from scipy.stats import norm

_GL_X, _GL_W = np.polynomial.legendre.leggauss(48)


def _mass(lo, hi):
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    return np.where(lo > 0, ndtr(-lo) - ndtr(-hi), ndtr(hi) - ndtr(lo))


def edges_from_grid(g: np.ndarray) -> np.ndarray:
    """Cell edges of a 1-D grid: the FP32 midpoints (as exact reals), +-inf."""
    g = np.asarray(g, np.float32)
    mids = (np.float32(0.5) * (g[1:] + g[:-1])).astype(np.float64)
    return np.concatenate([[-np.inf], mids, [np.inf]])


def transition_probs_1d(g0, g1, mu, s, A, b, tau, pieces: int = 8) -> np.ndarray:
    """P(X in C_i(g0), Y in C_j(g1)) for X ~ N(mu, s^2), Y = A X + b + tau eps,
    by Gauss-Legendre quadrature over each source cell (inner law exact)."""
    e0 = edges_from_grid(g0)
    e1 = edges_from_grid(g1)
    N0, N1 = len(g0), len(g1)
    P = np.zeros((N0, N1))
    if s == 0.0:
        i = int(np.searchsorted(e0[1:-1], mu, side="left"))
        m = A * mu + b
        P[i] = _mass((e1[:-1] - m) / tau, (e1[1:] - m) / tau)
        return P
    lo_all, hi_all = mu - 10.0 * s, mu + 10.0 * s
    for i in range(N0):
        lo = max(e0[i], lo_all)
        hi = min(e0[i + 1], hi_all)
        if hi <= lo:
            continue
        cuts = np.linspace(lo, hi, pieces + 1)
        for a, c in zip(cuts[:-1], cuts[1:]):
            x = 0.5 * (c - a) * _GL_X + 0.5 * (c + a)
            w = 0.5 * (c - a) * _GL_W * norm.pdf(x, mu, s)
            m = A * x + b
            inner = _mass((e1[None, :-1] - m[:, None]) / tau, (e1[None, 1:] - m[:, None]) / tau)
            P[i] += w @ inner
    return P


def chi2_check(counts: np.ndarray, P: np.ndarray, min_expect: float = 20.0):
    """Pearson chi-square of integer counts against probabilities P (same
    shape); cells with small expectation are pooled.  Returns (stat, dof,
    max |z| over unpooled cells)."""
    c = counts.reshape(-1).astype(np.float64)
    M = c.sum()
    E = M * P.reshape(-1) / P.sum()
    big = E >= min_expect
    stat = np.sum((c[big] - E[big]) ** 2 / E[big])
    dof = int(big.sum()) - 1
    rest_c, rest_e = c[~big].sum(), E[~big].sum()
    if rest_e >= min_expect:
        stat += (rest_c - rest_e) ** 2 / rest_e
        dof += 1
    zmax = float(np.max(np.abs(c[big] - E[big]) / np.sqrt(E[big]))) if big.any() else 0.0
    return stat, dof, zmax


def black_scholes_put(S0, K, r, sigma, T):
    if T <= 0:
        return max(K - S0, 0.0)
    d1 = (math.log(S0 / K) + (r + 0.5 * sigma * sigma) * T) / (sigma * math.sqrt(T))
    d2 = d1 - sigma * math.sqrt(T)
    return K * math.exp(-r * T) * norm.cdf(-d2) - S0 * norm.cdf(-d1)


def crr_put(S0, K, r, sigma, T, steps, exercise_every=None):
    """Cox-Ross-Rubinstein binomial put.  exercise_every=None: American
    (every step); an integer e: Bermudan, exercise allowed every e steps
    (and at maturity); 0: European."""
    dt = T / steps
    u = math.exp(sigma * math.sqrt(dt))
    d = 1.0 / u
    p = (math.exp(r * dt) - d) / (u - d)
    disc = math.exp(-r * dt)
    j = np.arange(steps + 1)
    S = S0 * u ** (steps - j) * d ** j
    V = np.maximum(K - S, 0.0)
    for step in range(steps - 1, -1, -1):
        V = disc * (p * V[:-1] + (1 - p) * V[1:])
        S = S[:-1] * d
        if exercise_every is None or (exercise_every and step % exercise_every == 0):
            V = np.maximum(V, K - S)
    return float(V[0])


def max_call_european_quadrature(S0, K, r, sig, rho, T, nodes: int = 400, width: float = 9.0):
    """E[e^{-rT} (max(S1, S2) - K)^+] for two correlated GBMs by tensor
    Gauss-Legendre quadrature over the standard bivariate normal."""
    x, w = np.polynomial.legendre.leggauss(nodes)
    x = width * x
    w = width * w * norm.pdf(x)
    z1 = x[:, None]
    z2 = rho * x[:, None] + math.sqrt(1 - rho * rho) * x[None, :]
    W = w[:, None] * w[None, :]
    S1 = S0 * np.exp((r - 0.5 * sig[0] ** 2) * T + sig[0] * math.sqrt(T) * z1)
    S2 = S0 * np.exp((r - 0.5 * sig[1] ** 2) * T + sig[1] * math.sqrt(T) * z2)
    pay = np.maximum(np.maximum(S1, S2) - K, 0.0)
    return float(math.exp(-r * T) * np.sum(W * pay))
