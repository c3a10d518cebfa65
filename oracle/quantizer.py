"""Oracle for the 1-D standard-normal optimal quadratic quantizer.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A grid minimising the quadratic quantization error (Sec. 2, eq. Qerr) is a
fixed point of Lloyd's method I: every point is the conditional mean of
N(0,1) over its own Voronoi cell, here the interval between the midpoints
of its neighbours.  For the standard normal that mean is closed-form,
(phi(a) - phi(b)) / (Phi(b) - Phi(a)).  This module iterates exactly that
map in FP64 until the largest step falls below ``tol``.
"""
from __future__ import annotations

import numpy as np
from scipy.special import ndtr, ndtri


def _pdf(x):
    return np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def _mass(lo, hi):
    """P(lo < Z < hi), taken from the nearer tail so upper cells keep their digits."""
    return np.where(lo > 0, ndtr(-lo) - ndtr(-hi), ndtr(hi) - ndtr(lo))


def cell_masses(x: np.ndarray) -> np.ndarray:
    a = np.concatenate([[-np.inf], 0.5 * (x[1:] + x[:-1]), [np.inf]])
    return _mass(a[:-1], a[1:])


def distortion(x: np.ndarray) -> float:
    """E min_i |Z - x_i|^2 for Z ~ N(0,1), closed form per interval:
    int_a^b (z - x)^2 phi = (1 + x^2) dP - 2x dphi_1 + dphi_2 with
    int z phi = -phi, int z^2 phi = Phi - z phi."""
    a = np.concatenate([[-np.inf], 0.5 * (x[1:] + x[:-1]), [np.inf]])
    lo, hi = a[:-1], a[1:]
    P = _mass(lo, hi)
    m1 = _pdf(lo) - _pdf(hi)                                  # int z phi
    with np.errstate(invalid="ignore"):
        zl = np.where(np.isinf(lo), 0.0, lo * _pdf(lo))
        zh = np.where(np.isinf(hi), 0.0, hi * _pdf(hi))
    m2 = P + zl - zh                                          # int z^2 phi
    return float(np.sum(m2 - 2.0 * x * m1 + x * x * P))


def lloyd_step(x: np.ndarray) -> np.ndarray:
    a = np.concatenate([[-np.inf], 0.5 * (x[1:] + x[:-1]), [np.inf]])
    P = _mass(a[:-1], a[1:])
    return (_pdf(a[:-1]) - _pdf(a[1:])) / P


def gauss_quantizer(N: int, tol: float = 1e-13, max_iter: int = 5_000_000) -> np.ndarray:
    """Lloyd I from the quantiles of N(0, 3) until max |x_new - x| < tol."""
    if N == 1:
        return np.zeros(1)
    x = np.sqrt(3.0) * ndtri((np.arange(N) + 0.5) / N)
    for _ in range(max_iter):
        xn = lloyd_step(x)
        if np.max(np.abs(xn - x)) < tol:
            return xn
        x = xn
    raise RuntimeError("Lloyd iteration did not converge")
