"""Oracle for the pricing surrogate: a 6-256-256-256-1 perceptron that maps
contract parameters to the tree price, trained by Adam on tree solves.

TEST INFRASTRUCTURE ONLY.  Loaded by ``tests/`` and the benchmark's CPU leg,
never by the product package; it shares no code with the GPU library.  Plain
numpy in FP64, one layer at a time, written for reading.

The paper prices one contract per tree solve (Sec. 2: the quantized backward
dynamic programming on the transition weights of Sec. 3 / 4).  The surrogate
learns the map from the contract parameters to that price, so that a query
inside the training box costs one network evaluation instead of a solve;
queries outside the box are sent back to the tree.

Network (parameters packed in one FP32 vector, rows = output units):
    u   = normalise(x):  u_c = 2 (x_c - lo_c) / (hi_c - lo_c) - 1   (0 when hi_c = lo_c)
    z1  = W1 u + b1,            h1 = silu(z1)            W1: [256][6]
    z2  = W2 q(h1) + b2,        h2 = silu(z2)            W2: [256][256]
    z3  = W3 q(h2) + b3,        h3 = silu(z3)            W3: [256][256]
    y   = s (w4 . h3 + b4) + base(x)                     w4: [256], b4: scalar
with silu(z) = z / (1 + e^-z); base(x) = 0, or with baseline = 1 the
Black-Scholes European put per unit strike on the raw inputs (S0/K, sigma,
r, T): e^{-rT} Phi(-d2) - (S0/K) Phi(-d1) (a control variate, inside the
box).  The weight matrices W1, W2, W3, w4 take BF16 values (the FP32 master
copy rounded to nearest even); biases stay FP32.
q(h) is the activation as the matrix cores see it: the sum of `terms` BF16
numbers (hi = bf16(h); with two terms also lo = bf16(h - hi)).  Layer 1 and
the head are not matrix products (6 inputs, 1 output) and use h unrounded.
quantize=False drops every rounding (the plain FP64 network).

Loss L = sum_b w_b (y_b - t_b)^2 / B.  The gradient is the exact gradient of
L with the roundings taken as the identity (straight-through): that is what
the GPU backward computes, up to its own BF16 rounding of the back-propagated
gradients.

Adam (Kingma & Ba 2015): m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID = 6, 256
OFF_W1 = 0
OFF_B1 = OFF_W1 + N_HID * N_IN
OFF_W2 = OFF_B1 + N_HID
OFF_B2 = OFF_W2 + N_HID * N_HID
OFF_W3 = OFF_B2 + N_HID
OFF_B3 = OFF_W3 + N_HID * N_HID
OFF_W4 = OFF_B3 + N_HID
OFF_B4 = OFF_W4 + N_HID
N_PARAMS = OFF_B4 + 1                      # 133 633


def bf16_round(x) -> np.ndarray:
    """Round to FP32, then to the nearest BF16 (ties to even), as FP64."""
    f = np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def split_terms(h: np.ndarray, terms: int) -> np.ndarray:
    """Value of h as `terms` BF16 numbers (hi, then lo = bf16(h - hi))."""
    hi = bf16_round(h)
    if terms == 1:
        return hi
    return hi + bf16_round(h - hi)


def unpack(p: np.ndarray):
    p = np.asarray(p, np.float64)
    W1 = p[OFF_W1:OFF_B1].reshape(N_HID, N_IN)
    b1 = p[OFF_B1:OFF_W2]
    W2 = p[OFF_W2:OFF_B2].reshape(N_HID, N_HID)
    b2 = p[OFF_B2:OFF_W3]
    W3 = p[OFF_W3:OFF_B3].reshape(N_HID, N_HID)
    b3 = p[OFF_B3:OFF_W4]
    w4 = p[OFF_W4:OFF_B4]
    b4 = p[OFF_B4]
    return W1, b1, W2, b2, W3, b3, w4, b4


def pack(W1, b1, W2, b2, W3, b3, w4, b4) -> np.ndarray:
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, np.ravel(W3), b3, w4,
                           np.atleast_1d(b4)]).astype(np.float64)


def normalise(x, lo, hi) -> np.ndarray:
    x = np.asarray(x, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    span = hi - lo
    fixed = span == 0
    u = 2.0 * (x - lo) / np.where(fixed, 1.0, span) - 1.0
    return np.where(fixed, 0.0, u)


def in_range(x, lo, hi) -> np.ndarray:
    """Every parameter inside the closed training box (compared in FP32)."""
    x = np.asarray(x, np.float32)
    return np.all((x >= np.asarray(lo, np.float32)) & (x <= np.asarray(hi, np.float32)), axis=1)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def bs_put(x) -> np.ndarray:
    """Black-Scholes European put per unit strike, rows (S0/K, sigma, r, T, ...)."""
    from scipy.special import ndtr
    x = np.asarray(x, np.float64)
    s, sig, r, T = x[:, 0], x[:, 1], x[:, 2], x[:, 3]
    v = sig * np.sqrt(T)
    d1 = (np.log(s) + (r + 0.5 * sig * sig) * T) / v
    return np.exp(-r * T) * ndtr(-(d1 - v)) - s * ndtr(-d1)


def forward(p, x, lo, hi, out_scale: float, terms: int = 2, quantize: bool = True,
            baseline: int = 0):
    """y [B] and the cache the backward needs."""
    W1, b1, W2, b2, W3, b3, w4, b4 = unpack(p)
    if quantize:
        W1, W2, W3, w4 = (bf16_round(w) for w in (W1, W2, W3, w4))
        q = lambda h: split_terms(h, terms)      # noqa: E731
    else:
        q = lambda h: h                          # noqa: E731
    u = normalise(x, lo, hi)
    z1 = u @ W1.T + b1
    h1 = silu(z1)
    a1 = q(h1)
    z2 = a1 @ W2.T + b2
    h2 = silu(z2)
    a2 = q(h2)
    z3 = a2 @ W3.T + b3
    h3 = silu(z3)
    y = out_scale * (h3 @ w4 + b4)
    if baseline:
        inside = in_range(x, lo, hi)
        y = y + np.where(inside, bs_put(np.where(inside[:, None], x, 1.0)), 0.0)
    cache = dict(u=u, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, h3=h3, W2=W2, W3=W3, w4=w4,
                 out_scale=out_scale)
    return y, cache


def backward(cache, dy) -> np.ndarray:
    """Gradient [N_PARAMS] of sum_b dy_b y_b (straight-through roundings)."""
    c = cache
    dy = np.asarray(dy, np.float64)
    s = c["out_scale"]
    dw4 = s * (c["h3"].T @ dy)
    db4 = s * np.sum(dy)
    dz3 = s * np.outer(dy, c["w4"]) * dsilu(c["z3"])
    dW3 = dz3.T @ c["a2"]
    db3 = dz3.sum(axis=0)
    dz2 = (dz3 @ c["W3"]) * dsilu(c["z2"])
    dW2 = dz2.T @ c["a1"]
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ c["W2"]) * dsilu(c["z1"])
    dW1 = dz1.T @ c["u"]
    db1 = dz1.sum(axis=0)
    return pack(dW1, db1, dW2, db2, dW3, db3, dw4, db4)


def loss_and_grad(p, x, t, w, lo, hi, out_scale: float, terms: int = 2, quantize: bool = True,
                  baseline: int = 0):
    """(L, dL/dp, y) for L = sum_b w_b (y_b - t_b)^2 / B."""
    y, cache = forward(p, x, lo, hi, out_scale, terms, quantize, baseline)
    t = np.asarray(t, np.float64)
    w = np.ones_like(t) if w is None else np.asarray(w, np.float64)
    B = t.size
    r = y - t
    L = float(np.sum(w * r * r) / B)
    g = backward(cache, 2.0 * w * r / B)
    return L, g, y


def adam(p, m, v, g, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step (step counts from 1); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
