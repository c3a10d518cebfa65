"""Pins for the surrogate oracle (oracle/mlp.py), on the CPU.

Each pin compares the oracle with something other than itself: torch's own
BF16 conversion, a float64 torch network and its autograd, central finite
differences, torch's Adam, a closed-form special case, and the box edges.
"""
import numpy as np
import pytest

import synth
from oracle import mlp as M

torch = pytest.importorskip("torch")

LO, HI = synth.PUT_BOX_LO, synth.PUT_BOX_HI


def _inputs(B, seed=0):
    return synth.box_queries(B, seed)


def test_bf16_round_matches_torch_conversion():
    rng = np.random.default_rng(0)
    bits = rng.integers(0x00800000, 0x7F000000, 200_000, dtype=np.uint32)
    # include exact ties (low half 0x8000) with even and odd upper halves
    bits[:1000] = (bits[:1000] & 0xFFFF0000) | 0x8000
    f = np.concatenate([bits.view(np.float32), -bits.view(np.float32)])
    ref = torch.from_numpy(f).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(f), ref)
    # two terms carry ~16 significant bits
    h = rng.standard_normal(10_000)
    assert np.max(np.abs(M.split_terms(h, 2) - h) / np.abs(h)) < 2.0 ** -15
    assert np.max(np.abs(M.split_terms(h, 1) - h) / np.abs(h)) <= 2.0 ** -8


def _torch_net(p, x, lo, hi, s):
    """The same network from torch building blocks (float64, no rounding)."""
    P = torch.from_numpy(np.asarray(p, np.float64)).requires_grad_()
    W1 = P[M.OFF_W1:M.OFF_B1].view(256, 6)
    b1 = P[M.OFF_B1:M.OFF_W2]
    W2 = P[M.OFF_W2:M.OFF_B2].view(256, 256)
    b2 = P[M.OFF_B2:M.OFF_W3]
    W3 = P[M.OFF_W3:M.OFF_B3].view(256, 256)
    b3 = P[M.OFF_B3:M.OFF_W4]
    w4 = P[M.OFF_W4:M.OFF_B4]
    b4 = P[M.OFF_B4]
    lo_t = torch.tensor(np.asarray(lo, np.float64))
    hi_t = torch.tensor(np.asarray(hi, np.float64))
    span = hi_t - lo_t
    u = torch.where(span == 0, torch.zeros(()), 2 * (torch.from_numpy(np.asarray(x, np.float64))
                                                       - lo_t) / torch.where(span == 0, 1, span) - 1)
    F = torch.nn.functional
    h = F.silu(F.linear(u, W1, b1))
    h = F.silu(F.linear(h, W2, b2))
    h = F.silu(F.linear(h, W3, b3))
    return s * (h @ w4 + b4), P


def test_forward_and_gradient_match_torch_autograd():
    p = synth.mlp_init(3).astype(np.float64)
    p[M.OFF_B1:M.OFF_W2] = np.linspace(-0.5, 0.5, 256)     # nonzero biases
    x = _inputs(64, 1)
    t = np.random.default_rng(2).uniform(0, 0.3, 64)
    w = np.random.default_rng(3).uniform(0.5, 2.0, 64)
    L, g, y = M.loss_and_grad(p, x, t, w, LO, HI, 0.1, quantize=False)
    yt, P = _torch_net(p, x, LO, HI, 0.1)
    assert np.allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-15)
    Lt = (torch.from_numpy(w) * (yt - torch.from_numpy(t)) ** 2).mean()
    Lt.backward()
    assert L == pytest.approx(Lt.item(), rel=1e-12)
    gt = P.grad.numpy()
    assert np.allclose(g, gt, rtol=1e-9, atol=1e-14 * np.abs(gt).max())


def test_gradient_matches_central_differences():
    p = synth.mlp_init(4).astype(np.float64)
    p[M.OFF_B2:M.OFF_W3] = 0.1
    x = _inputs(16, 5)
    t = np.full(16, 0.05)
    _, g, _ = M.loss_and_grad(p, x, t, None, LO, HI, 0.1, quantize=False)
    rng = np.random.default_rng(6)
    idx = np.concatenate([rng.integers(a, b, 6) for a, b in
                          ((M.OFF_W1, M.OFF_B1), (M.OFF_B1, M.OFF_W2), (M.OFF_W2, M.OFF_B2),
                           (M.OFF_B2, M.OFF_W3), (M.OFF_W3, M.OFF_B3), (M.OFF_B3, M.OFF_W4),
                           (M.OFF_W4, M.OFF_B4))] + [np.array([M.OFF_B4])])
    for i in idx:
        h = 1e-5 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (M.loss_and_grad(pp, x, t, None, LO, HI, 0.1, quantize=False)[0]
              - M.loss_and_grad(pm, x, t, None, LO, HI, 0.1, quantize=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3 * np.abs(g).max()), i


def test_straight_through_gradient_with_rounding():
    """quantize=True: the gradient is the plain one evaluated at the rounded
    weights and activations (torch autograd with identity-gradient rounds)."""
    p = synth.mlp_init(7).astype(np.float64)
    x = _inputs(32, 8)
    t = np.full(32, 0.1)
    for terms in (1, 2):
        L, g, y = M.loss_and_grad(p, x, t, None, LO, HI, 0.1, terms=terms)

        class Round(torch.autograd.Function):
            @staticmethod
            def forward(ctx, a):
                hi = a.to(torch.float32).to(torch.bfloat16).to(torch.float64)
                if terms == 1:
                    return hi
                return hi + (a - hi).to(torch.float32).to(torch.bfloat16).to(torch.float64)

            @staticmethod
            def backward(ctx, gr):
                return gr

        def rw(a):                       # weights: one BF16 term
            return a + (a.to(torch.float32).to(torch.bfloat16).to(torch.float64) - a).detach()
        P = torch.from_numpy(p).requires_grad_()
        u = torch.from_numpy(M.normalise(x, LO, HI))
        F = torch.nn.functional
        W1 = rw(P[M.OFF_W1:M.OFF_B1].view(256, 6))
        W2 = rw(P[M.OFF_W2:M.OFF_B2].view(256, 256))
        W3 = rw(P[M.OFF_W3:M.OFF_B3].view(256, 256))
        w4 = rw(P[M.OFF_W4:M.OFF_B4])
        h = F.silu(F.linear(u, W1, P[M.OFF_B1:M.OFF_W2]))
        h = F.silu(F.linear(Round.apply(h), W2, P[M.OFF_B2:M.OFF_W3]))
        h = F.silu(F.linear(Round.apply(h), W3, P[M.OFF_B3:M.OFF_W4]))
        yt = 0.1 * (h @ w4 + P[M.OFF_B4])
        ((yt - torch.from_numpy(t)) ** 2).mean().backward()
        assert np.allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-15)
        assert np.allclose(g, P.grad.numpy(), rtol=1e-9, atol=1e-13)
        # and the rounding matters: the plain network differs
        y0, _ = M.forward(p, x, LO, HI, 0.1, quantize=False)
        assert np.max(np.abs(y0 - y)) > 1e-7


def test_adam_matches_torch():
    rng = np.random.default_rng(9)
    p = rng.standard_normal(1000)
    P = torch.from_numpy(p.copy()).requires_grad_()
    opt = torch.optim.Adam([P], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for step in range(1, 5):
        g = rng.standard_normal(1000) * 10.0 ** rng.integers(-6, 1, 1000)
        P.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m, v = M.adam(p, m, v, g, step, 3e-3)
        assert np.allclose(p, P.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_constant_network_closed_form():
    """W2 = W3 = 0: h3 = silu(b3) whatever the input, so
    y = s (w4 . silu(b3) + b4) exactly."""
    p = synth.mlp_init(10).astype(np.float64)
    p[M.OFF_W2:M.OFF_B2] = 0.0
    p[M.OFF_W3:M.OFF_B3] = 0.0
    b3 = np.linspace(-3, 3, 256)
    p[M.OFF_B3:M.OFF_W4] = b3
    p[M.OFF_B4] = 0.25
    y, _ = M.forward(p, _inputs(10, 11), LO, HI, 0.5, quantize=False)
    w4 = p[M.OFF_W4:M.OFF_B4]
    assert np.allclose(y, 0.5 * (np.sum(w4 * b3 / (1 + np.exp(-b3))) + 0.25), rtol=1e-14)


def test_black_scholes_baseline():
    """The control variate: the Black-Scholes put per unit strike against the
    test helper's own formula, put-call parity, and its limits."""
    from tests import _exact
    x = synth.box_queries(200, 41)
    b = M.bs_put(x)
    for q in range(0, 200, 23):
        s, sig, r, T = (float(v) for v in x[q, :4])
        assert b[q] == pytest.approx(_exact.black_scholes_put(s, 1.0, r, sig, T), rel=1e-12)
    # put-call parity with the call from the same d1, d2: C - P = S/K - e^{-rT}
    from scipy.special import ndtr
    s, sig, r, T = (x[:, c].astype(np.float64) for c in range(4))
    v = sig * np.sqrt(T)
    d1 = (np.log(s) + (r + 0.5 * sig ** 2) * T) / v
    call = s * ndtr(d1) - np.exp(-r * T) * ndtr(d1 - v)
    assert np.allclose(call - b, s - np.exp(-r * T), atol=1e-14)
    assert np.all(b > 0) and np.all(b >= np.exp(-r * T) - s - 1e-15)
    # the network adds it inside the box only
    p = synth.mlp_init(12).astype(np.float64)
    xb = synth.box_queries(50, 42, frac_out=0.2)
    y0, _ = M.forward(p, xb, LO, HI, 0.1)
    y1, _ = M.forward(p, xb, LO, HI, 0.1, baseline=1)
    inside = M.in_range(xb, LO, HI)
    assert np.allclose((y1 - y0)[inside], M.bs_put(xb[inside]), rtol=1e-12)
    assert np.array_equal(y1[~inside], y0[~inside])


def test_box_edges_and_fixed_slot():
    x = np.tile(LO, (6, 1)).astype(np.float32)
    x[1] = HI
    x[2, 1] = np.nextafter(LO[1], np.float32(0))        # just below sigma_min
    x[3, 3] = np.nextafter(HI[3], np.float32(10))       # just above T_max
    x[4, 5] = 0.01                                       # fixed rho slot moved
    assert M.in_range(x, LO, HI).tolist() == [True, True, False, False, False, True]
    u = M.normalise(x[:2], LO, HI)
    assert np.allclose(u[0, :5], -1.0) and np.allclose(u[1, :5], 1.0)
    assert np.all(u[:, 5] == 0.0)                        # fixed slot feeds 0
