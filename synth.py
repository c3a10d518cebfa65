"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds none of the method's arithmetic: it only builds input data
of the shapes the paper's workloads have (Sec. 3: M samples, n layers, N_k
points per layer) -- AR(1) coefficients of a standardized Brownian motion,
sorted test grids, contract parameters -- with numpy in FP64, rounded once to
FP32.  Both the GPU library and the oracle consume these arrays; neither
imports the other.

State convention: X_k = W_{t_k} (a d-dimensional Brownian motion with
correlation matrix R), t_k = k T / n.  Then X_{k+1} = X_k + sqrt(dt) C eps
(A = I, b = 0, T_k = sqrt(dt) C with C C^T = R) and X_k ~ sqrt(t_k) C z.
"""
from __future__ import annotations

import numpy as np
from scipy.special import ndtri

SEED_BASE = 0x5EED0000


def corr_matrix(d: int, rho: float) -> np.ndarray:
    R = np.full((d, d), float(rho))
    np.fill_diagonal(R, 1.0)
    return R


def bm_model(d: int, n: int, T: float = 1.0, rho: float = 0.0, x0=None):
    """AR(1) coefficients (A, b, T, mu, L, x0) of the standardized Brownian
    motion sampled at t_k = k T / n, FP32."""
    C = np.linalg.cholesky(corr_matrix(d, rho)) if d > 1 else np.ones((1, 1))
    dt = T / n
    A = np.broadcast_to(np.eye(d), (n, d, d)).astype(np.float32)
    b = np.zeros((n, d), np.float32)
    Tm = np.broadcast_to(np.sqrt(dt) * C, (n, d, d)).astype(np.float32)
    x0v = np.zeros(d) if x0 is None else np.asarray(x0, np.float64).reshape(d)
    mu = np.broadcast_to(x0v, (n + 1, d)).astype(np.float32)
    L = np.stack([np.sqrt(k * dt) * C for k in range(n + 1)]).astype(np.float32)
    return dict(d=d, n=n, A=A, b=b, T=Tm, mu=mu, L=L, x0=x0v.astype(np.float32))


def ou_model(n: int, alpha=(1.0, 5.0), sig=(1.0, 1.0), rho: float = 0.0, T: float = 1.0):
    """Two-factor Ornstein-Uhlenbeck state of the swing-option model (Sec. 3):
    X_{k+1} = diag(e^{-alpha dt}) X_k + T_k eps with the exact Gaussian
    increment covariance; X_0 = 0.  FP32."""
    a = np.asarray(alpha, np.float64)
    s = np.asarray(sig, np.float64)
    dt = T / n
    R = corr_matrix(2, rho)

    def cov(t):
        S = np.zeros((2, 2))
        for i in range(2):
            for j in range(2):
                lam = a[i] + a[j]
                S[i, j] = s[i] * s[j] * R[i, j] * (1.0 - np.exp(-lam * t)) / lam
        return S

    Ad = np.diag(np.exp(-a * dt))
    Tk = np.linalg.cholesky(cov(dt))
    A = np.broadcast_to(Ad, (n, 2, 2)).astype(np.float32)
    b = np.zeros((n, 2), np.float32)
    Tm = np.broadcast_to(Tk, (n, 2, 2)).astype(np.float32)
    mu = np.zeros((n + 1, 2), np.float32)
    L = np.zeros((n + 1, 2, 2))
    for k in range(1, n + 1):
        L[k] = np.linalg.cholesky(cov(k * dt))
    return dict(d=2, n=n, A=A, b=b, T=Tm, mu=mu, L=L.astype(np.float32),
                x0=np.zeros(2, np.float32))


def ou1_model(n: int, alpha: float = 2.0, sig: float = 0.8, theta: float = 0.5,
              x0: float = -0.3, T: float = 1.0):
    """One-factor Ornstein-Uhlenbeck state reverting to theta:
    X_{k+1} = e^{-alpha dt} X_k + theta (1 - e^{-alpha dt}) + T_k eps, with the
    exact Gaussian marginals of X_k from X_0 = x0.  FP32."""
    dt = T / n
    a = np.exp(-alpha * dt)
    sd = lambda t: sig * np.sqrt((1.0 - np.exp(-2.0 * alpha * t)) / (2.0 * alpha))
    t = np.arange(n + 1) * dt
    mu = theta + (x0 - theta) * np.exp(-alpha * t)
    return dict(d=1, n=n, A=np.full((n, 1, 1), a, np.float32),
                b=np.full((n, 1), theta * (1.0 - a), np.float32),
                T=np.full((n, 1, 1), sd(dt), np.float32), mu=mu.reshape(-1, 1).astype(np.float32),
                L=sd(t).reshape(-1, 1, 1).astype(np.float32), x0=np.array([x0], np.float32))


def quantile_grid_1d(N: int) -> np.ndarray:
    """Sorted N(0,1) test grid: quantiles of N(0, 3) (the point density
    f^{1/3} of asymptotically optimal quadratic quantizers), FP64."""
    if N == 1:
        return np.zeros(1)
    u = (np.arange(N) + 0.5) / N
    return np.sqrt(3.0) * ndtri(u)


def layer_grids(model: dict, Ns, base=None, rng=None, jitter: float = 0.0):
    """Concatenated FP32 grid for layers 0..n: layer 0 is {x0}; layer k >= 1
    is x0 + sqrt(t_k) C G_k with G_k a standard-normal test grid of N_k
    points (1-D quantile grid, or the product of two/three 1-D grids).
    Ns: list of per-layer sizes (len n+1, Ns[0] == 1) or per-layer shapes."""
    d, n = model["d"], model["n"]
    L = model["L"].astype(np.float64)
    x0 = model["x0"].astype(np.float64)
    parts = [x0.reshape(1, d)]
    N = [1]
    for k in range(1, n + 1):
        spec = Ns[k]
        if d == 1:
            G = (quantile_grid_1d(int(spec)) if base is None else base(int(spec))).reshape(-1, 1)
        else:
            shape = spec if isinstance(spec, (tuple, list)) else _split(int(spec), d)
            axes = [quantile_grid_1d(int(s)) if base is None else base(int(s)) for s in shape]
            mesh = np.meshgrid(*axes, indexing="ij")
            G = np.stack([m.reshape(-1) for m in mesh], axis=1)
        if jitter > 0.0 and rng is not None:
            G = G + jitter * rng.standard_normal(G.shape)
            if d == 1:
                G = np.sort(G, axis=0)
        # L[k] = sqrt(t_k) C for the Brownian model; the marginal map is generic.
        pts = x0 + G @ L[k].T
        parts.append(pts)
        N.append(pts.shape[0])
    grid = np.concatenate(parts, axis=0).astype(np.float32)
    if d == 1:
        # rounding to FP32 must keep 1-D grids strictly increasing
        off = 0
        for Nk in N:
            g = grid[off:off + Nk, 0]
            assert np.all(np.diff(g) > 0), "1-D test grid not strictly increasing in FP32"
            off += Nk
    return grid, np.asarray(N, np.int32)


def _split(N: int, d: int):
    """Factor N into d near-equal integer sides (product grid shape)."""
    if d == 2:
        a = int(np.floor(np.sqrt(N)))
        while N % a:
            a -= 1
        return (a, N // a)
    a = int(round(N ** (1.0 / 3.0)))
    while N % a:
        a -= 1
    b, c = _split(N // a, 2)
    return (a, b, c)


def seeds(R: int):
    return [SEED_BASE + r for r in range(R)]


def contract_box(rng: np.random.Generator, count: int, d: int = 1):
    """Contract parameters drawn uniformly in the training box of the
    surrogate: S0/K, sigma, r, T, n, rho."""
    return dict(
        s0_over_k=rng.uniform(1 / 1.2, 1 / 0.8, count),
        sigma=rng.uniform(0.1, 0.4, count),
        r=rng.uniform(0.0, 0.1, count),
        T=rng.uniform(0.25, 2.0, count),
        n=rng.integers(10, 101, count),
        rho=(rng.uniform(-0.5, 0.9, count) if d > 1 else np.zeros(count)),
    )


def batch_contracts(count: int, seed: int = 0x5EED0000, n_range=(10, 100),
                    N_range=(50, 2000), M: int = 1_000_000, shrink: float = 1.0):
    """Uneven contracts: per contract d alternating 1 / 2, n uniform in
    n_range, N_max log-uniform in N_range, per-layer sizes
    N_k = round(N_min + (N_max - N_min) sqrt(k/n)) with N_min = max(10, N_max/10)
    (2-D: near-square product shapes).  `shrink` scales n and N down for tests."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(count):
        d = 1 + (c % 2)
        n = max(2, int(round(rng.integers(n_range[0], n_range[1] + 1) * shrink)))
        Nmax = int(round(np.exp(rng.uniform(np.log(N_range[0]), np.log(N_range[1]))) * shrink))
        Nmax = max(Nmax, 4)
        Nmin = max(2, int(round(max(10 * shrink, Nmax / 10))))
        sizes = [1]
        for k in range(1, n + 1):
            Nk = int(round(Nmin + (Nmax - Nmin) * np.sqrt(k / n)))
            if d == 1:
                sizes.append(max(Nk, 1))
            else:
                a = max(1, int(np.floor(np.sqrt(Nk))))
                sizes.append((a, max(1, Nk // a)))
        T = float(rng.uniform(0.25, 2.0))
        rho = float(rng.uniform(-0.5, 0.9)) if d == 2 else 0.0
        out.append(dict(d=d, n=n, sizes=sizes, T=T, rho=rho, M=M,
                        sigma=float(rng.uniform(0.1, 0.4)), K_over_S0=float(rng.uniform(0.8, 1.2)),
                        r=float(rng.uniform(0.0, 0.1))))
    return out


# --------------------------------------------------------------- surrogate

#: Training box of the put surrogate: (S0/K, sigma, r, T, n, rho); rho is
#: fixed at 0 for a one-factor contract.
PUT_BOX_LO = np.array([1 / 1.2, 0.1, 0.0, 0.25, 10.0, 0.0], np.float32)
PUT_BOX_HI = np.array([1 / 0.8, 0.4, 0.1, 2.0, 100.0, 0.0], np.float32)


def mlp_init(seed: int, n_in: int = 6, n_hid: int = 256) -> np.ndarray:
    """Initial FP32 parameters of the 6-256-256-256-1 network, packed
    (W1, b1, W2, b2, W3, b3, w4, b4; rows = output units): weights
    N(0, 1/fan_in), biases 0, head N(0, 1/(4 fan_in))."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((n_in, n_hid), (n_hid, n_hid), (n_hid, n_hid)):
        parts.append(rng.standard_normal((fan_out, fan_in)).ravel() / np.sqrt(fan_in))
        parts.append(np.zeros(fan_out))
    parts.append(rng.standard_normal(n_hid) / np.sqrt(4.0 * n_hid))
    parts.append(np.zeros(1))
    return np.concatenate(parts).astype(np.float32)


def box_queries(count: int, seed: int, lo=PUT_BOX_LO, hi=PUT_BOX_HI, frac_out: float = 0.0):
    """Contract parameters uniform in the box (n integer), FP32 [count][6];
    the last round(frac_out * count) of them leave the box in one random
    coordinate that is not fixed, by 5-50 % of its span, and stay valid
    contracts (above the box, or below it for S0/K and r only)."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    x = lo + rng.random((count, lo.size)) * (hi - lo)
    x[:, 4] = rng.integers(int(lo[4]), int(hi[4]) + 1, count)
    n_out = int(round(frac_out * count))
    free = np.flatnonzero(hi > lo)
    for q in range(count - n_out, count):
        c = int(rng.choice(free))
        step = rng.uniform(0.05, 0.5) * (hi[c] - lo[c])
        below = c in (0, 2) and rng.random() < 0.5
        x[q, c] = lo[c] - step if below else hi[c] + step
        if c == 4:
            x[q, c] = np.ceil(x[q, c])
    return x.astype(np.float32)


# ----------------------------------------------------- samples of other laws

def marginal_samples(d: int, M: int, seed: int, bad: int = 0) -> np.ndarray:
    """Samples of a non-Gaussian marginal, FP32 [M][d]: coordinate 0 a
    log-normal shifted to mean ~0 (skewed, heavy right tail), coordinate 1 a
    two-component Gaussian mixture, coordinate 2 uniform on [-2, 3], with a
    linear mixing so the coordinates correlate; `bad` of them (at seeded
    positions) replaced by inadmissible values (NaN, +-inf, +-100)."""
    rng = np.random.default_rng(seed)
    cols = [np.exp(0.6 * rng.standard_normal(M)) - np.exp(0.18),
            np.where(rng.random(M) < 0.3, rng.normal(-1.5, 0.4, M), rng.normal(0.8, 0.7, M)),
            rng.uniform(-2.0, 3.0, M)]
    x = np.stack(cols[:d], axis=1)
    if d > 1:
        mix = np.tril(np.full((d, d), 0.4)) + 0.6 * np.eye(d)
        x = x @ mix.T
    x = x.astype(np.float32)
    if bad:
        pos = rng.choice(M, size=bad, replace=False)
        vals = np.array([np.nan, np.inf, -np.inf, 100.0, -100.0], np.float32)
        x[pos, rng.integers(0, d, bad)] = vals[rng.integers(0, vals.size, bad)]
    return x


def product_base(d: int, sizes, base) -> np.ndarray:
    """Product of 1-D standard grids base(n) (one per axis), FP32 [prod][d],
    the last axis fastest."""
    axes = [np.asarray(base(int(n)), np.float64) for n in sizes]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.ravel() for m in mesh], axis=1)[:, :d].astype(np.float32)
