"""Oracle for the quantization-tree forward step and backward dynamic programming.

TEST INFRASTRUCTURE ONLY.  Loaded by ``tests/``, by the smoke check in
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``; never by the
product package.  It shares no code with the GPU library.

The numerical work lives in ``oracle.c`` (plain C, FP32 with explicit fused
multiply-adds, FP64 for the backward step); this module only loads it with
ctypes and marshals numpy arrays.  The paper is Pages & Wilbertz,
arXiv:1101.3228: Sec. 2 (Voronoi cells, transition weights, quantized BDP),
Sec. 3 (AR(1) proposition, Algorithm I), Sec. 4 (Algorithm III).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

LAYERWISE = 0
PATHWISE = 1


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (IEEE FP32, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-Wall", "-o", _LIB_PATH + ".tmp", _SRC, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Model(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("n", ctypes.c_int32),
                ("A", ctypes.c_void_p), ("b", ctypes.c_void_p), ("T", ctypes.c_void_p),
                ("mu", ctypes.c_void_p), ("L", ctypes.c_void_p), ("x0", ctypes.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.oracle_philox4x32_10.argtypes = [P, P, P]
        L.oracle_ln_u24.argtypes = [ctypes.c_uint32]
        L.oracle_ln_u24.restype = ctypes.c_float
        L.oracle_sincos_2pi_u24.argtypes = [ctypes.c_uint32, P, P]
        L.oracle_box_muller.argtypes = [ctypes.c_uint32, ctypes.c_uint32, P, P]
        L.oracle_layer_pair.argtypes = [P, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_uint32, P, P]
        L.oracle_path_noise.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_uint32, P]
        L.oracle_cell.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P]
        L.oracle_cell.restype = ctypes.c_int32
        L.oracle_transitions.argtypes = [P, P, P, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32,
                                         P, ctypes.c_int32]
        L.oracle_transitions.restype = ctypes.c_int
        L.oracle_bdp.argtypes = [P, P, ctypes.c_int32, P, ctypes.c_int32, P, P]
        L.oracle_bdp.restype = ctypes.c_int64
        L.oracle_payoff.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, P, P, P]
        L.oracle_forward_payoff.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, P,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, P, P, P]
        L.oracle_swing.argtypes = [P, P, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32, P]
        L.oracle_swing.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def ln_u24(K: int) -> float:
    return float(np.float32(lib().oracle_ln_u24(int(K))))


def sincos_2pi_u24(J: int):
    s = np.zeros(1, np.float32)
    c = np.zeros(1, np.float32)
    lib().oracle_sincos_2pi_u24(int(J), _ptr(s), _ptr(c))
    return s[0], c[0]


def box_muller(ra: int, rb: int):
    z0 = np.zeros(1, np.float32)
    z1 = np.zeros(1, np.float32)
    lib().oracle_box_muller(int(ra), int(rb), _ptr(z0), _ptr(z1))
    return z0[0], z1[0]


class Model:
    """Host-side AR(1) model X_{k+1} = A_k X_k + b_k + T_k eps_k with the
    marginal X_k ~ mu_k + L_k z (Proposition, Sec. 3).  FP32 arrays."""

    def __init__(self, d, n, A, b, T, mu, L, x0):
        self.d, self.n = int(d), int(n)
        self.A = np.ascontiguousarray(A, np.float32).reshape(n, d, d)
        self.b = np.ascontiguousarray(b, np.float32).reshape(n, d)
        self.T = np.ascontiguousarray(T, np.float32).reshape(n, d, d)
        self.mu = np.ascontiguousarray(mu, np.float32).reshape(n + 1, d)
        self.L = np.ascontiguousarray(L, np.float32).reshape(n + 1, d, d)
        self.x0 = np.ascontiguousarray(x0, np.float32).reshape(d)
        self._c = _Model(self.d, self.n, self.A.ctypes.data, self.b.ctypes.data,
                         self.T.ctypes.data, self.mu.ctypes.data, self.L.ctypes.data,
                         self.x0.ctypes.data)

    def cptr(self):
        return ctypes.byref(self._c)


def layer_pair(model: Model, k: int, m: int, seed: int, contract: int = 0):
    x = np.zeros(3, np.float32)
    y = np.zeros(3, np.float32)
    lib().oracle_layer_pair(model.cptr(), k, m, seed, contract, _ptr(x), _ptr(y))
    return x[:model.d].copy(), y[:model.d].copy()


def path_noise(d: int, k: int, m: int, seed: int, contract: int = 0):
    e = np.zeros(3, np.float32)
    lib().oracle_path_noise(d, k, m, seed, contract, _ptr(e))
    return e[:d].copy()


def cell(grid_k: np.ndarray, d: int, x) -> int:
    g = np.ascontiguousarray(grid_k, np.float32)
    xv = np.ascontiguousarray(np.atleast_1d(x), np.float32)
    N = g.size // d
    return int(lib().oracle_cell(_ptr(g), N, d, _ptr(xv)))


def count_offsets(N) -> np.ndarray:
    N = np.asarray(N, np.int64)
    return np.concatenate([[0], np.cumsum(N[:-1] * N[1:])])


def point_offsets(N) -> np.ndarray:
    N = np.asarray(N, np.int64)
    return np.concatenate([[0], np.cumsum(N)])


def transitions(model: Model, grid: np.ndarray, N, M: int, seed: int, contract: int = 0,
                mode: int = LAYERWISE, m0: int = 0, nthreads: int = 1) -> np.ndarray:
    """Integer transition counts, layers concatenated (Algorithm I / III)."""
    N = np.ascontiguousarray(N, np.int32)
    g = np.ascontiguousarray(grid, np.float32)
    total = int(count_offsets(N)[-1])
    counts = np.zeros(max(total, 1), np.int32)
    rc = lib().oracle_transitions(model.cptr(), _ptr(g), _ptr(N), m0, M, seed, contract,
                                  mode, _ptr(counts), nthreads)
    if rc != 0:
        raise ValueError(f"oracle_transitions rejected its arguments (code {rc})")
    return counts[:total]


def layer_counts(counts: np.ndarray, N, k: int) -> np.ndarray:
    off = count_offsets(N)
    return counts[off[k]:off[k + 1]].reshape(int(N[k]), int(N[k + 1]))


def bdp(counts: np.ndarray, N, phi: np.ndarray, want_all: bool = False):
    """Backward dynamic programming in FP64; returns (V0[n_pay], V_all or None, empty)."""
    N = np.ascontiguousarray(N, np.int32)
    n = N.size - 1
    P = int(point_offsets(N)[-1])
    phi = np.ascontiguousarray(phi, np.float64).reshape(-1, P)
    n_pay = phi.shape[0]
    c = np.ascontiguousarray(counts, np.int32)
    V0 = np.zeros(n_pay, np.float64)
    V_all = np.zeros((n_pay, P), np.float64) if want_all else None
    empty = lib().oracle_bdp(_ptr(c), _ptr(N), n, _ptr(phi), n_pay,
                             _ptr(V_all) if want_all else None, _ptr(V0))
    return V0, V_all, int(empty)


PUT, MAX_CALL, EUROPEAN = 0, 1, 2


def forward_payoff(model: dict, N, grid: np.ndarray, S0: float, K: float, r: float, T: float,
                   sigma, mix=None) -> np.ndarray:
    """v_k(x) = e^{-r t_k} (S0 exp(sigma . mix (x - mu_k) - var_k / 2) - K) on the grid."""
    d = int(model["d"])
    N = np.ascontiguousarray(N, np.int32)
    n = N.size - 1
    g = np.ascontiguousarray(grid, np.float32)
    mu = np.ascontiguousarray(model["mu"], np.float32)
    L = np.ascontiguousarray(model["L"], np.float32)
    sig = np.ascontiguousarray(np.resize(np.atleast_1d(np.asarray(sigma, np.float64)), d))
    mx = None if mix is None else np.ascontiguousarray(np.asarray(mix, np.float64).reshape(d, d))
    v = np.zeros(int(point_offsets(N)[-1]), np.float64)
    lib().oracle_forward_payoff(d, n, _ptr(N), _ptr(g), _ptr(mu), _ptr(L), S0, K, r, T,
                                _ptr(sig), None if mx is None else _ptr(mx), _ptr(v))
    return v


def swing(counts: np.ndarray, N, v: np.ndarray, Qmin: int, Qmax: int, want_all: bool = False):
    """Swing option by the bang-bang BDP in FP64: (P0, P_all [Qmax+1][points] or None)."""
    N = np.ascontiguousarray(N, np.int32)
    n = N.size - 1
    P = int(point_offsets(N)[-1])
    c = np.ascontiguousarray(counts, np.int32)
    vv = np.ascontiguousarray(v, np.float64)
    P_all = np.zeros((Qmax + 1, P), np.float64) if want_all else None
    P0 = lib().oracle_swing(_ptr(c), _ptr(N), n, _ptr(vv), int(Qmin), int(Qmax),
                            _ptr(P_all) if want_all else None)
    return float(P0), P_all


def payoff(kind: int, d: int, N, grid: np.ndarray, S0: float, K: float, r: float, T: float,
           sigma, mix=None) -> np.ndarray:
    """mix: optional [d][d] map from the grid state to the Brownian factors
    of the log-prices (None: identity)."""
    N = np.ascontiguousarray(N, np.int32)
    n = N.size - 1
    g = np.ascontiguousarray(grid, np.float32)
    sig = np.ascontiguousarray(np.atleast_1d(sigma), np.float64)
    if sig.size < d:
        sig = np.resize(sig, d)
    mx = None if mix is None else np.ascontiguousarray(np.asarray(mix, np.float64).reshape(d, d))
    phi = np.zeros(int(point_offsets(N)[-1]), np.float64)
    lib().oracle_payoff(kind, d, n, _ptr(N), _ptr(g), S0, K, r, T, _ptr(sig),
                        None if mx is None else _ptr(mx), _ptr(phi))
    return phi


def _bulk_setup():
    L = lib()
    if getattr(L, "_bulk", False):
        return L
    P = ctypes.c_void_p
    L.oracle_ln_u24_bulk.argtypes = [ctypes.c_uint32, ctypes.c_int64, P]
    L.oracle_sincos_bulk.argtypes = [ctypes.c_uint32, ctypes.c_int64, P, P]
    L.oracle_box_muller_bulk.argtypes = [P, P, ctypes.c_int64, P, P]
    L.oracle_philox_bulk.argtypes = [P, P, ctypes.c_int64, P]
    L.oracle_layer_pairs_bulk.argtypes = [P, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64,
                                          ctypes.c_uint64, ctypes.c_uint32, P, P]
    L.oracle_pi_estimate.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64]
    L.oracle_pi_estimate.restype = ctypes.c_double
    L._bulk = True
    return L


def ln_u24_bulk(K0: int, count: int) -> np.ndarray:
    out = np.zeros(count, np.float32)
    _bulk_setup().oracle_ln_u24_bulk(K0, count, _ptr(out))
    return out


def sincos_bulk(J0: int, count: int):
    s = np.zeros(count, np.float32)
    c = np.zeros(count, np.float32)
    _bulk_setup().oracle_sincos_bulk(J0, count, _ptr(s), _ptr(c))
    return s, c


def box_muller_bulk(ra: np.ndarray, rb: np.ndarray):
    ra = np.ascontiguousarray(ra, np.uint32)
    rb = np.ascontiguousarray(rb, np.uint32)
    z0 = np.zeros(ra.size, np.float32)
    z1 = np.zeros(ra.size, np.float32)
    _bulk_setup().oracle_box_muller_bulk(_ptr(ra), _ptr(rb), ra.size, _ptr(z0), _ptr(z1))
    return z0, z1


def philox_bulk(ctrs: np.ndarray, key) -> np.ndarray:
    c = np.ascontiguousarray(ctrs, np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros_like(c)
    _bulk_setup().oracle_philox_bulk(_ptr(c), _ptr(k), c.shape[0], _ptr(out))
    return out


def layer_pairs(model: Model, k: int, m0: int, count: int, seed: int, contract: int = 0):
    x = np.zeros((count, model.d), np.float32)
    y = np.zeros((count, model.d), np.float32)
    _bulk_setup().oracle_layer_pairs_bulk(model.cptr(), k, m0, count, seed, contract,
                                          _ptr(x), _ptr(y))
    return x, y


def pi_estimate(seed: int, rep: int, npts: int) -> float:
    return float(_bulk_setup().oracle_pi_estimate(seed, rep, npts))


def layer_counts_one(model: Model, grid: np.ndarray, N, k: int, M: int, seed: int,
                     contract: int = 0, m0: int = 0, nthreads: int = 1) -> np.ndarray:
    """Counts of the single layer k -> k+1 (time-layer parallel estimate)."""
    L = lib()
    if not getattr(L, "_one", False):
        P = ctypes.c_void_p
        L.oracle_layer_counts.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_uint64,
                                          ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                          P, ctypes.c_int32]
        L.oracle_layer_counts.restype = ctypes.c_int
        L._one = True
    N = np.ascontiguousarray(N, np.int32)
    g = np.ascontiguousarray(grid, np.float32)
    if not 0 <= k < N.size - 1:
        raise ValueError(f"layer {k} outside 0..{N.size - 2}")
    out = np.zeros((int(N[k]), int(N[k + 1])), np.int32)
    rc = L.oracle_layer_counts(model.cptr(), _ptr(g), _ptr(N), k, m0, M, seed, contract,
                               _ptr(out), nthreads)
    if rc != 0:
        raise ValueError(f"oracle_layer_counts rejected its arguments (code {rc})")
    return out


def cells_bulk(grid_k: np.ndarray, d: int, x: np.ndarray) -> np.ndarray:
    """Voronoi cells of many points (plain loop in C)."""
    L = lib()
    if not getattr(L, "_cells", False):
        P = ctypes.c_void_p
        L.oracle_cells_bulk.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int64, P]
        L.oracle_cells_bulk.restype = None
        L._cells = True
    g = np.ascontiguousarray(grid_k, np.float32)
    xv = np.ascontiguousarray(x, np.float32).reshape(-1, d)
    out = np.zeros(xv.shape[0], np.int32)
    L.oracle_cells_bulk(_ptr(g), g.size // d, d, _ptr(xv), xv.shape[0], _ptr(out))
    return out


def lloyd(d: int, grid: np.ndarray, L, M: int, iters: int, seed: int, fresh: bool = True):
    """Randomized Lloyd iteration for the quadratic quantization error of
    X = L z (Sec. 2, eq. Qerr).  Returns (grid float32 [N][d], distortion
    float64 [iters])."""
    Lib = lib()
    P = ctypes.c_void_p
    Lib.oracle_lloyd.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_uint64,
                                 ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32, P]
    Lib.oracle_lloyd.restype = ctypes.c_int
    g = np.ascontiguousarray(np.asarray(grid, np.float32).reshape(-1, d)).copy()
    Lm = np.ascontiguousarray(np.asarray(L, np.float32).reshape(d, d))
    dist = np.zeros(max(iters, 1), np.float64)
    rc = Lib.oracle_lloyd(d, g.shape[0], _ptr(Lm), _ptr(g), M, iters, seed, int(bool(fresh)),
                          _ptr(dist))
    if rc != 0:
        raise MemoryError("oracle_lloyd")
    return g, dist[:iters]


def lloyd_samples(d: int, L, seed: int, it: int, count: int, fresh: bool = True) -> np.ndarray:
    """The samples X = L z of one Lloyd iteration (m = 0 .. count-1)."""
    Lib = lib()
    P = ctypes.c_void_p
    Lib.oracle_lloyd_sample.argtypes = [ctypes.c_int32, P, ctypes.c_uint64, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_uint64, P]
    Lib.oracle_lloyd_sample.restype = None
    Lm = np.ascontiguousarray(np.asarray(L, np.float32).reshape(d, d))
    out = np.zeros((count, d), np.float32)
    x = np.zeros(3, np.float32)
    for m in range(count):
        Lib.oracle_lloyd_sample(d, _ptr(Lm), seed, int(bool(fresh)), it, m, _ptr(x))
        out[m] = x[:d]
    return out


def sample_moments(d: int, x: np.ndarray):
    """Exact integer moment sums of the admissible samples (finite, within
    [-64, 64]): returns (count, s1 int64[d], s2 int64[d][d])."""
    Lib = lib()
    P = ctypes.c_void_p
    Lib.oracle_sample_moments.argtypes = [ctypes.c_int32, P, ctypes.c_int64, P, P]
    Lib.oracle_sample_moments.restype = ctypes.c_int64
    xv = np.ascontiguousarray(np.asarray(x, np.float32).reshape(-1, d))
    s1 = np.zeros(d, np.int64)
    s2 = np.zeros((d, d), np.int64)
    cnt = Lib.oracle_sample_moments(d, _ptr(xv), xv.shape[0], _ptr(s1), _ptr(s2))
    return int(cnt), s1, s2


def moment_grid(d: int, x: np.ndarray, base: np.ndarray):
    """Moment-matching grid (Sec. 2): base [N][d] mapped by the sample mean
    and the Cholesky factor of the sample covariance of x [M][d].  Returns
    (grid float32 [N][d], mean [d], cov [d][d], chol [d][d], count)."""
    Lib = lib()
    P = ctypes.c_void_p
    Lib.oracle_moment_map.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, ctypes.c_int32,
                                      P, P]
    Lib.oracle_moment_map.restype = None
    cnt, s1, s2 = sample_moments(d, x)
    b = np.ascontiguousarray(np.asarray(base, np.float32).reshape(-1, d))
    grid = np.zeros_like(b)
    mom = np.zeros(d + 2 * d * d, np.float64)
    Lib.oracle_moment_map(d, cnt, _ptr(s1), _ptr(s2), _ptr(b), b.shape[0], _ptr(grid),
                          _ptr(mom))
    return (grid, mom[:d], mom[d:d + d * d].reshape(d, d), mom[d + d * d:].reshape(d, d), cnt)


def lloyd_empirical(d: int, grid: np.ndarray, x: np.ndarray, batch: int, steps: int,
                    gamma: float = 1.0):
    """Lloyd steps (gamma = 1) or relaxed steps (0 < gamma < 1) of eq. Qerr on
    windows of `batch` samples of x [M][d].  Returns (grid float32 [N][d],
    distortion float64 [steps], rejected samples)."""
    Lib = lib()
    P = ctypes.c_void_p
    Lib.oracle_lloyd_empirical.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_int64,
                                           ctypes.c_int64, ctypes.c_int32, ctypes.c_double, P, P]
    Lib.oracle_lloyd_empirical.restype = ctypes.c_int
    g = np.ascontiguousarray(np.asarray(grid, np.float32).reshape(-1, d)).copy()
    xv = np.ascontiguousarray(np.asarray(x, np.float32).reshape(-1, d))
    dist = np.zeros(max(steps, 1), np.float64)
    rej = np.zeros(1, np.int64)
    rc = Lib.oracle_lloyd_empirical(d, g.shape[0], _ptr(g), _ptr(xv), xv.shape[0], int(batch),
                                    int(steps), float(gamma), _ptr(dist), _ptr(rej))
    if rc != 0:
        raise MemoryError("oracle_lloyd_empirical")
    return g, dist[:steps], int(rej[0])


def _strat_setup():
    Lib = lib()
    if getattr(Lib, "_strat", False):
        return Lib
    P = ctypes.c_void_p
    Lib.oracle_ln64.argtypes = [ctypes.c_double]
    Lib.oracle_ln64.restype = ctypes.c_double
    Lib.oracle_ppnd16.argtypes = [ctypes.c_double]
    Lib.oracle_ppnd16.restype = ctypes.c_double
    Lib.oracle_strat_edges.argtypes = [P, ctypes.c_int32, ctypes.c_float, ctypes.c_float, P]
    Lib.oracle_strat_edges.restype = None
    Lib.oracle_strat_row.argtypes = [P, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32]
    Lib.oracle_strat_row.restype = ctypes.c_int64
    Lib.oracle_strat_pair.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_uint64,
                                      ctypes.c_uint64, ctypes.c_uint32, P, P]
    Lib.oracle_strat_pair.restype = None
    Lib.oracle_transitions_stratified.argtypes = [P, P, P, ctypes.c_uint64, ctypes.c_int32,
                                                  ctypes.c_uint64, ctypes.c_uint32, P]
    Lib.oracle_transitions_stratified.restype = ctypes.c_int
    Lib._strat = True
    return Lib


def ln64(x: float) -> float:
    return float(_strat_setup().oracle_ln64(float(x)))


def ppnd16(p: float) -> float:
    """Standard normal quantile (AS 241)."""
    return float(_strat_setup().oracle_ppnd16(float(p)))


def strat_edges(grid_k: np.ndarray, mu: float, L: float) -> np.ndarray:
    """Marginal probabilities below the cell edges of a 1-D layer [N + 1]."""
    g = np.ascontiguousarray(grid_k, np.float32).ravel()
    e = np.zeros(g.size + 1, np.float64)
    _strat_setup().oracle_strat_edges(_ptr(g), g.size, float(mu), float(L), _ptr(e))
    return e


def strat_rows(edges: np.ndarray, M: int, alloc: int) -> np.ndarray:
    """Samples of every row of a layer (alloc 0 equal, 1 proportional)."""
    Lib = _strat_setup()
    e = np.ascontiguousarray(edges, np.float64)
    return np.array([Lib.oracle_strat_row(_ptr(e), i, M, alloc) for i in range(e.size - 1)],
                    np.int64)


def strat_pairs(model: Model, k: int, edges: np.ndarray, i: int, t0: int, count: int,
                seed: int, contract: int = 0):
    """(X_k, X_{k+1}) of samples t0 .. t0+count-1 of row i of layer k."""
    Lib = _strat_setup()
    e = np.ascontiguousarray(edges, np.float64)
    xs = np.zeros(count, np.float32)
    ys = np.zeros(count, np.float32)
    x = ctypes.c_float()
    y = ctypes.c_float()
    for t in range(count):
        Lib.oracle_strat_pair(model.cptr(), k, _ptr(e), i, t0 + t, seed, contract,
                              ctypes.byref(x), ctypes.byref(y))
        xs[t], ys[t] = x.value, y.value
    return xs, ys


def transitions_stratified(model: Model, grid: np.ndarray, N, M: int, seed: int,
                           contract: int = 0, alloc: int = 1) -> np.ndarray:
    """Stratified counts (d = 1): the samples of X_k are drawn cell by cell
    from the marginal conditioned on the cell, M per cell (alloc 0) or
    max(1, rint(M p_i)) (alloc 1); row i sums to its sample count."""
    N = np.ascontiguousarray(N, np.int32)
    g = np.ascontiguousarray(grid, np.float32)
    total = int(count_offsets(N)[-1])
    counts = np.zeros(max(total, 1), np.int32)
    rc = _strat_setup().oracle_transitions_stratified(model.cptr(), _ptr(g), _ptr(N), M, alloc,
                                                      seed, contract, _ptr(counts))
    if rc != 0:
        raise ValueError(f"oracle_transitions_stratified rejected its arguments (code {rc})")
    return counts[:total]
