"""Python binding of the qtree HIP library (quantization-tree forward step and
backward dynamic programming on MI355X, after Pages & Wilbertz,
arXiv:1101.3228).

Argument marshalling only: every step runs in libqtree.so (HIP kernels for
gfx950 behind the C-ABI declared in include/qtree.h).  torch supplies device
memory and the current stream.  If the library is missing this module raises
on import of the binding -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqtree.so")

LAYERWISE = 0
PATHWISE = 1
PUT, MAX_CALL, EUROPEAN = 0, 1, 2

_STATUS = {0: "ok", 1: "EINVAL", 2: "ENOMEM", 3: "EOVERFLOW", 4: "EDEVICE", 5: "EUNSUPPORTED"}


class QtreeError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"qtree {_STATUS.get(status, status)}: {detail}")
        self.status = status


class _Model(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("n", ctypes.c_int32),
                ("A", ctypes.c_void_p), ("b", ctypes.c_void_p), ("T", ctypes.c_void_p),
                ("mu", ctypes.c_void_p), ("L", ctypes.c_void_p), ("x0", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libqtree.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1101_3228_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, u64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double)
    L.qtree_status_string.argtypes = [ctypes.c_int]
    L.qtree_status_string.restype = ctypes.c_char_p
    L.qtree_last_error.restype = ctypes.c_char_p
    L.qtree_version.restype = ctypes.c_char_p
    L.qtree_workspace_size.argtypes = [i32, i32, P, u64, P]
    L.qtree_plan_create.argtypes = [P, P, P, P, ctypes.c_size_t, P]
    L.qtree_plan_destroy.argtypes = [P]
    L.qtree_plan_destroy.restype = None
    for f in ("qtree_plan_dim", "qtree_plan_layers"):
        getattr(L, f).argtypes = [P]
        getattr(L, f).restype = i32
    for f in ("qtree_plan_count_entries", "qtree_plan_points"):
        getattr(L, f).argtypes = [P]
        getattr(L, f).restype = i64
    L.qtree_transitions.argtypes = [P, u64, u64, u64, u32, ctypes.c_int, P, P]
    L.qtree_transitions_add.argtypes = [P, u64, u64, u64, u32, ctypes.c_int, P, P]
    L.qtree_transitions_fixed_scratch.argtypes = [P, u64, u64, u64, u32, ctypes.c_int, P, P]
    L.qtree_transitions_fixed_scratch.restype = ctypes.c_int
    L.qtree_pi_workspace_size.argtypes = [P, P]
    L.qtree_pi.argtypes = [P, P, P, ctypes.c_size_t, P]
    L.qtree_bdp_many.argtypes = [P, P, ctypes.c_size_t, i64, P, P, P]
    L.qtree_bdp_many_trees.argtypes = [i32, P, P, P, P, P, P, P, ctypes.c_size_t, P]
    L.qtree_bdp_many_trees.restype = ctypes.c_int
    for f in ("qtree_pi_workspace_size", "qtree_pi", "qtree_bdp_many"):
        getattr(L, f).restype = ctypes.c_int
    L.qtree_transitions_add.restype = ctypes.c_int
    L.qtree_bdp.argtypes = [P, P, P, i32, P, P, P]
    L.qtree_payoff.argtypes = [P, i32, f64, f64, f64, f64, P, P, P, P]
    L.qtree_gauss_quantizer.argtypes = [i32, P]
    L.qtree_box_muller.argtypes = [P, P, i64, P, P, P]
    L.qtree_plan_tune.argtypes = [P, i32, i64]
    L.qtree_plan_tune.restype = ctypes.c_int
    L.qtree_plan_trace.argtypes = [P, P]
    L.qtree_plan_trace.restype = ctypes.c_int
    L.qtree_plan_cell_search.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.qtree_plan_cell_search.restype = ctypes.c_int
    L.qtree_plan_batch_samples.argtypes = [P]
    L.qtree_plan_batch_samples.restype = i64
    L.qtree_payoff_batch.argtypes = [P, i32, P, P, P, P, P, P, P, P, P]
    L.qtree_payoff_batch.restype = ctypes.c_int
    L.qtree_payoff_forward.argtypes = [P, f64, f64, f64, f64, P, P, P, P]
    L.qtree_payoff_forward.restype = ctypes.c_int
    L.qtree_swing.argtypes = [P, P, P, i32, i32, P, P, P]
    L.qtree_swing.restype = ctypes.c_int
    L.qtree_pi_quarter_disc.argtypes = [u64, u32, i32, u64, P, P]
    L.qtree_pi_quarter_disc.restype = ctypes.c_int
    L.qtree_lloyd_workspace_size.argtypes = [i32, i32]
    L.qtree_lloyd_workspace_size.restype = ctypes.c_size_t
    L.qtree_lloyd.argtypes = [i32, i32, P, P, P, u64, i32, u64, i32, P, P, ctypes.c_size_t, P]
    L.qtree_lloyd.restype = ctypes.c_int
    L.qtree_lloyd_samples.argtypes = [i32, i32, P, P, P, u64, u64, i32, f64, P, P, P,
                                      ctypes.c_size_t, P]
    L.qtree_lloyd_samples.restype = ctypes.c_int
    L.qtree_sample_moments.argtypes = [i32, P, u64, P, P]
    L.qtree_sample_moments.restype = ctypes.c_int
    L.qtree_moment_grid.argtypes = [i32, P, P, i32, P, P, P]
    L.qtree_moment_grid.restype = ctypes.c_int
    L.qtree_strat_workspace_size.argtypes = [P, u64, i32]
    L.qtree_strat_workspace_size.restype = ctypes.c_size_t
    L.qtree_transitions_stratified.argtypes = [P, u64, i32, u64, u32, P, P, ctypes.c_size_t, P]
    L.qtree_transitions_stratified.restype = ctypes.c_int
    L.qtree_strat_row.argtypes = [P, i32, i32, u64, i32]
    L.qtree_strat_band.argtypes = [P, P, P, P]
    L.qtree_strat_band.restype = ctypes.c_int
    L.qtree_transitions_stratified_banded.argtypes = [P, u64, i32, u64, u32, P, P, P,
                                                      ctypes.c_size_t, P]
    L.qtree_transitions_stratified_banded.restype = ctypes.c_int
    L.qtree_bdp_banded.argtypes = [P, P, P, i32, P, P, P]
    L.qtree_bdp_banded.restype = ctypes.c_int
    L.qtree_strat_row.restype = ctypes.c_int64
    L.qtree_strat_samples.argtypes = [P, i32, i32, u64, i32, u64, i64, u64, u32, P, P, P]
    L.qtree_strat_samples.restype = ctypes.c_int
    L.qtree_layer_samples.argtypes = [P, i32, u64, i64, u64, u32, P, P, P]
    L.qtree_cells.argtypes = [P, i32, P, i64, P, P]
    for f in ("qtree_workspace_size", "qtree_plan_create", "qtree_transitions", "qtree_bdp",
              "qtree_payoff", "qtree_gauss_quantizer", "qtree_box_muller",
              "qtree_layer_samples", "qtree_cells"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise QtreeError(status, lib().qtree_last_error().decode())


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def version() -> str:
    return lib().qtree_version().decode()


def gauss_quantizer(N: int) -> np.ndarray:
    """Stationary (Lloyd) quantizer of N(0,1) with N points, FP64 (host)."""
    out = np.zeros(int(N), np.float64)
    _check(lib().qtree_gauss_quantizer(int(N), _np_ptr(out)))
    return out


def workspace_size(d: int, n: int, N, batch_samples: int = 0) -> int:
    Nn = np.ascontiguousarray(N, np.int32)
    b = ctypes.c_size_t(0)
    _check(lib().qtree_workspace_size(int(d), int(n), _np_ptr(Nn), int(batch_samples),
                                      ctypes.byref(b)))
    return int(b.value)


class Plan:
    """A validated model + grids resident in a device workspace (one
    qtree_plan).  model: dict of FP32 host arrays d, n, A, b, T, mu, L, x0;
    grid: host float32 [sum N_k, d]; N: host int32 [n+1]."""

    def __init__(self, model: dict, grid: np.ndarray, N, device: str = "cuda",
                 batch_samples: int = 0):
        import torch
        self.d, self.n = int(model["d"]), int(model["n"])
        self.N = np.ascontiguousarray(N, np.int32)
        keep = {k: np.ascontiguousarray(model[k], np.float32) for k in
                ("A", "b", "T", "mu", "L", "x0")}
        self._keep = keep
        g = np.ascontiguousarray(grid, np.float32)
        self.grid = g
        cm = _Model(self.d, self.n, *(keep[k].ctypes.data for k in ("A", "b", "T", "mu", "L",
                                                                    "x0")))
        size = workspace_size(self.d, self.n, self.N, batch_samples)
        self.workspace = torch.empty(size, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(lib().qtree_plan_create(ctypes.byref(cm), _np_ptr(g), _np_ptr(self.N),
                                       self.workspace.data_ptr(), size, ctypes.byref(h)))
        self._h = h
        self.entries = int(lib().qtree_plan_count_entries(h))
        self.batch_samples = int(lib().qtree_plan_batch_samples(h))
        self.points = int(lib().qtree_plan_points(h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.qtree_plan_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def tune(self, chunk: int | None = None, xcd_map: int | None = None,
             count: int | None = None, groups: int | None = None,
             nd_samples: int | None = None, tail: int | None = None,
             buckets: int | None = None):
        """Launch tuning (QTREE_TUNE_CHUNK / _XCD_MAP / _COUNT / _GROUPS /
        _ND_SAMPLES / _TAIL / _BUCKETS); results unchanged."""
        if buckets is not None:
            _check(lib().qtree_plan_tune(self._h, 6, int(buckets)))
        if nd_samples is not None:
            _check(lib().qtree_plan_tune(self._h, 4, int(nd_samples)))
        if tail is not None:
            _check(lib().qtree_plan_tune(self._h, 5, int(tail)))
        if chunk is not None:
            _check(lib().qtree_plan_tune(self._h, 0, int(chunk)))
        if xcd_map is not None:
            _check(lib().qtree_plan_tune(self._h, 1, int(xcd_map)))
        if count is not None:
            _check(lib().qtree_plan_tune(self._h, 2, int(count)))
        if groups is not None:
            _check(lib().qtree_plan_tune(self._h, 3, int(groups)))
        return self

    def autotune(self, M: int, seed: int = 1, counts=None, stream=None) -> dict:
        """qtree_plan_autotune: time the candidate forward configurations and
        keep the fastest; returns it with its time."""
        if counts is None:
            counts = self.new_counts()
        ms = ctypes.c_double(0.0)
        L = lib()
        L.qtree_plan_autotune.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.qtree_plan_autotune.restype = ctypes.c_int
        _check(L.qtree_plan_autotune(self._h, int(M), int(seed), counts.data_ptr(),
                                     _stream_handle(stream), ctypes.byref(ms)))
        return {"ms": ms.value, **self.tuning()}

    def tuning(self) -> dict:
        """The plan's launch tuning (groups, tail share, samples per lane,
        d = 2 bucket tables on or off)."""
        L = lib()
        L.qtree_plan_get_tune.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.qtree_plan_get_tune.restype = ctypes.c_int64
        return {"groups": int(L.qtree_plan_get_tune(self._h, 3)),
                "tail": int(L.qtree_plan_get_tune(self._h, 5)),
                "nd_samples": int(L.qtree_plan_get_tune(self._h, 4)),
                "buckets": int(L.qtree_plan_get_tune(self._h, 6))}

    def count_offsets(self) -> np.ndarray:
        N = self.N.astype(np.int64)
        return np.concatenate([[0], np.cumsum(N[:-1] * N[1:])])

    def point_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.N.astype(np.int64))])

    def new_counts(self):
        import torch
        return torch.empty(max(self.entries, 4), dtype=torch.int32, device=self.workspace.device)

    def transitions(self, M: int, seed: int, contract: int = 0, mode: int = LAYERWISE,
                    m0: int = 0, counts=None, stream=None):
        """Transition counts (device int32 [entries]); asynchronous on `stream`."""
        if counts is None:
            counts = self.new_counts()
        _check(lib().qtree_transitions(self._h, int(m0), int(M), int(seed), int(contract),
                                       int(mode), counts.data_ptr(), _stream_handle(stream)))
        return counts[:self.entries]

    def transitions_fixed_scratch(self, M: int, seed: int, contract: int = 0,
                                  mode: int = LAYERWISE, m0: int = 0, counts=None, stream=None):
        """The counts of `transitions`, with the two-pass scratch taken from the
        library's fixed device array (the call allocates nothing; `counts`
        must then be passed in by a caller that cannot allocate)."""
        if counts is None:
            counts = self.new_counts()
        _check(lib().qtree_transitions_fixed_scratch(self._h, int(m0), int(M), int(seed),
                                                     int(contract), int(mode), counts.data_ptr(),
                                                     _stream_handle(stream)))
        return counts[:self.entries]

    def transitions_stratified(self, M: int, seed: int, contract: int = 0, alloc: int = 1,
                               counts=None, stream=None):
        """Stratified counts (d = 1): the samples of X_k are drawn cell by cell
        from the marginal conditioned on the cell, M per cell (alloc 0) or
        max(1, rint(M p_i)) (alloc 1); row i sums to its sample count."""
        import torch
        if counts is None:
            counts = self.new_counts()
        need = lib().qtree_strat_workspace_size(self._h, int(M), int(alloc))
        ws = getattr(self, "_strat_ws", None)
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 16), dtype=torch.uint8, device=self.workspace.device)
            self._strat_ws = ws
        _check(lib().qtree_transitions_stratified(self._h, int(M), int(alloc), int(seed),
                                                  int(contract), counts.data_ptr(),
                                                  ws.data_ptr(), ws.numel(),
                                                  _stream_handle(stream)))
        return counts[:self.entries]

    def strat_band(self):
        """Banded layout of the stratified counts (d = 1): (values, row_off
        int64 [R + 1], row_lo int32 [R]) over the R = sum_{k<n} N_k rows."""
        R = int(np.sum(self.N[:-1]))
        values = ctypes.c_int64(0)
        off = np.zeros(R + 1, np.int64)
        lo = np.zeros(max(R, 1), np.int32)
        _check(lib().qtree_strat_band(self._h, ctypes.byref(values), _np_ptr(off), _np_ptr(lo)))
        return int(values.value), off, lo[:R]

    def transitions_stratified_banded(self, M: int, seed: int, contract: int = 0,
                                      alloc: int = 1, band=None, overflow=None, stream=None):
        """Banded stratified counts: (band device int32 [values], overflow
        device uint32 [1] as int32)."""
        import torch
        dev = self.workspace.device
        values = self.strat_band()[0]
        if band is None:
            band = torch.empty(max(values, 1), dtype=torch.int32, device=dev)
        if overflow is None:
            overflow = torch.empty(1, dtype=torch.int32, device=dev)
        need = lib().qtree_strat_workspace_size(self._h, int(M), int(alloc))
        ws = getattr(self, "_strat_ws", None)
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 16), dtype=torch.uint8, device=dev)
            self._strat_ws = ws
        _check(lib().qtree_transitions_stratified_banded(
            self._h, int(M), int(alloc), int(seed), int(contract), band.data_ptr(),
            overflow.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream)))
        return band[:values], overflow

    def bdp_banded(self, band, phi, V=None, want_v0: bool = True, stream=None):
        """qtree_bdp on banded counts; as `bdp`."""
        import torch
        phi2 = phi.reshape(-1, self.points)
        n_pay = phi2.shape[0]
        if V is None:
            V = torch.empty((n_pay, self.points), dtype=torch.float64, device=phi.device)
        V0 = np.zeros(n_pay, np.float64) if want_v0 else None
        _check(lib().qtree_bdp_banded(self._h, band.data_ptr(), phi2.data_ptr(), n_pay,
                                      V.data_ptr(), _np_ptr(V0) if want_v0 else None,
                                      _stream_handle(stream)))
        return V0, V

    def strat_row(self, k: int, i: int, M: int, alloc: int = 1) -> int:
        """Samples of row i of layer k in the stratified counts."""
        return int(lib().qtree_strat_row(self._h, int(k), int(i), int(M), int(alloc)))

    def transitions_add(self, counts, M: int, seed: int, contract: int = 0,
                        mode: int = LAYERWISE, m0: int = 0, stream=None):
        """Add the counts of samples m0..m0+M-1 onto `counts`; asynchronous."""
        _check(lib().qtree_transitions_add(self._h, int(m0), int(M), int(seed), int(contract),
                                           int(mode), counts.data_ptr(), _stream_handle(stream)))
        return counts

    def buckets(self, k: int):
        """(lo float32[2], scale float32[2], B int32[2]) of layer k's d = 2
        bucket tables (B = 0: none)."""
        lo = np.zeros(2, np.float32)
        sc = np.zeros(2, np.float32)
        B = np.zeros(2, np.int32)
        L = lib()
        L.qtree_plan_buckets.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]
        L.qtree_plan_buckets.restype = ctypes.c_int
        _check(L.qtree_plan_buckets(self._h, int(k), _np_ptr(lo), _np_ptr(sc), _np_ptr(B)))
        return lo, sc, B

    def bucket_counts(self, k: int) -> np.ndarray:
        """Candidate counts of layer k's buckets, uint16 [B0, B1] (empty when
        the layer has no tables; 0xFFFF: a full bucket)."""
        lo, sc, B = self.buckets(k)
        out = np.zeros((int(B[0]), int(B[1])), np.uint16)
        if B[0] == 0:
            return out
        L = lib()
        L.qtree_plan_bucket_counts.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
        L.qtree_plan_bucket_counts.restype = ctypes.c_int
        _check(L.qtree_plan_bucket_counts(self._h, int(k), _np_ptr(out)))
        return out

    def cell_search(self):
        """(guide K, guide buckets) of the 1-D cell search; (-1, 0): the
        breadth-first binary search (and every d >= 2 plan)."""
        k, b = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().qtree_plan_cell_search(self._h, ctypes.byref(k), ctypes.byref(b)))
        return int(k.value), int(b.value)

    def trace(self, event=None):
        """Record `event` (torch.cuda.Event) after each sampling pass."""
        if event is not None and event.cuda_event == 0:
            event.record()  # create the underlying hipEvent_t
        _check(lib().qtree_plan_trace(self._h, event.cuda_event if event is not None else None))
        return self

    def payoff_batch(self, kinds, S0, K, r, T, sigma, mix=None, out=None, stream=None):
        """Obstacles of n contracts in one launch: device float64 [n, points].
        sigma: [n, d] (or broadcastable); mix: optional [n, d, d] map from the
        grid state to the log-price factors (None: identity)."""
        import torch
        kinds = np.ascontiguousarray(np.atleast_1d(kinds), np.int32)
        n = kinds.size
        arr = [np.ascontiguousarray(np.broadcast_to(np.asarray(v, np.float64), (n,)))
               for v in (S0, K, r, T)]
        sig = np.asarray(sigma, np.float64).reshape(n, -1)
        sig = np.ascontiguousarray(np.broadcast_to(sig[:, :self.d] if sig.shape[1] >= self.d
                                                   else sig, (n, self.d)), np.float64)
        mx = None
        if mix is not None:
            mx = np.ascontiguousarray(np.broadcast_to(
                np.asarray(mix, np.float64).reshape(-1, self.d, self.d), (n, self.d, self.d)))
        if out is None:
            out = torch.empty((n, self.points), dtype=torch.float64, device=self.workspace.device)
        _check(lib().qtree_payoff_batch(self._h, n, _np_ptr(kinds), *(_np_ptr(v) for v in arr),
                                        _np_ptr(sig), None if mx is None else _np_ptr(mx),
                                        out.data_ptr(), _stream_handle(stream)))
        return out

    def payoff(self, kind: int, S0: float, K: float, r: float, T: float, sigma, mix=None,
               out=None, stream=None):
        """Discounted obstacle phi on the grid points (device float64 [points])."""
        import torch
        sig = np.ascontiguousarray(np.resize(np.atleast_1d(np.asarray(sigma, np.float64)),
                                             self.d), np.float64)
        mx = None if mix is None else np.ascontiguousarray(
            np.asarray(mix, np.float64).reshape(self.d, self.d))
        if out is None:
            out = torch.empty(self.points, dtype=torch.float64, device=self.workspace.device)
        _check(lib().qtree_payoff(self._h, int(kind), float(S0), float(K), float(r), float(T),
                                  _np_ptr(sig), None if mx is None else _np_ptr(mx),
                                  out.data_ptr(), _stream_handle(stream)))
        return out

    def payoff_forward(self, S0: float, K: float, r: float, T: float, sigma, mix=None,
                       out=None, stream=None):
        """Forward on the sum of the factors, e^{-r t_k}(S_k - K), on the grid
        points (device float64 [points])."""
        import torch
        sig = np.ascontiguousarray(np.resize(np.atleast_1d(np.asarray(sigma, np.float64)),
                                             self.d), np.float64)
        mx = None if mix is None else np.ascontiguousarray(
            np.asarray(mix, np.float64).reshape(self.d, self.d))
        if out is None:
            out = torch.empty(self.points, dtype=torch.float64, device=self.workspace.device)
        _check(lib().qtree_payoff_forward(self._h, float(S0), float(K), float(r), float(T),
                                          _np_ptr(sig), None if mx is None else _np_ptr(mx),
                                          out.data_ptr(), _stream_handle(stream)))
        return out

    def swing(self, counts, v, Qmin: int, Qmax: int, P=None, want_p0: bool = True,
              stream=None):
        """Swing option (bang-bang BDP over the consumed volume): returns
        (P0 or None, P device float64 [points, Qmax + 1])."""
        import torch
        if P is None:
            P = torch.empty((self.points, int(Qmax) + 1), dtype=torch.float64,
                            device=v.device)
        p0 = np.zeros(1, np.float64)
        _check(lib().qtree_swing(self._h, counts.data_ptr(), v.data_ptr(), int(Qmin), int(Qmax),
                                 P.data_ptr(), _np_ptr(p0) if want_p0 else None,
                                 _stream_handle(stream)))
        return (float(p0[0]) if want_p0 else None), P

    def pi(self, counts, out=None, stream=None):
        """Transition weights pi = c / p of the counts (device workspace of
        qtree_pi, uint8), for bdp_many."""
        import torch
        b = ctypes.c_size_t(0)
        _check(lib().qtree_pi_workspace_size(self._h, ctypes.byref(b)))
        if out is None:
            out = torch.empty(b.value + 256, dtype=torch.uint8, device=counts.device)
        base = (out.data_ptr() + 255) // 256 * 256
        _check(lib().qtree_pi(self._h, counts.data_ptr(), base, b.value,
                              _stream_handle(stream)))
        out._qtree_pi = (base, b.value)
        return out

    def bdp_many(self, pi, specs, V0=None, stream=None):
        """V_0 of many contracts on one tree (qtree_bdp_many).  pi: from
        Plan.pi; specs: device uint8 tensor of qtree_payoff_spec records (or a
        host PAYOFF_SPEC array, copied over); returns device float64 [n]."""
        import torch
        if isinstance(specs, np.ndarray):
            specs = torch.from_numpy(specs.view(np.uint8).reshape(-1)).to(pi.device)
        nq = specs.numel() // PAYOFF_SPEC.itemsize
        if V0 is None:
            V0 = torch.empty(nq, dtype=torch.float64, device=pi.device)
        base, size = pi._qtree_pi
        _check(lib().qtree_bdp_many(self._h, base, size, nq, specs.data_ptr(), V0.data_ptr(),
                                    _stream_handle(stream)))
        return V0

    def bdp(self, counts, phi, V=None, want_v0: bool = True, stream=None):
        """Backward dynamic programming (FP64).  phi: device float64
        [n_pay, points] (or [points]).  Returns (V0 numpy [n_pay] or None, V)."""
        import torch
        phi2 = phi.reshape(-1, self.points)
        n_pay = phi2.shape[0]
        if V is None:
            V = torch.empty((n_pay, self.points), dtype=torch.float64, device=phi.device)
        V0 = np.zeros(n_pay, np.float64) if want_v0 else None
        _check(lib().qtree_bdp(self._h, counts.data_ptr(), phi2.data_ptr(), n_pay, V.data_ptr(),
                               _np_ptr(V0) if want_v0 else None, _stream_handle(stream)))
        return V0, V


#: Host image of qtree_payoff_spec (one contract's obstacle parameters).
PAYOFF_SPEC = np.dtype([("S0", "<f8"), ("K", "<f8"), ("r", "<f8"), ("Tm", "<f8"),
                        ("sigma", "<f8", (3,)), ("mix", "<f8", (9,)), ("kind", "<i4"),
                        ("has_mix", "<i4")])


def payoff_specs(d: int, kinds, S0, K, r, T, sigma, mix=None) -> np.ndarray:
    """Pack contract parameters into qtree_payoff_spec records (host):
    sigma [n, d] (broadcastable), mix [n, d, d] or None (identity)."""
    kinds = np.atleast_1d(np.asarray(kinds, np.int32))
    n = kinds.size
    out = np.zeros(n, PAYOFF_SPEC)
    out["kind"] = kinds
    for f, v in (("S0", S0), ("K", K), ("r", r), ("Tm", T)):
        out[f] = np.broadcast_to(np.asarray(v, np.float64), (n,))
    out["sigma"][:, :d] = np.broadcast_to(np.asarray(sigma, np.float64).reshape(-1, d), (n, d))
    if mix is not None:
        m = np.broadcast_to(np.asarray(mix, np.float64).reshape(-1, d * d), (n, d * d))
        out["mix"][:, :d * d] = m
        out["has_mix"] = 1
    return out


def box_muller(ra, rb, stream=None):
    """Diagnostic: Box-Muller of device uint32 word pairs (torch int32 views)."""
    import torch
    z0 = torch.empty(ra.numel(), dtype=torch.float32, device=ra.device)
    z1 = torch.empty_like(z0)
    _check(lib().qtree_box_muller(ra.data_ptr(), rb.data_ptr(), ra.numel(), z0.data_ptr(),
                                  z1.data_ptr(), _stream_handle(stream)))
    return z0, z1


def pi_quarter_disc(seed: int, rep0: int, reps: int, npts: int, inside=None, stream=None):
    """Quarter-disc counts of `reps` repetitions of npts Philox points
    (device uint64 tensor [reps], as int64)."""
    import torch
    if inside is None:
        inside = torch.zeros(reps, dtype=torch.int64, device="cuda")
    _check(lib().qtree_pi_quarter_disc(int(seed), int(rep0), int(reps), int(npts),
                                       inside.data_ptr(), _stream_handle(stream)))
    return inside


def lloyd(d: int, grid0, L, M: int, steps: int, seed: int, fresh: bool = True, grid=None,
          distortion=None, workspace=None, device="cuda", stream=None):
    """Grid optimization (Sec. 2, eq. Qerr): `steps` randomized Lloyd steps of
    M samples of X = L z from the host start grid grid0 [N][d].  Returns
    (grid, distortion): device float32 [N, d] and float64 [steps]."""
    import torch
    g0 = np.ascontiguousarray(np.asarray(grid0, np.float32).reshape(-1, d))
    Lm = np.ascontiguousarray(np.asarray(L, np.float32).reshape(d, d))
    N = g0.shape[0]
    if grid is None:
        grid = torch.empty((N, d), dtype=torch.float32, device=device)
    if distortion is None:
        distortion = torch.zeros(max(steps, 1), dtype=torch.float64, device=grid.device)
    ws_bytes = lib().qtree_lloyd_workspace_size(int(d), int(N))
    if workspace is None:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=grid.device)
    _check(lib().qtree_lloyd(int(d), int(N), _np_ptr(Lm), _np_ptr(g0), grid.data_ptr(), int(M),
                             int(steps), int(seed), int(bool(fresh)), distortion.data_ptr(),
                             workspace.data_ptr(), workspace.numel(), _stream_handle(stream)))
    return grid, distortion


def bdp_many_trees(trees, specs, q_begin, V0=None, workspace=None, stream=None):
    """V_0 of many contracts on many trees in one launch (qtree_bdp_many_trees).
    trees: [(plan, pi)] with pi from Plan.pi; specs: device uint8 tensor of
    qtree_payoff_spec records, tree t pricing records q_begin[t] ..
    q_begin[t+1] - 1; returns device float64 [q_begin[-1]]."""
    import torch
    T = len(trees)
    qb = np.ascontiguousarray(q_begin, np.int64)
    assert qb.size == T + 1
    dev = specs.device
    if V0 is None:
        V0 = torch.empty(max(int(qb[-1]), 1), dtype=torch.float64, device=dev)
    if workspace is None:
        workspace = torch.empty(max(80 * T, 16), dtype=torch.uint8, device=dev)
    plans = (ctypes.c_void_p * max(T, 1))(*[p.handle.value for p, _ in trees])
    pis = (ctypes.c_void_p * max(T, 1))(*[pi._qtree_pi[0] for _, pi in trees])
    sizes = (ctypes.c_size_t * max(T, 1))(*[pi._qtree_pi[1] for _, pi in trees])
    _check(lib().qtree_bdp_many_trees(T, plans, pis, sizes, _np_ptr(qb), specs.data_ptr(),
                                      V0.data_ptr(), workspace.data_ptr(), workspace.numel(),
                                      _stream_handle(stream)))
    return V0


def lloyd_samples(grid0, x, batch: int, steps: int, gamma: float = 1.0, grid=None,
                  distortion=None, rejected=None, workspace=None, stream=None):
    """Lloyd steps (gamma = 1) or relaxed steps (0 < gamma < 1) of eq. Qerr on
    windows of `batch` samples of the device set x [M, d] (float32), from the
    host start grid grid0 [N][d].  Returns (grid [N, d] float32, distortion
    [steps] float64, rejected [1] int64), all on x's device."""
    import torch
    d = int(x.shape[1])
    g0 = np.ascontiguousarray(np.asarray(grid0, np.float32).reshape(-1, d))
    N = g0.shape[0]
    dev = x.device
    if grid is None:
        grid = torch.empty((N, d), dtype=torch.float32, device=dev)
    if distortion is None:
        distortion = torch.zeros(max(steps, 1), dtype=torch.float64, device=dev)
    if rejected is None:
        rejected = torch.zeros(1, dtype=torch.int64, device=dev)
    ws_bytes = lib().qtree_lloyd_workspace_size(d, int(N))
    if workspace is None:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    _check(lib().qtree_lloyd_samples(d, int(N), _np_ptr(g0), grid.data_ptr(), x.data_ptr(),
                                     int(x.shape[0]), int(batch), int(steps), float(gamma),
                                     distortion.data_ptr(), rejected.data_ptr(),
                                     workspace.data_ptr(), workspace.numel(),
                                     _stream_handle(stream)))
    return grid, distortion, rejected


def sample_moments(x, sums=None, stream=None):
    """Exact integer moment sums of the admissible samples of the device set
    x [M, d]: device int64 [1 + d + d d] = (count, s1, s2)."""
    import torch
    d = int(x.shape[1])
    if sums is None:
        sums = torch.empty(1 + d + d * d, dtype=torch.int64, device=x.device)
    _check(lib().qtree_sample_moments(d, x.data_ptr(), int(x.shape[0]), sums.data_ptr(),
                                      _stream_handle(stream)))
    return sums


def moment_grid(x, base, stream=None):
    """Moment-matching grid (Sec. 2): the device base grid [N, d] mapped by the
    sample mean and the Cholesky factor of the sample covariance of the device
    set x [M, d].  Returns (grid [N, d] float32, moments [d + 2 d d] float64:
    mean, covariance, factor)."""
    import torch
    d = int(x.shape[1])
    sums = sample_moments(x, stream=stream)
    grid = torch.empty_like(base)
    mom = torch.empty(d + 2 * d * d, dtype=torch.float64, device=x.device)
    _check(lib().qtree_moment_grid(d, sums.data_ptr(), base.data_ptr(), int(base.shape[0]),
                                   grid.data_ptr(), mom.data_ptr(), _stream_handle(stream)))
    return grid, mom


def layer_samples(plan: Plan, k: int, m0: int, count: int, seed: int, contract: int = 0,
                  stream=None):
    """Diagnostic: (X_k, X_{k+1}) of LAYERWISE samples m0..m0+count-1."""
    import torch
    dev = plan.workspace.device
    x = torch.empty((max(count, 1), plan.d), dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    _check(lib().qtree_layer_samples(plan.handle, int(k), int(m0), int(count), int(seed),
                                     int(contract), x.data_ptr(), y.data_ptr(),
                                     _stream_handle(stream)))
    return x[:count], y[:count]


def strat_samples(plan: Plan, k: int, i: int, M: int, alloc: int, t0: int, count: int,
                  seed: int, contract: int = 0, stream=None):
    """Diagnostic: (X_k, X_{k+1}) of samples t0..t0+count-1 of row i of
    layer k in the stratified counts."""
    import torch
    dev = plan.workspace.device
    x = torch.empty(max(count, 1), dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    _check(lib().qtree_strat_samples(plan.handle, int(k), int(i), int(M), int(alloc), int(t0),
                                     int(count), int(seed), int(contract), x.data_ptr(),
                                     y.data_ptr(), _stream_handle(stream)))
    return x[:count], y[:count]


def cells(plan: Plan, k: int, x, stream=None):
    """Diagnostic: Voronoi cell in layer k of device points x [count, d]."""
    import torch
    x = x.contiguous()
    count = x.shape[0]
    out = torch.empty(max(count, 1), dtype=torch.int32, device=x.device)
    _check(lib().qtree_cells(plan.handle, int(k), x.data_ptr(), int(count), out.data_ptr(),
                             _stream_handle(stream)))
    return out[:count]


class _Contract(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("M", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("contract_id", ctypes.c_uint32), ("counts", ctypes.c_void_p),
                ("phi", ctypes.c_void_p), ("n_pay", ctypes.c_int32), ("V", ctypes.c_void_p)]


def _batch_setup():
    L = lib()
    if getattr(L, "_batch", False):
        return L
    P = ctypes.c_void_p
    L.qtree_tuner_create.argtypes = [ctypes.c_char_p, P]
    L.qtree_tuner_create.restype = ctypes.c_int
    L.qtree_tuner_destroy.argtypes = [P]
    L.qtree_tuner_destroy.restype = None
    L.qtree_tuner_lookup.argtypes = [P, ctypes.c_char_p]
    L.qtree_tuner_lookup.restype = ctypes.c_int32
    L.qtree_batch_plan.argtypes = [P, ctypes.c_int32, P, ctypes.c_size_t, ctypes.c_uint32, P]
    L.qtree_batch_plan.restype = ctypes.c_int
    L.qtree_batch_run.argtypes = [P, P, P]
    L.qtree_batch_run.restype = ctypes.c_int
    L.qtree_batch_info.argtypes = [P, P, P, P, P, P]
    L.qtree_batch_info.restype = ctypes.c_int
    L.qtree_batch_tuning.argtypes = [P, P, P, P]
    L.qtree_batch_tuning.restype = ctypes.c_int
    L.qtree_batch_set_config.argtypes = [P, ctypes.c_int32]
    L.qtree_batch_set_config.restype = ctypes.c_int
    L.qtree_batch_signature.argtypes = [P]
    L.qtree_batch_signature.restype = ctypes.c_char_p
    L.qtree_batch_destroy.argtypes = [P]
    L.qtree_batch_destroy.restype = None
    L._batch = True
    return L


class Tuner:
    """Autotuner handle with an optional text cache file."""

    def __init__(self, cache_path: str | None = None):
        h = ctypes.c_void_p()
        _check(_batch_setup().qtree_tuner_create(cache_path.encode() if cache_path else None,
                                                 ctypes.byref(h)))
        self._h = h

    def lookup(self, signature: str) -> int:
        return int(_batch_setup().qtree_tuner_lookup(self._h, signature.encode()))

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._h.value and _lib is not None:
            _lib.qtree_tuner_destroy(self._h)
            self._h = None


class Batch:
    """Many contracts priced together (sampling launches, histogram
    launch, one BDP launch; optional hipGraph replay).  items: list of dicts
    with plan, M, seed, contract_id, counts, phi [n_pay, points], V."""

    def __init__(self, items, tuner: Tuner | None = None, scratch_bytes: int = 0,
                 graph: bool = False):
        L = _batch_setup()
        self.items = items
        arr = (_Contract * len(items))()
        for i, it in enumerate(items):
            plan = it["plan"]
            phi = it["phi"].reshape(-1, plan.points)
            arr[i] = _Contract(plan.handle.value, int(it["M"]), int(it["seed"]),
                               int(it.get("contract_id", 0)), it["counts"].data_ptr(),
                               phi.data_ptr(), phi.shape[0], it["V"].data_ptr())
        self._arr = arr
        self.n_pay = [it["phi"].reshape(-1, it["plan"].points).shape[0] for it in items]
        h = ctypes.c_void_p()
        _check(L.qtree_batch_plan(arr, len(items), tuner._h if tuner else None,
                                  int(scratch_bytes), 1 if graph else 0, ctypes.byref(h)))
        self._h = h
        self.tuner = tuner

    def run(self, want_v0: bool = True, stream=None):
        V0 = np.zeros(sum(self.n_pay), np.float64) if want_v0 else None
        _check(_batch_setup().qtree_batch_run(self._h, _np_ptr(V0) if want_v0 else None,
                                              _stream_handle(stream)))
        return V0

    def info(self):
        u, t = ctypes.c_int64(), ctypes.c_int64()
        g, p1, pn = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(_batch_setup().qtree_batch_info(self._h, ctypes.byref(u), ctypes.byref(t),
                                               ctypes.byref(g), ctypes.byref(p1),
                                               ctypes.byref(pn)))
        return {"units": u.value, "tiles": t.value, "groups": g.value,
                "per_cu_1d": p1.value, "per_cu_nd": pn.value}

    def tuning(self):
        """(configuration code, measured forward ms, candidates timed)."""
        c, t = ctypes.c_int32(), ctypes.c_int32()
        ms = ctypes.c_double()
        _check(_batch_setup().qtree_batch_tuning(self._h, ctypes.byref(c), ctypes.byref(ms),
                                                 ctypes.byref(t)))
        return {"config": c.value, "ms": ms.value, "timed": t.value}

    def set_config(self, code: int):
        _check(_batch_setup().qtree_batch_set_config(self._h, int(code)))

    @property
    def signature(self) -> str:
        return _batch_setup().qtree_batch_signature(self._h).decode()

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._h.value and _lib is not None:
            _lib.qtree_batch_destroy(self._h)
            self._h = None
