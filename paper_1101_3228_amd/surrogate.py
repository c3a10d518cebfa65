"""Pricing surrogate on the quantization tree (binding of include/qtree_mlp.h).

``MLP`` marshals arguments to the network kernels of libqtree.so (forward,
gradient, Adam step).  ``PutTreePricer`` prices American / European puts with
the tree of the paper (transition counts of the time-layer parallel forward
step, Sec. 4, and the backward dynamic programming, Sec. 2); ``Surrogate``
trains the network on such prices and answers queries with it, sending the
queries outside its training box back to the tree.

Brownian scaling: the tree runs on the standardised Brownian motion W_s at
s_k = k / n, whose transition counts depend only on n and the grid size.  A
contract with maturity T and volatility sigma is the payoff
phi(S0 exp((r - sigma^2/2) t_k + sigma sqrt(T) W_{s_k})), t_k = k T / n, on
the same tree (the payoff map mix = sqrt(T)), so one forward step per n
serves every (S0/K, sigma, r, T).
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import (EUROPEAN, PAYOFF_SPEC, PUT, Plan, _check, _np_ptr, _stream_handle,
               bdp_many_trees, gauss_quantizer, lib, payoff_specs)

N_PARAMS = 133633
N_INPUTS = 6

_ready = False


def _setup():
    global _ready
    L = lib()
    if _ready:
        return L
    P, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    L.qtree_mlp_workspace_size.argtypes = [i64, P]
    L.qtree_mlp_create.argtypes = [P, P, P, f32, i32, i32, i64, P, ctypes.c_size_t, P]
    L.qtree_mlp_destroy.argtypes = [P]
    L.qtree_mlp_destroy.restype = None
    L.qtree_mlp_get_params.argtypes = [P, P]
    L.qtree_mlp_set_params.argtypes = [P, P]
    L.qtree_mlp_forward.argtypes = [P, P, i64, P, P, P]
    L.qtree_mlp_grad.argtypes = [P, P, P, P, P, i64, P, P, P]
    L.qtree_mlp_train_step.argtypes = [P, P, P, P, P, i64, P, P, P]
    for f in ("qtree_mlp_workspace_size", "qtree_mlp_create", "qtree_mlp_get_params",
              "qtree_mlp_set_params", "qtree_mlp_forward", "qtree_mlp_grad",
              "qtree_mlp_train_step"):
        getattr(L, f).restype = ctypes.c_int
    _ready = True
    return L


class _Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


class MLP:
    """The 6-256-256-256-1 network in a device workspace."""

    def __init__(self, params, lo, hi, out_scale: float = 0.1, act_terms: int = 2,
                 max_batch: int = 0, baseline: int = 0, device: str = "cuda"):
        import torch
        L = _setup()
        p = np.ascontiguousarray(params, np.float32)
        if p.size != N_PARAMS:
            raise ValueError(f"need {N_PARAMS} parameters, got {p.size}")
        self.lo = np.ascontiguousarray(lo, np.float32)
        self.hi = np.ascontiguousarray(hi, np.float32)
        nbytes = ctypes.c_size_t()
        _check(L.qtree_mlp_workspace_size(int(max_batch), ctypes.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        self._ws = (base + 255) // 256 * 256
        self._h = ctypes.c_void_p()
        _check(L.qtree_mlp_create(_np_ptr(p), _np_ptr(self.lo), _np_ptr(self.hi),
                                  float(out_scale), int(act_terms), int(baseline),
                                  int(max_batch), self._ws,
                                  nbytes.value, ctypes.byref(self._h)))
        self.device = self.workspace.device
        self.max_batch = int(max_batch)

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            try:
                lib().qtree_mlp_destroy(self._h)
            except Exception:
                pass
            self._h = None

    def params(self) -> np.ndarray:
        out = np.empty(N_PARAMS, np.float32)
        _check(_setup().qtree_mlp_get_params(self._h, _np_ptr(out)))
        return out

    def set_params(self, params) -> None:
        p = np.ascontiguousarray(params, np.float32)
        _check(_setup().qtree_mlp_set_params(self._h, _np_ptr(p)))

    def forward(self, x, y=None, in_range=None, want_mask: bool = True, stream=None):
        """x: device float32 [B, 6] raw parameters -> (y [B], in_range uint8 [B] or None)."""
        import torch
        B = x.shape[0]
        if y is None:
            y = torch.empty(B, dtype=torch.float32, device=x.device)
        if want_mask and in_range is None:
            in_range = torch.empty(B, dtype=torch.uint8, device=x.device)
        _check(_setup().qtree_mlp_forward(self._h, x.data_ptr(), B, y.data_ptr(),
                                          _ptr(in_range) if want_mask else None,
                                          _stream_handle(stream)))
        return y, (in_range if want_mask else None)

    def grad(self, x, t, w=None, idx=None, B: int | None = None, grad=None, loss=None,
             stream=None):
        """Gradient of sum_b w_b (y_b - t_b)^2 / B: (grad [133633], loss [1]) device float32."""
        import torch
        B = int(idx.numel() if (B is None and idx is not None) else (B or t.numel()))
        if grad is None:
            grad = torch.empty(N_PARAMS, dtype=torch.float32, device=x.device)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(_setup().qtree_mlp_grad(self._h, x.data_ptr(), t.data_ptr(), _ptr(w), _ptr(idx),
                                       B, grad.data_ptr(), loss.data_ptr(),
                                       _stream_handle(stream)))
        return grad, loss

    def train_step(self, x, t, w, idx, B: int, lr: float, beta1: float = 0.9,
                   beta2: float = 0.999, eps: float = 1e-8, loss=None, idx_offset: int = 0,
                   stream=None):
        """One Adam step on rows idx[idx_offset : idx_offset + B]."""
        opt = _Adam(lr, beta1, beta2, eps)
        ip = None if idx is None else idx.data_ptr() + 4 * int(idx_offset)
        _check(_setup().qtree_mlp_train_step(self._h, x.data_ptr(), t.data_ptr(), _ptr(w), ip,
                                             int(B), ctypes.byref(opt), _ptr(loss),
                                             _stream_handle(stream)))


# ---------------------------------------------------------------- the tree

def unit_bm_model(n: int) -> dict:
    """AR(1) coefficients of the standardised Brownian motion at s_k = k/n
    (A = 1, b = 0, T_k = sqrt(1/n), X_k ~ sqrt(k/n) z), FP32."""
    dt = 1.0 / n
    return dict(d=1, n=n,
                A=np.ones((n, 1, 1), np.float32), b=np.zeros((n, 1), np.float32),
                T=np.full((n, 1, 1), math.sqrt(dt), np.float32),
                mu=np.zeros((n + 1, 1), np.float32),
                L=np.sqrt(np.arange(n + 1) * dt).astype(np.float32).reshape(n + 1, 1, 1),
                x0=np.zeros(1, np.float32))


def unit_bm_grid(n: int, N: int):
    """Layer grids sqrt(k/n) z^(N) (z^(N) the quadratic-optimal N(0,1)
    quantizer), layer 0 = {0}: (float32 [points, 1], N int32 [n+1])."""
    z = gauss_quantizer(N)
    parts = [np.zeros(1)] + [math.sqrt(k / n) * z for k in range(1, n + 1)]
    return (np.concatenate(parts).astype(np.float32).reshape(-1, 1),
            np.array([1] + [N] * n, np.int32))


class PutTreePricer:
    """Tree prices V_0 / K of puts; counts are computed once per n (M pairs
    per layer, Philox seed `seed`) and kept on the device.

    Every n uses the same Philox contract id (common random numbers): sample
    m of layer k then has the same normals in every tree, and on the grids
    sqrt(k/n) z^(N) its cells are those of (z, (sqrt(k) z + eps)/sqrt(k+1))
    in the fixed N(0,1) quantizer whatever n is (up to FP32 rounding at cell
    edges).  The price is then a smooth function of n as well, not n
    independent Monte Carlo draws."""

    def __init__(self, N: int = 100, M: int = 10_000_000, seed: int = 0x5EED0000,
                 american: bool = True, device: str = "cuda", chunk: int = 8192,
                 contract: int = 0):
        self.N, self.M, self.seed, self.american = int(N), int(M), int(seed), bool(american)
        self.device, self.chunk, self.contract = device, int(chunk), int(contract)
        self._trees = {}

    def tree(self, n: int):
        """(plan, counts, pi) of the tree with n layers, built on first use."""
        n = int(n)
        if n not in self._trees:
            grid, N = unit_bm_grid(n, self.N)
            plan = Plan(unit_bm_model(n), grid, N, device=self.device, batch_samples=self.M)
            counts = plan.transitions(self.M, self.seed, contract=self.contract)
            self._trees[n] = (plan, counts, plan.pi(counts))
        return self._trees[n]

    def specs(self, x) -> dict:
        """Contract records of the queries grouped by n, for one many-tree
        launch: {"n": [n per group], "rows": [query rows per group],
        "q_begin": int64 [groups + 1], "specs": device qtree_payoff_spec bytes
        of every group in order}; x: host [Q, 6] rows (S0/K, sigma, r, T, n,
        rho)."""
        import torch
        x = np.asarray(x, np.float64)
        kind = PUT if self.american else PUT | EUROPEAN
        ns = np.rint(x[:, 4]).astype(np.int64)
        if np.any(ns < 1):
            raise ValueError("n must be >= 1")
        out = {"n": [], "rows": [], "q_begin": [0]}
        recs = []
        for n in np.unique(ns):
            rows = np.flatnonzero(ns == n)
            q = x[rows]
            recs.append(payoff_specs(1, np.full(rows.size, kind, np.int32), q[:, 0], 1.0,
                                     q[:, 2], q[:, 3], q[:, 1].reshape(-1, 1),
                                     np.sqrt(q[:, 3]).reshape(-1, 1, 1)))
            out["n"].append(int(n))
            out["rows"].append(rows)
            out["q_begin"].append(out["q_begin"][-1] + rows.size)
        out["q_begin"] = np.asarray(out["q_begin"], np.int64)
        allrec = np.concatenate(recs) if recs else np.zeros(0, PAYOFF_SPEC)
        out["specs"] = torch.from_numpy(allrec.view(np.uint8).reshape(-1)).to(self.device)
        return out

    def price_specs(self, groups: dict, out=None, stream=None):
        """V_0 / K of pre-built query groups (see specs) on the device, every
        n in one qtree_bdp_many_trees launch.  Returns device float64
        [queries] in group order."""
        trees = [self.tree(n) for n in groups["n"]]
        return bdp_many_trees([(p, pi) for p, _, pi in trees], groups["specs"],
                              groups["q_begin"], V0=out, stream=stream)

    def price(self, x, stream=None) -> np.ndarray:
        """x: host float [Q, 6] rows (S0/K, sigma, r, T, n, rho) -> V_0 / K (float64)."""
        x = np.asarray(x, np.float64)
        out = np.empty(x.shape[0], np.float64)
        if x.shape[0] == 0:
            return out
        groups = self.specs(x)
        vals = self.price_specs(groups, stream=stream).cpu().numpy()
        for g, rows in enumerate(groups["rows"]):
            out[rows] = vals[groups["q_begin"][g]:groups["q_begin"][g + 1]]
        return out


class Surrogate:
    """Network trained on tree prices; queries outside the box go to the tree."""

    def __init__(self, pricer: PutTreePricer, lo, hi, params, out_scale: float = 0.1,
                 act_terms: int = 2, max_batch: int = 4096, baseline: int = 1,
                 device: str = "cuda"):
        self.pricer = pricer
        self.net = MLP(params, lo, hi, out_scale=out_scale, act_terms=act_terms,
                       max_batch=max_batch, baseline=baseline, device=device)
        self.max_batch = int(max_batch)

    def fit(self, x, t, epochs: int, lr: float = 2e-3, lr_final: float = 1e-5,
            floor: float = 1e-2, seed: int = 0, batch: int | None = None,
            log=None) -> list:
        """Adam on the relative loss ((y - t) / max(t, floor))^2 with a cosine
        learning-rate decay from lr to lr_final; returns the loss per epoch."""
        import torch
        dev = self.net.device
        B = int(batch or self.max_batch)
        xd = torch.as_tensor(np.ascontiguousarray(x, np.float32), device=dev)
        td = torch.as_tensor(np.ascontiguousarray(t, np.float32), device=dev)
        wh = 1.0 / np.maximum(np.asarray(t, np.float64), floor) ** 2
        wd = torch.as_tensor((wh / wh.mean()).astype(np.float32), device=dev)
        n_rows = xd.shape[0]
        steps = n_rows // B
        total = max(1, epochs * steps)
        rng = np.random.default_rng(seed)
        loss = torch.zeros(steps, dtype=torch.float32, device=dev)
        hist = []
        it = 0
        for ep in range(epochs):
            idx = torch.as_tensor(rng.permutation(n_rows).astype(np.int32), device=dev)
            for s in range(steps):
                a = it / total
                lr_s = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * a))
                self.net.train_step(xd, td, wd, idx, B, lr_s, loss=loss[s:s + 1],
                                    idx_offset=s * B)
                it += 1
            hist.append(float(loss.mean().item()) / float(wh.mean()))
            if log is not None:
                log(ep, hist[-1])
        return hist

    def price(self, x, stream=None):
        """x: host float [Q, 6] -> (V_0 / K float64 [Q], used_tree bool [Q])."""
        import torch
        xd = torch.as_tensor(np.ascontiguousarray(x, np.float32), device=self.net.device)
        y, mask = self.net.forward(xd, stream=stream)
        inside = mask.cpu().numpy().astype(bool)
        out = y.double().cpu().numpy()
        if not inside.all():
            out[~inside] = self.pricer.price(np.asarray(x)[~inside], stream=stream)
        return out, ~inside
