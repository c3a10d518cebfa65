"""How far the d >= 2 cell rule departs from the exact nearest neighbour on
the 2-D workload's own grids (Sec. 2: Voronoi cells and the nearest
neighbour projection; Sec. 4: brute-force search over the grid).

The oracle (and the GPU path, which reproduces it bit for bit) assigns a
point x to the lowest index p minimising the FP32 half-norm key
k_p = h_p - <x, g_p>, h_p = |g_p|^2 / 2 (two fused multiply-adds per point),
where the plain form evaluates |x - g_p|^2 = (x_0 - g_0)^2 + (x_1 - g_1)^2
unfused.  Both are the nearest neighbour in exact arithmetic
(|x - g_p|^2 = |x|^2 + 2 k_p); they differ only in rounding.  This test
takes Philox samples of the 2-D workload (n = 30 layers, 40 x 50 products of
N(0, 1) quadratic-optimal grids mapped by sqrt(t_k) chol(R), rho = 0.3) at
early, middle and late layers, and compares the half-norm cell and the plain
form's cell with the FP64 argmin:

  - every half-norm disagreement lies within the derived rounding slack of
    the key: with u = 2^-24, h_p carries a relative error below 2.01 u and
    the two fused steps one rounding each, so
    |k~_p - k_p| <= E_p = 4.1 u (h_p + |x_0 g_0| + |x_1 g_1|), and a
    disagreement q != p* needs (d2_q - d2_p*) / 2 <= E_q + E_p*;
  - every plain-form disagreement lies within its slack (each squared
    difference carries 3 roundings, the sum one more: relative 4.01 u);
  - the disagreement rates are printed (pytest -s) and bounded.

Sample count per layer: 200 000 (QTREE_C3_CELL_SAMPLES overrides it).
"""
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth

U = 2.0 ** -24
LAYERS = (1, 15, 29)          # pairs (X_k, X_{k+1}): grids 1, 2, 15, 16, 29, 30


def _c3(O):
    from oracle import quantizer
    spec = synth.bm_model(2, 30, T=1.0, rho=0.3)
    grid, N = synth.layer_grids(spec, [1] + [(40, 50)] * 30, base=quantizer.gauss_quantizer)
    mdl = O.Model(spec["d"], spec["n"], spec["A"], spec["b"], spec["T"], spec["mu"],
                  spec["L"], spec["x0"])
    return mdl, grid, N


def _plain_cells(P32, G32, cand):
    """Cell by the plain unfused FP32 form over the candidate indices
    (lowest index on ties)."""
    g = G32[cand]                                   # [M, C, 2]
    dx = (P32[:, None, 0] - g[:, :, 0]).astype(np.float32)
    dy = (P32[:, None, 1] - g[:, :, 1]).astype(np.float32)
    dist = (dx * dx).astype(np.float32) + (dy * dy).astype(np.float32)
    dist = dist.astype(np.float32)
    best = dist.min(axis=1, keepdims=True)
    idx = np.where(dist == best, cand, np.iinfo(np.int64).max)
    return idx.min(axis=1)


def test_halfnorm_cells_match_fp64_within_slack_at_2d_workload(oracle_lib):
    O = oracle_lib
    mdl, grid, N = _c3(O)
    off = O.point_offsets(N)
    M = int(os.environ.get("QTREE_C3_CELL_SAMPLES", "200000"))
    n_pts = n_hn = n_plain = n_both = 0
    worst_hn = 0.0
    for k in LAYERS:
        x, y = O.layer_pairs(mdl, k, 0, M, synth.SEED_BASE)
        for layer, P32 in ((k, x), (k + 1, y)):
            G32 = grid[off[layer]:off[layer + 1]]
            G64 = G32.astype(np.float64)
            P64 = P32.astype(np.float64)
            hn = O.cells_bulk(G32.reshape(-1), 2, P32).astype(np.int64)
            # exact nearest neighbours in FP64 (the six nearest as candidates)
            _, cand = cKDTree(G64).query(P64, k=6)
            d2c = np.sum((P64[:, None, :] - G64[cand]) ** 2, axis=2)
            dmin = d2c.min(axis=1)
            pstar = np.where(d2c == dmin[:, None], cand, np.iinfo(np.int64).max).min(axis=1)
            # the candidate set holds every point the FP32 rules could pick
            assert np.all(d2c.max(axis=1) > dmin * (1 + 1e-5) + 1e-30)
            d2 = lambda idx: np.sum((P64 - G64[idx]) ** 2, axis=1)
            h = 0.5 * np.sum(G64 ** 2, axis=1)
            E = lambda idx: 4.1 * U * (h[idx] + np.abs(P64[:, 0] * G64[idx, 0])
                                       + np.abs(P64[:, 1] * G64[idx, 1]))
            bad = hn != pstar
            gap = 0.5 * (d2(hn) - d2(pstar))
            assert np.all(gap >= 0.0)
            slack = E(hn) + E(pstar)
            assert np.all(gap[bad] <= slack[bad]), (layer, np.max(gap[bad] / slack[bad]))
            if bad.any():
                worst_hn = max(worst_hn, float(np.max(gap[bad] / slack[bad])))
            plain = _plain_cells(P32, G32, cand)
            bad_p = plain != pstar
            gap_p = d2(plain) - d2(pstar)
            assert np.all(gap_p[bad_p] <= 4.01 * U * (d2(plain) + d2(pstar))[bad_p])
            n_pts += P32.shape[0]
            n_hn += int(bad.sum())
            n_plain += int(bad_p.sum())
            n_both += int((hn != plain).sum())
    rate_hn, rate_plain, rate_both = n_hn / n_pts, n_plain / n_pts, n_both / n_pts
    print(f"\n2-D workload cells over {n_pts} points (layers {LAYERS} and successors): "
          f"half-norm vs FP64 {n_hn} ({rate_hn:.2e}), plain form vs FP64 {n_plain} "
          f"({rate_plain:.2e}), half-norm vs plain {n_both} ({rate_both:.2e}); "
          f"largest half-norm gap / slack {worst_hn:.3f}")
    # rounding-level departures only: well under one point in ten thousand
    assert rate_hn < 1e-4
    assert rate_plain < 1e-4
