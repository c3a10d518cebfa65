"""Pins for the oracle's nearest-neighbour projection (Sec. 2, Voronoi cells).

The FP32 rules are compared with FP64 brute-force argmin of the Euclidean
distance: they may disagree only where the two nearest candidates are
closer than the rounding slack of the FP32 rule, and ties go to the lowest
index.
"""
import numpy as np
import pytest


def _ulp32(x):
    x = np.abs(np.asarray(x, np.float64))
    return 2.0 ** (np.floor(np.log2(np.maximum(x, 2.0**-126))) - 23)


def test_cell_1d_matches_searchsorted_and_fp64_argmin(oracle_lib):
    rng = np.random.default_rng(3)
    for N in (1, 2, 3, 7, 64, 100, 257):
        g = np.sort(rng.standard_normal(N)).astype(np.float32)
        g = np.unique(g)
        N = g.size
        xs = np.concatenate([rng.standard_normal(400) * 2.0,
                             0.5 * (g[1:] + g[:-1])]).astype(np.float32)
        mids32 = (np.float32(0.5) * (g[1:] + g[:-1])).astype(np.float32)
        for x in xs:
            c = oracle_lib.cell(g, 1, x)
            # library binary search over the FP32 midpoints (left side = strict <)
            assert c == int(np.searchsorted(mids32, x, side="left"))
            d64 = np.abs(np.float64(x) - g.astype(np.float64))
            best = int(np.argmin(d64))
            if c != best:
                # only inside the rounding slack of the FP32 midpoint
                mid = 0.5 * (np.float64(g[min(c, best)]) + np.float64(g[max(c, best)]))
                assert abs(np.float64(x) - mid) <= _ulp32(mid)


def test_cell_1d_ties_and_ends(oracle_lib):
    g = np.array([-1.0, 0.0, 2.0, 3.0], np.float32)
    assert oracle_lib.cell(g, 1, -0.5) == 0        # exactly on the first midpoint -> lower
    assert oracle_lib.cell(g, 1, np.nextafter(np.float32(-0.5), np.float32(1))) == 1
    assert oracle_lib.cell(g, 1, 1.0) == 1
    assert oracle_lib.cell(g, 1, 2.5) == 2
    assert oracle_lib.cell(g, 1, -1e30) == 0
    assert oracle_lib.cell(g, 1, 1e30) == 3
    assert oracle_lib.cell(np.array([5.0], np.float32), 1, -3.0) == 0


@pytest.mark.parametrize("d", [2, 3])
def test_cell_nd_matches_fp64_argmin(oracle_lib, d):
    rng = np.random.default_rng(10 + d)
    mism = 0
    for trial in range(6):
        N = int(rng.integers(1, 60))
        g = (rng.standard_normal((N, d)) * rng.uniform(0.2, 3.0)).astype(np.float32)
        X = (rng.standard_normal((300, d)) * 2.0).astype(np.float32)
        g64 = g.astype(np.float64)
        for x in X:
            c = oracle_lib.cell(g.reshape(-1), d, x)
            d2 = np.sum((x.astype(np.float64) - g64) ** 2, axis=1)
            best = int(np.argmin(d2))
            if c != best:
                mism += 1
                # the half-norm key h - <x, g> carries about d + 2 roundings of
                # size ulp(|g|^2/2 + |<x, g>|); distances are twice the key
                scale = 0.5 * np.sum(g64 ** 2, axis=1) + np.abs(g64 @ x.astype(np.float64))
                slack = 2.0 * (d + 3) * 2.0**-24 * max(scale[c], scale[best])
                assert d2[c] - d2[best] <= slack
    assert mism < 10


def test_cell_nd_ties_lowest_index(oracle_lib):
    g = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 0.0], [-1.0, 0.0]], np.float32)
    # equidistant from points 0, 1 and 2 (duplicate of 0): lowest index wins
    assert oracle_lib.cell(g.reshape(-1), 2, np.array([0.0, 0.0], np.float32)) == 0
    assert oracle_lib.cell(g.reshape(-1), 2, np.array([0.9, 0.1], np.float32)) == 0
    assert oracle_lib.cell(g.reshape(-1), 2, np.array([0.1, 0.9], np.float32)) == 1
    assert oracle_lib.cell(g.reshape(-1), 2, np.array([-0.9, 0.0], np.float32)) == 3
