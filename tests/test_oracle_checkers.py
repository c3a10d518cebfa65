"""Pins for the two oracle entry points that check the full-size GPU runs.

`layer_counts_one` (one layer's counts, threads splitting the samples) and
`cells_bulk` (many points, one grid) are what the large parity tests
compare against.  They are tied here to the pinned whole-tree
`transitions` and the one-point `cell` (Sec. 4, Algorithm III: each layer's
counts are a function of that layer's samples alone; Sec. 2: the cell of a
point is the nearest-neighbour projection), so a wrong layer offset, grid
slice or thread split in them fails on the CPU.
"""
import numpy as np
import pytest

import synth


def _model(O, d, n, rho=0.0):
    spec = synth.bm_model(d, n, T=1.0, rho=rho)
    return spec, O.Model(spec["d"], spec["n"], spec["A"], spec["b"], spec["T"], spec["mu"],
                         spec["L"], spec["x0"])


def _sizes(d, n, rng):
    if d == 1:
        return [1] + [int(rng.integers(3, 40)) for _ in range(n)]
    if d == 2:
        return [1] + [(int(rng.integers(2, 7)), int(rng.integers(2, 7))) for _ in range(n)]
    return [1] + [(2, int(rng.integers(2, 4)), int(rng.integers(2, 4))) for _ in range(n)]


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("m0", [0, 1, 12_345])
def test_layer_counts_one_equals_block_of_transitions(oracle_lib, d, m0):
    O = oracle_lib
    rng = np.random.default_rng(100 * d + m0 % 97)
    n = 5
    spec, mdl = _model(O, d, n, rho=0.3 if d > 1 else 0.0)
    grid, N = synth.layer_grids(spec, _sizes(d, n, rng))
    M, seed = 20_001, synth.SEED_BASE + 7
    whole = O.transitions(mdl, grid, N, M, seed=seed, contract=3, m0=m0)
    for k in range(n):
        for threads in (1, 3):
            one = O.layer_counts_one(mdl, grid, N, k, M, seed, contract=3, m0=m0,
                                     nthreads=threads)
            assert np.array_equal(one, O.layer_counts(whole, N, k)), (d, m0, k, threads)
            assert int(one.sum()) == M


def test_layer_counts_one_rejects_bad_layer(oracle_lib):
    O = oracle_lib
    spec, mdl = _model(O, 1, 3)
    grid, N = synth.layer_grids(spec, [1, 4, 4, 4])
    for k in (-1, 3):
        with pytest.raises(ValueError):
            O.layer_counts_one(mdl, grid, N, k, 10, 1)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_cells_bulk_equals_cell_one_by_one(oracle_lib, d):
    O = oracle_lib
    rng = np.random.default_rng(40 + d)
    for N in (1, 2, 9, 50):
        if d == 1:
            g = np.unique(rng.standard_normal(N).astype(np.float32)).reshape(-1, 1)
        else:
            g = rng.standard_normal((N, d)).astype(np.float32)
            g[N // 2] = g[0]            # a duplicate point: ties go to the lower index
        x = (rng.standard_normal((300, d)) * 1.5).astype(np.float32)
        q = min(3, g.shape[0])
        x[:q] = g[:q]                   # points on grid points
        got = O.cells_bulk(g.reshape(-1), d, x)
        want = np.array([O.cell(g.reshape(-1), d, xi) for xi in x], np.int32)
        assert np.array_equal(got, want), (d, N)
