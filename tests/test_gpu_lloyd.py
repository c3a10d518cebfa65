"""GPU checks of the grid optimizer (qtree_lloyd, randomized Lloyd steps for
eq. Qerr, Sec. 2) against the oracle.

The cell sums are exact integers on both sides and every other operation is
the same FP32/FP64 sequence, so the grids after several steps and the
distortion of every step are compared bit for bit.
"""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1101_3228_amd as qt  # noqa: E402


def _case(name):
    print(f"[gpu-case] {name}", flush=True)


def _compare(d, g0, L, M, steps, seed, fresh):
    g, dist = qt.lloyd(d, g0, L, M, steps, seed, fresh=fresh)
    rg, rdist = O.lloyd(d, g0, L, M, steps, seed, fresh=fresh)
    assert np.array_equal(g.cpu().numpy().view(np.uint32), rg.view(np.uint32))
    assert np.array_equal(dist.cpu().numpy()[:steps], rdist)
    return rg, rdist


@pytest.mark.parametrize("N,M,fresh", [(1, 1000, True), (2, 10_007, True), (7, 33_333, False),
                                       (100, 65_537, True), (513, 40_000, True)])
def test_lloyd_1d_bitwise(N, M, fresh):
    _case(f"lloyd d=1 N={N} M={M}")
    g0 = np.sort(np.random.default_rng(N).normal(size=N)).astype(np.float32)
    g0 = np.unique(g0)
    _compare(1, g0, [[1.3]], M, 3, 0x5EED0021, fresh)


@pytest.mark.parametrize("N,M,fresh", [(1, 999, True), (5, 20_011, True), (37, 50_000, False),
                                       (500, 70_001, True)])
def test_lloyd_2d_bitwise(N, M, fresh):
    _case(f"lloyd d=2 N={N} M={M}")
    g0 = np.random.default_rng(N).normal(size=(N, 2)).astype(np.float32)
    L = np.array([[1.0, 0.0], [0.45, 0.9]])
    _compare(2, g0, L, M, 3, 0x5EED0022, fresh)


@pytest.mark.parametrize("N", [27, 100])
def test_lloyd_3d_bitwise(N):
    _case(f"lloyd d=3 N={N}")
    g0 = np.random.default_rng(N).normal(size=(N, 3)).astype(np.float32)
    L = np.array([[1.0, 0.0, 0.0], [0.3, 0.9, 0.0], [-0.2, 0.1, 0.7]])
    _compare(3, g0, L, 30_001, 2, 0x5EED0023, True)


def test_lloyd_large_grid_and_converges():
    """The largest 2-D grid, and the distortion of an optimized grid is below
    the start's (the grid's quality, not only its parity)."""
    _case("lloyd d=2 N=2048")
    g0 = np.random.default_rng(9).normal(size=(2048, 2)).astype(np.float32)
    _, dist = _compare(2, g0, np.eye(2), 200_000, 2, 0x5EED0024, True)
    assert dist[1] < dist[0]


def test_lloyd_fixed_samples_distortion_is_monotone_on_device():
    _case("lloyd fixed samples")
    g0 = np.random.default_rng(3).normal(size=(60, 2)).astype(np.float32)
    g, dist = qt.lloyd(2, g0, np.eye(2), 30_000, 12, 0x5EED0025, fresh=False)
    dd = dist.cpu().numpy()
    assert np.all(np.diff(dd) <= 1e-9 * dd[:-1])


def test_lloyd_errors_leave_the_output_untouched():
    _case("lloyd errors")
    out = torch.full((4, 2), 7.0, dtype=torch.float32, device="cuda")
    with pytest.raises(qt.QtreeError):
        qt.lloyd(2, np.zeros((4, 2)) + 100.0, np.eye(2), 1000, 1, 1, grid=out)
    assert torch.all(out == 7.0)
