"""GPU parity of the grids for marginals of any law (Sec. 2: moment-matching
sub-optimal grids; the Lloyd condition of eq. Qerr on a caller's sample set)
against the oracle.  Moment sums are exact integers and must be equal; the
mean, covariance and Cholesky factor (FP64) and the mapped grid (FP32) bit
for bit; Lloyd and relaxed Lloyd steps: grids bit for bit, distortions equal
as FP64 numbers, inadmissible samples counted alike.  Sample sets are
non-Gaussian (skewed, bimodal, uniform, correlated) with inadmissible values
(NaN, +-inf, +-100) planted, sizes with ragged tails and windows that wrap."""
import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1101_3228_amd as qt  # noqa: E402

SIZES = {1: (40,), 2: (10, 12), 3: (4, 5, 6)}


def _case(name):
    print(f"[gpu-case] {name}", flush=True)


def _bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint32 if a.dtype == np.float32 else np.uint64)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_moments_and_moment_grid_bitwise(d):
    _case(f"moment grid d={d} M=1000003")
    x = synth.marginal_samples(d, 1_000_003, synth.SEED_BASE + d, bad=97)
    base = synth.product_base(d, SIZES[d], qt.gauss_quantizer)
    xd = torch.from_numpy(x).cuda()
    sums = qt.sample_moments(xd).cpu().numpy()
    cnt, s1, s2 = O.sample_moments(d, x)
    assert sums[0] == cnt and cnt < x.shape[0]
    assert np.array_equal(sums[1:1 + d], s1)
    assert np.array_equal(sums[1 + d:].reshape(d, d), s2)
    grid, mom = qt.moment_grid(xd, torch.from_numpy(base).cuda())
    rg, mean, cov, chol, rc = O.moment_grid(d, x, base)
    assert np.array_equal(_bits(grid.cpu().numpy()), _bits(rg))
    ref = np.concatenate([mean, cov.ravel(), chol.ravel()])
    assert np.array_equal(_bits(mom.cpu().numpy()), _bits(ref))


def test_moment_grid_edge_cases():
    _case("moment grid: empty set, all inadmissible, one point, degenerate direction")
    base = synth.product_base(2, (3, 3), qt.gauss_quantizer)
    bd = torch.from_numpy(base).cuda()
    cases = {
        "empty": np.zeros((0, 2), np.float32),
        "inadmissible": np.full((1000, 2), np.nan, np.float32),
        "one point": np.array([[0.25, -1.5]], np.float32),
        "degenerate": np.stack([np.linspace(-1, 1, 501), np.full(501, 0.5)], 1).astype(np.float32),
    }
    for name, x in cases.items():
        xd = torch.from_numpy(x).cuda() if x.size else torch.empty((0, 2), device="cuda")
        grid, mom = qt.moment_grid(xd, bd)
        rg, mean, cov, chol, rc = O.moment_grid(2, x, base)
        assert np.array_equal(_bits(grid.cpu().numpy()), _bits(rg)), name
        ref = np.concatenate([mean, cov.ravel(), chol.ravel()])
        assert np.array_equal(_bits(mom.cpu().numpy()), _bits(ref)), name


LLOYD_CASES = [
    # d, M, batch, steps, gamma, bad
    (1, 50_000, 20_011, 7, 1.0, 13),
    (1, 30_001, 30_001, 5, 0.3, 0),
    (2, 60_000, 70_001, 5, 1.0, 31),     # windows longer than the set
    (2, 200_003, 65_536, 6, 0.5, 7),
    (3, 80_000, 33_333, 4, 1.0, 5),
    (3, 40_000, 40_000, 3, 0.25, 0),
]


@pytest.mark.parametrize("d,M,batch,steps,gamma,bad", LLOYD_CASES)
def test_lloyd_on_sample_sets_bitwise(d, M, batch, steps, gamma, bad):
    _case(f"lloyd samples d={d} M={M} batch={batch} steps={steps} gamma={gamma}")
    x = synth.marginal_samples(d, M, synth.SEED_BASE + 10 * d + steps, bad=bad)
    base = synth.product_base(d, SIZES[d], qt.gauss_quantizer)
    g0, *_ = O.moment_grid(d, x, base)
    if d == 1:
        g0 = np.sort(g0, axis=0)
    grid, dist, rej = qt.lloyd_samples(g0, torch.from_numpy(x).cuda(), batch, steps, gamma)
    rg, rdist, rrej = O.lloyd_empirical(d, g0, x, batch, steps, gamma)
    assert np.array_equal(_bits(grid.cpu().numpy()), _bits(rg))
    assert np.array_equal(_bits(dist.cpu().numpy()), _bits(rdist))
    assert int(rej.item()) == rrej
    if gamma == 1.0 and batch == M and bad == 0:
        assert np.all(np.diff(rdist) <= 0)        # Lloyd on a fixed measure


def test_lloyd_large_grid_on_samples():
    _case("lloyd samples d=2 N=500 M=1e6 batch=1e6 steps=3")
    x = synth.marginal_samples(2, 1_000_000, synth.SEED_BASE + 77, bad=100)
    base = synth.product_base(2, (20, 25), qt.gauss_quantizer)
    g0, *_ = O.moment_grid(2, x, base)
    grid, dist, rej = qt.lloyd_samples(g0, torch.from_numpy(x).cuda(), 1_000_000, 3)
    rg, rdist, rrej = O.lloyd_empirical(2, g0, x, 1_000_000, 3)
    assert np.array_equal(_bits(grid.cpu().numpy()), _bits(rg))
    assert np.array_equal(_bits(dist.cpu().numpy()), _bits(rdist))
    assert int(rej.item()) == rrej == 3 * 100


def test_lloyd_window_of_inadmissible_samples_keeps_the_grid():
    _case("lloyd samples: a window with no admissible sample")
    x = np.full((64, 2), np.inf, np.float32)
    g0 = synth.product_base(2, (3, 3), qt.gauss_quantizer)
    grid, dist, rej = qt.lloyd_samples(g0, torch.from_numpy(x).cuda(), 64, 2)
    assert np.array_equal(_bits(grid.cpu().numpy()), _bits(g0))
    assert np.all(dist.cpu().numpy() == 0.0) and int(rej.item()) == 128


def test_lloyd_samples_rejects_bad_requests():
    _case("lloyd samples: argument errors")
    x = torch.zeros((10, 2), device="cuda")
    g0 = synth.product_base(2, (2, 2), qt.gauss_quantizer)
    out = torch.full((4, 2), 7.0, device="cuda")
    for kw, status in (({"gamma": 0.0}, 1), ({"gamma": 1.5}, 1), ({"batch": 0}, 3),
                       ({"steps": 0}, 1)):
        args = {"batch": 5, "steps": 1, "gamma": 1.0, **kw}
        with pytest.raises(qt.QtreeError) as err:
            qt.lloyd_samples(g0, x, args["batch"], args["steps"], args["gamma"], grid=out)
        assert err.value.status == status, kw
    with pytest.raises(qt.QtreeError) as err:
        qt.lloyd_samples(g0, torch.zeros((0, 2), device="cuda"), 5, 1, grid=out)
    assert err.value.status == 1
    assert bool((out == 7.0).all())
