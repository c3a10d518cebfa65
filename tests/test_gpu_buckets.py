"""The d = 2 bucketed cell search against the full scan and the oracle.

Each bucket of a layer's reachable box lists every grid point that can be
the FP32 argmin of the half-norm key anywhere in it (the key's rounding
slack included), so the cell must be the brute-force search's cell (Sec. 2:
the nearest-neighbour projection; Sec. 4: the brute-force search) bit for
bit: on the time-layer samples themselves, on the grid points, on midpoints
of neighbouring points (near-ties), on points placed exactly on bucket
edges and one ulp either side, on duplicated grid points (exact ties), and
outside the box (the full-scan fallback); counts with the tables on and off
equal the oracle's."""
import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1101_3228_amd as qt  # noqa: E402


def _case(name):
    print(f"[gpu-case] {name}", flush=True)


def _omodel(spec):
    return O.Model(spec["d"], spec["n"], spec["A"], spec["b"], spec["T"], spec["mu"], spec["L"],
                   spec["x0"])


def _edge_points(plan, k, g, rng, count=3000):
    """Points on bucket edges of layer k (and one ulp either side) along
    both axes, the other coordinate drawn inside the box."""
    lo, sc, B = plan.buckets(k)
    if B[0] == 0:
        return np.zeros((0, 2), np.float32)
    f32 = np.float32
    pts = []
    for axis in (0, 1):
        i = rng.integers(0, B[axis] + 1, count)
        # the FP32 edge lo + i / scale and its neighbours
        e = (lo[axis] + (i.astype(np.float32) / sc[axis]).astype(f32)).astype(f32)
        other = 1 - axis
        span = (B[other] / sc[other]).astype(f32)
        o = (lo[other] + rng.random(count).astype(f32) * span).astype(f32)
        for v in (e, np.nextafter(e, f32(-np.inf)), np.nextafter(e, f32(np.inf))):
            p = np.empty((count, 2), f32)
            p[:, axis] = v
            p[:, other] = o
            pts.append(p)
    return np.concatenate(pts)


GRIDS = {
    "product": lambda spec: synth.layer_grids(spec, [1] + [(40, 50)] * spec["n"],
                                              base=qt.gauss_quantizer),
    "quantile": lambda spec: synth.layer_grids(spec, [1] + [700] * spec["n"]),
    "jitter_ties": lambda spec: synth.layer_grids(spec, [1] + [300] * spec["n"],
                                                  rng=np.random.default_rng(3), jitter=0.3),
}


@pytest.mark.parametrize("model,grid", [("bm2", "product"), ("ou2", "quantile"),
                                        ("bm2", "jitter_ties")])
def test_bucketed_cells_equal_full_scan_and_oracle(model, grid):
    _case(f"bucketed cells {model} {grid}")
    spec = (synth.bm_model(2, 4, T=1.0, rho=0.3) if model == "bm2"
            else synth.ou_model(4, alpha=(0.5, 8.0), sig=(0.7, 1.3), rho=-0.6))
    g_all, N = GRIDS[grid](spec)
    if grid == "jitter_ties":
        # exact ties: every layer repeats some of its points
        off = np.concatenate([[0], np.cumsum(N)])
        for k in range(1, spec["n"] + 1):
            blk = g_all[off[k]:off[k + 1]]
            blk[1::7] = blk[0::7][:len(blk[1::7])]
    plan = qt.Plan(spec, g_all, N)
    off = np.concatenate([[0], np.cumsum(N)])
    rng = np.random.default_rng(17)
    for k in range(spec["n"] + 1):
        g = g_all[off[k]:off[k + 1]].reshape(-1, 2)
        lo, sc, B = plan.buckets(k)
        if N[k] > 1:
            assert B[0] == B[1] and B[0] * B[0] >= 8 * N[k]
        else:
            assert B[0] == 0
        pts = [g.astype(np.float32), ((g[:-1] + g[1:]) * 0.5).astype(np.float32),
               _edge_points(plan, k, g, rng),
               (rng.standard_normal((20_000, 2)) * 8.0).astype(np.float32)]   # also far out
        kk = min(k, spec["n"] - 1)
        xs, ys = qt.layer_samples(plan, kk, 0, 200_000, seed=0x5EED0050)
        pts.append((xs if k == kk else ys).cpu().numpy())
        x = np.concatenate(pts).astype(np.float32)
        xd = torch.from_numpy(x).cuda()
        got = qt.cells(plan, k, xd).cpu().numpy()
        plan.tune(buckets=0)
        full = qt.cells(plan, k, xd).cpu().numpy()
        plan.tune(buckets=1)
        ref = O.cells_bulk(g, 2, x)
        assert np.array_equal(full, ref), k
        assert np.array_equal(got, ref), (k, int(np.sum(got != ref)))


def test_bucketed_counts_equal_full_scan_and_oracle():
    """The 2-D workload's grids (40 x 50 products mapped by sqrt(t_k)
    chol(R)) on 8 layers, M = 400 001 pairs per layer: counts with and
    without the tables equal the oracle's."""
    _case("bucketed counts, 2-D workload grids, n=8, M=400001")
    spec = synth.bm_model(2, 8, T=1.0, rho=0.3)
    grid, N = synth.layer_grids(spec, [1] + [(40, 50)] * 8, base=qt.gauss_quantizer)
    plan = qt.Plan(spec, grid, N)
    assert plan.tuning()["nd_samples"] == 4  # the default with bucket tables
    M, seed = 400_001, 0x5EED0051
    ref = O.transitions(_omodel(spec), grid, N, M, seed=seed, contract=3, nthreads=16)
    # both samples-per-lane settings, with and without the tables
    for s in (4, 8):
        plan.tune(nd_samples=s, buckets=1)
        on = plan.transitions(M, seed, contract=3).cpu().numpy()
        plan.tune(buckets=0)
        off_ = plan.transitions(M, seed, contract=3).cpu().numpy()
        assert np.array_equal(off_, ref), s
        assert np.array_equal(on, ref), s
    plan.tune(nd_samples=4, buckets=1)
