"""GPU checks of the breadth-first fallback of the 1-D cell search.

A layer whose grid packs many points into a tiny interval has no guide table
with at most four midpoints per bucket (even 8192 buckets leave dozens of
midpoints in one bucket), so its plan searches every layer breadth-first.
The forward (both modes), the stratified counts and a batch that mixes such a
contract with ordinary ones must still give the oracle's counts bit for bit.
"""
import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1101_3228_amd as qt  # noqa: E402


def _case(name):
    print(f"[gpu-case] {name}", flush=True)


def _clustered(n):
    """A standard-normal quantile grid of n - 40 points plus 40 points packed
    into [0.3, 0.3 + 1e-5) (well above FP32 spacing after scaling)."""
    base = synth.quantile_grid_1d(n - 40)
    cluster = 0.3 + 1e-5 * np.arange(40) / 40.0
    g = np.sort(np.concatenate([base, cluster]))
    assert np.all(np.diff(g) > 0)
    return g


def _omodel(spec):
    return O.Model(spec["d"], spec["n"], spec["A"], spec["b"], spec["T"], spec["mu"], spec["L"],
                   spec["x0"])


def _clustered_plan():
    spec = synth.bm_model(1, 3, T=1.0)
    grid, N = synth.layer_grids(spec, [1, 90, 120, 101], base=_clustered)
    # the cluster survives the FP32 grid: dozens of midpoints within 1e-5 L_k
    gk = grid[1:91, 0].astype(np.float64)
    assert np.sum(np.diff(gk) < 1e-4) >= 30
    plan = qt.Plan(spec, grid, N)
    assert plan.cell_search() == (-1, 0)  # breadth-first search on every layer
    return spec, grid, N, plan


@pytest.mark.parametrize("mode", [0, 1])
def test_clustered_grid_counts_bitwise(mode):
    _case(f"clustered grid counts mode {mode}")
    spec, grid, N, plan = _clustered_plan()
    M = 150_001
    got = plan.transitions(M, 0x5EED0041, contract=3, mode=mode, m0=17).cpu().numpy()
    ref = O.transitions(_omodel(spec), grid, N, M, seed=0x5EED0041, contract=3, mode=mode, m0=17)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("alloc", [0, 1])
def test_clustered_grid_stratified_bitwise(alloc):
    _case(f"clustered grid stratified alloc {alloc}")
    spec, grid, N, plan = _clustered_plan()
    M = 3_001 if alloc == 0 else 200_000
    got = plan.transitions_stratified(M, 0x5EED0042, contract=1, alloc=alloc).cpu().numpy()
    ref = O.transitions_stratified(_omodel(spec), grid, N, M, seed=0x5EED0042, contract=1,
                                   alloc=alloc)
    assert np.array_equal(got, ref)


def test_batch_mixing_clustered_and_ordinary_contracts():
    """One contract without usable guide tables sends the batch's whole 1-D
    launch to the breadth-first search; every contract still matches its own
    plan, and the plans match the oracle."""
    _case("batch with a clustered contract")
    items = []
    cases = [("clustered", None), ("plain", [1, 64, 80, 80, 33]), ("plain", [1, 7, 300, 2])]
    for i, (kind, shape) in enumerate(cases):
        if kind == "clustered":
            spec, grid, N, plan = _clustered_plan()
        else:
            spec = synth.bm_model(1, len(shape) - 1, T=0.8)
            grid, N = synth.layer_grids(spec, shape)
            plan = qt.Plan(spec, grid, N, batch_samples=1)
            assert plan.cell_search()[0] >= 0
        phi = plan.payoff(qt.PUT, 100.0, 100.0, 0.05, 0.8, [0.2])[None, :].contiguous()
        items.append(dict(plan=plan, M=50_001 + 1000 * i, seed=0x5EED0043 + i, contract_id=i,
                          counts=plan.new_counts(), phi=phi, V=torch.empty_like(phi),
                          spec=spec, grid=grid, N=N))
    batch = qt.Batch(items, scratch_bytes=64 << 20)
    batch.run(want_v0=False)
    torch.cuda.synchronize()
    for it in items:
        ref = O.transitions(_omodel(it["spec"]), it["grid"], it["N"], it["M"], seed=it["seed"],
                            contract=it["contract_id"])
        assert np.array_equal(it["counts"].cpu().numpy(), ref), it["contract_id"]
