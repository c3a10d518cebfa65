"""GPU checks of the stratified time-layer counts (d = 1) against the oracle:
per-sample (X_k, X_{k+1}) bit for bit, counts bit for bit over ragged shapes
(single-point layers, several hundred cells, Ms not a multiple of the
workgroup), every row summing to Ms, and the BDP on stratified counts."""
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


CASES = {
    "bm": (lambda: synth.bm_model(1, 7, T=1.5), [1, 37, 64, 100, 1, 129, 500, 2]),
    "shifted": (lambda: synth.bm_model(1, 4, T=0.7, x0=[0.4]), [1, 9, 16, 33, 8]),
}


@pytest.mark.parametrize("name,alloc", [("bm", 1), ("shifted", 0)])
def test_strat_samples_bitwise(name, alloc):
    _case(f"strat samples {name} alloc {alloc}")
    mk, shape = CASES[name]
    spec = mk()
    grid, N = synth.layer_grids(spec, shape)
    plan = qt.Plan(spec, grid, N)
    mdl = _omodel(spec)
    off = np.concatenate([[0], np.cumsum(N)])
    M = 40_000 if alloc else 997
    for k in range(spec["n"]):
        gk = grid[off[k]:off[k + 1], 0]
        e = O.strat_edges(gk, spec["mu"][k, 0], spec["L"][k, 0, 0])
        rows = O.strat_rows(e, M, alloc)
        # the first and last rows reach the quantile's tail branches
        for i in sorted({0, N[k] // 2, N[k] - 1}):
            assert plan.strat_row(k, i, M, alloc) == rows[i]
            count = int(min(2000, rows[i]))
            for t0 in sorted({0, int(rows[i]) - count}):
                gx, gy = qt.strat_samples(plan, k, i, M, alloc, t0, count, seed=0x5EED0031,
                                          contract=2)
                ox, oy = O.strat_pairs(mdl, k, e, i, t0, count, seed=0x5EED0031, contract=2)
                assert np.array_equal(gx.cpu().numpy().view(np.uint32), ox.view(np.uint32))
                assert np.array_equal(gy.cpu().numpy().view(np.uint32), oy.view(np.uint32))


@pytest.mark.parametrize("name,M,alloc", [("bm", 997, 0), ("bm", 300_000, 1), ("bm", 4096, 0),
                                          ("shifted", 50_001, 1)])
def test_strat_counts_bitwise(name, M, alloc):
    _case(f"strat counts {name} M={M} alloc={alloc}")
    mk, shape = CASES[name]
    spec = mk()
    grid, N = synth.layer_grids(spec, shape)
    plan = qt.Plan(spec, grid, N)
    got = plan.transitions_stratified(M, 0x5EED0032, contract=1, alloc=alloc).cpu().numpy()
    ref = O.transitions_stratified(_omodel(spec), grid, N, M, seed=0x5EED0032, contract=1,
                                   alloc=alloc)
    assert np.array_equal(got, ref)
    off, poff = 0, 0
    for k in range(spec["n"]):
        blk = got[off:off + N[k] * N[k + 1]].reshape(N[k], N[k + 1])
        e = O.strat_edges(grid[poff:poff + N[k], 0], spec["mu"][k, 0], spec["L"][k, 0, 0])
        assert np.array_equal(blk.sum(axis=1), O.strat_rows(e, M, alloc)), k
        off += N[k] * N[k + 1]
        poff += N[k]


def test_strat_bdp_matches_oracle():
    _case("strat bdp")
    spec = synth.bm_model(1, 10, T=1.0)
    grid, N = synth.layer_grids(spec, [1] + [50] * 10, base=qt.gauss_quantizer)
    plan = qt.Plan(spec, grid, N)
    counts = plan.transitions_stratified(100_000, 0x5EED0033)
    phi = plan.payoff(qt.PUT, 100.0, 100.0, 0.05, 1.0, 0.2)
    V0, _ = plan.bdp(counts, phi)
    ref = O.transitions_stratified(_omodel(spec), grid, N, 100_000, seed=0x5EED0033)
    rV0, _, _ = O.bdp(ref, N, O.payoff(0, 1, N, grid, 100.0, 100.0, 0.05, 1.0, 0.2))
    assert V0[0] == pytest.approx(rV0[0], rel=1e-12)


def test_strat_rejects_bad_requests():
    _case("strat errors")
    spec = synth.bm_model(2, 2)
    grid, N = synth.layer_grids(spec, [1, (3, 3), (3, 4)])
    plan2 = qt.Plan(spec, grid, N)
    with pytest.raises(qt.QtreeError) as e:
        plan2.transitions_stratified(100, 1)
    assert e.value.status == 5
    spec1 = synth.bm_model(1, 2)
    grid1, N1 = synth.layer_grids(spec1, [1, 5, 6])
    plan1 = qt.Plan(spec1, grid1, N1)
    for M, alloc, status in ((0, 1, 3), (1 << 31, 0, 3), (100, 2, 1)):
        with pytest.raises(qt.QtreeError) as e:
            plan1.transitions_stratified(M, 1, alloc=alloc)
        assert e.value.status == status
    assert plan1.strat_row(0, 5, 100, 1) == -1                   # row out of range
