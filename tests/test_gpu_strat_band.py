"""Banded stratified counts (d = 1): the packed band of every row, expanded,
must equal the oracle's dense stratified counts bit for bit (zeros outside
the band included) with no sample outside its band; the band must contain
the cells of the extreme samples the oracle's own arithmetic produces (the
cell's end quantiles and the largest Box-Muller normals of either sign);
the BDP on banded counts agrees with the oracle's BDP on the dense ones."""
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


def _expand(plan, band, N):
    """Dense counts (layers concatenated) from the packed band."""
    values, off, lo = plan.strat_band()
    out = []
    r = 0
    for k in range(len(N) - 1):
        blk = np.zeros((N[k], N[k + 1]), np.int32)
        for i in range(N[k]):
            w = off[r + 1] - off[r]
            blk[i, lo[r]:lo[r] + w] = band[off[r]:off[r + 1]]
            r += 1
        out.append(blk.ravel())
    return np.concatenate(out)


CASES = {
    "bm": (lambda: synth.bm_model(1, 7, T=1.5), [1, 37, 64, 100, 1, 129, 500, 2]),
    "shifted": (lambda: synth.bm_model(1, 4, T=0.7, x0=[0.4]), [1, 9, 16, 33, 8]),
    "ou": (lambda: synth.ou1_model(5, alpha=2.0, sig=0.8, theta=0.5, x0=-0.3, T=3.0),
           [1, 64, 64, 64, 64, 64]),
}


@pytest.mark.parametrize("name,M,alloc", [("bm", 997, 0), ("bm", 300_000, 1),
                                          ("shifted", 50_001, 1), ("ou", 20_000, 0)])
def test_banded_counts_equal_the_dense_oracle(name, M, alloc):
    _case(f"strat banded {name} M={M} alloc={alloc}")
    mk, shape = CASES[name]
    spec = mk()
    grid, N = synth.layer_grids(spec, shape)
    plan = qt.Plan(spec, grid, N)
    band, overflow = plan.transitions_stratified_banded(M, 0x5EED0034, contract=2, alloc=alloc)
    assert int(overflow.item()) == 0
    got = _expand(plan, band.cpu().numpy(), N)
    ref = O.transitions_stratified(_omodel(spec), grid, N, M, seed=0x5EED0034, contract=2,
                                   alloc=alloc)
    assert np.array_equal(got, ref)
    dense = plan.transitions_stratified(M, 0x5EED0034, contract=2, alloc=alloc).cpu().numpy()
    assert np.array_equal(dense, ref)


def test_band_holds_the_extreme_samples():
    """Row i's samples reach their extremes at the cell's end probabilities
    (clamped as the sampler clamps them) and at the largest Box-Muller normal
    of either sign (radius word 0, angle 0 or one half turn); the cells of
    those X_{k+1}, by the oracle's arithmetic and cell rule, lie in the band."""
    _case("strat band extremes")
    spec = synth.bm_model(1, 6, T=2.0, x0=[0.3])
    grid, N = synth.layer_grids(spec, [1, 5, 40, 200, 7, 300, 33], base=qt.gauss_quantizer)
    plan = qt.Plan(spec, grid, N)
    values, off, lo = plan.strat_band()
    eps_hi, _ = O.box_muller(0, 0)
    eps_lo, _ = O.box_muller(0, 1 << 31)
    assert eps_hi > 5.76 and eps_lo < -5.76
    poff = np.concatenate([[0], np.cumsum(N)])
    f32 = np.float32
    r = 0
    for k in range(spec["n"]):
        gk = grid[poff[k]:poff[k + 1], 0]
        gk1 = grid[poff[k + 1]:poff[k + 2], 0]
        mu, L = spec["mu"][k, 0], spec["L"][k, 0, 0]
        A, b, T = spec["A"][k, 0, 0], spec["b"][k, 0], spec["T"][k, 0, 0]
        e = O.strat_edges(gk, mu, L)
        for i in range(N[k]):
            cells = []
            for p in (e[i], e[i + 1]):
                p = min(max(p, 2.0 ** -1074), 1.0 - 2.0 ** -53)
                x = f32(np.float64(L) * np.float64(f32(O.ppnd16(p))) + np.float64(mu))
                for eps in (eps_lo, eps_hi):
                    y = f32(np.float64(T) * np.float64(eps)
                            + np.float64(f32(np.float64(A) * np.float64(x) + np.float64(b))))
                    cells.append(O.cell(gk1.reshape(-1, 1), 1, [y]))
            assert lo[r] <= min(cells) and max(cells) < lo[r] + (off[r + 1] - off[r]), (k, i)
            r += 1
    dense = sum(int(N[k]) * int(N[k + 1]) for k in range(spec["n"]))
    print(f"[gpu-case] band values {values} of {dense} dense entries", flush=True)


def test_banded_bdp_matches_the_oracle():
    _case("strat banded bdp, n=50 N=500")
    spec = synth.bm_model(1, 50, T=1.0)
    grid, N = synth.layer_grids(spec, [1] + [500] * 50, base=qt.gauss_quantizer)
    plan = qt.Plan(spec, grid, N)
    values, off, lo = plan.strat_band()
    dense = int(sum(int(N[k]) * int(N[k + 1]) for k in range(50)))
    print(f"[gpu-case] band values {values} of {dense} dense entries "
          f"({values / dense:.3f})", flush=True)
    M = 2_000
    band, overflow = plan.transitions_stratified_banded(M, 0x5EED0035)
    assert int(overflow.item()) == 0
    phis = np.stack([O.payoff(0, 1, N, grid, 100.0, 100.0 * kr, 0.05, 1.0, s)
                     for s in (0.1, 0.3) for kr in (0.8, 1.2)])
    V0, _ = plan.bdp_banded(band, torch.from_numpy(phis).cuda())
    ref = O.transitions_stratified(_omodel(spec), grid, N, M, seed=0x5EED0035)
    assert np.array_equal(_expand(plan, band.cpu().numpy(), N), ref)
    rV0, _, _ = O.bdp(ref, N, phis)
    assert np.allclose(V0, rV0, rtol=1e-9, atol=0)


def test_banded_calls_reject_d2():
    _case("strat banded errors")
    spec = synth.bm_model(2, 2)
    grid, N = synth.layer_grids(spec, [1, (3, 3), (3, 4)])
    plan = qt.Plan(spec, grid, N)
    with pytest.raises(qt.QtreeError) as e:
        plan.strat_band()
    assert e.value.status == 5
