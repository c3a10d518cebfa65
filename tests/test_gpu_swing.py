"""GPU checks of the swing option (qtree_swing) and its forward obstacle
(qtree_payoff_forward) against the FP64 oracle.

Tolerances: the forward is the same FP64 formula on both sides (device exp
against host exp, ~1 ulp each): 1e-13 relative.  The swing sums the same
terms in another order (64 lanes, then a butterfly): 1e-12 of the largest
|P|, and the infeasible states (-inf) at exactly the same places.
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


def _ou_tree(n, side, M, seed=5, rho=-0.4):
    spec = synth.ou_model(n, alpha=(1.0, 5.0), sig=(1.0, 1.0), rho=rho)
    grid, N = synth.layer_grids(spec, [1] + [side] * n)
    plan = qt.Plan(spec, grid, N, batch_samples=M)
    counts = plan.transitions(M, seed)
    return spec, grid, N, plan, counts


def test_forward_payoff_matches_oracle():
    _case("forward payoff")
    for spec, shapes, sig in ((synth.bm_model(1, 4, T=1.3), [1, 7, 9, 11, 13], [0.3]),
                              (synth.ou_model(5, rho=0.5), [1] + [(4, 6)] * 5, [0.7, 1.4])):
        grid, N = synth.layer_grids(spec, shapes)
        plan = qt.Plan(spec, grid, N)
        d = spec["d"]
        mix = None if d == 1 else np.array([[1.0, 0.0], [0.3, 0.9]])
        for mx in (None, mix):
            got = plan.payoff_forward(20.0, 19.5, 0.03, 1.3, sig, mix=mx).cpu().numpy()
            ref = O.forward_payoff(spec, N, grid, 20.0, 19.5, 0.03, 1.3, sig, mix=mx)
            assert np.allclose(got, ref, rtol=1e-13, atol=1e-12)


def _compare(Pg, Pr):
    Pg = Pg.T                                  # GPU [point][level], oracle [level][point]
    fin = np.isfinite(Pr)
    assert np.array_equal(fin, np.isfinite(Pg))
    assert np.array_equal(Pr[~fin], Pg[~fin])
    scale = np.abs(Pr[fin]).max()
    assert np.abs(Pg[fin] - Pr[fin]).max() <= 1e-12 * scale


@pytest.mark.parametrize("Q", [(0, 0), (0, 1), (2, 5), (0, 8), (8, 8), (3, 3)])
def test_swing_matches_oracle(Q):
    _case(f"swing Q={Q}")
    n = 8
    spec, grid, N, plan, counts = _ou_tree(n, (5, 6), 60_001)
    v = plan.payoff_forward(20.0, 20.0, 0.0, 1.0, [0.7, 1.4])
    P0, P = plan.swing(counts, v, *Q)
    rP0, rP = O.swing(counts.cpu().numpy(), N, v.cpu().numpy(), *Q, want_all=True)
    _compare(P.cpu().numpy(), rP)
    assert P0 == pytest.approx(rP0, rel=1e-12, abs=1e-14)


def test_swing_with_empty_rows_and_long_horizon():
    """Few samples leave rows no sample reached (continuation 0); a 120-date
    tree with volume range (30, 80) spans many 16-level passes."""
    _case("swing empty rows / long horizon")
    spec, grid, N, plan, counts = _ou_tree(6, (7, 7), 300, seed=9)
    c = counts.cpu().numpy()
    assert (c.reshape(-1)[: 49 * 49] == 0).any()
    v = plan.payoff_forward(20.0, 20.5, 0.01, 1.0, [0.7, 1.4])
    for Q in ((0, 3), (2, 6)):
        _, P = plan.swing(counts, v, *Q)
        _compare(P.cpu().numpy(), O.swing(c, N, v.cpu().numpy(), *Q, want_all=True)[1])
    spec, grid, N, plan, counts = _ou_tree(120, (6, 6), 20_000, seed=13)
    v = plan.payoff_forward(20.0, 20.0, 0.0, 1.0, [0.7, 1.4])
    P0, P = plan.swing(counts, v, 30, 80)
    rP0, rP = O.swing(counts.cpu().numpy(), N, v.cpu().numpy(), 30, 80, want_all=True)
    _compare(P.cpu().numpy(), rP)
    assert P0 == pytest.approx(rP0, rel=1e-12)


def test_swing_rejects_bad_constraints():
    _case("swing errors")
    spec, grid, N, plan, counts = _ou_tree(4, (3, 3), 1000)
    v = plan.payoff_forward(20.0, 20.0, 0.0, 1.0, [0.7, 1.4])
    for Q in ((3, 2), (-1, 2), (0, 5)):
        with pytest.raises(qt.QtreeError) as e:
            plan.swing(counts, v, *Q)
        assert e.value.status == 1
