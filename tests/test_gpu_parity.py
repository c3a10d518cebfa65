"""GPU parity: the HIP path (through the C-ABI) against the oracle.

Integer results (Philox words turned into samples, cell indices, transition
counts) must be bit-identical; the FP64 backward step must agree within
1e-9 relative (the tolerance of the specification); payoffs within 1e-13
relative (FP64 exp of two libraries).  Sizes: small cases with several
workgroup chunks and ragged tails, the full-size 1-D workload (n = 50,
N = 500, M = 1e7) with whole sampled layers recomputed by the oracle, and the
full-size 2-D workload (n = 30, N = 2000, M = 1e7) with per-sample checks
and the first layer recomputed.
"""
import os

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1101_3228_amd as qt  # noqa: E402

THREADS = min(16, os.cpu_count() or 1)


def _omodel(spec):
    return O.Model(spec["d"], spec["n"], spec["A"], spec["b"], spec["T"], spec["mu"], spec["L"],
                   spec["x0"])


def _plan(spec, grid, N):
    return qt.Plan(spec, grid, N)


def _lloyd(N):
    return qt.gauss_quantizer(N)


def _print_case(name):
    print(f"[gpu-case] {name}", flush=True)


# ---------------------------------------------------------------- arithmetic

def test_box_muller_every_radius_and_angle():
    _print_case("box_muller exhaustive")
    K = np.arange(2**24, dtype=np.uint64)
    ra = (K << np.uint64(8)).astype(np.uint32)          # u_a = (K + 1) 2^-24, all K
    rb = np.zeros_like(ra)
    g0, g1 = qt.box_muller(torch.from_numpy(ra.view(np.int32)).cuda(),
                           torch.from_numpy(rb.view(np.int32)).cuda())
    o0, o1 = O.box_muller_bulk(ra, rb)
    assert np.array_equal(g0.cpu().numpy().view(np.uint32), o0.view(np.uint32))
    assert np.array_equal(g1.cpu().numpy().view(np.uint32), o1.view(np.uint32))
    ra2 = np.full(2**24, 0x5A5A5A5A, np.uint32)           # fixed radius, every angle
    rb2 = (K << np.uint64(8)).astype(np.uint32)
    g0, g1 = qt.box_muller(torch.from_numpy(ra2.view(np.int32)).cuda(),
                           torch.from_numpy(rb2.view(np.int32)).cuda())
    o0, o1 = O.box_muller_bulk(ra2, rb2)
    assert np.array_equal(g0.cpu().numpy().view(np.uint32), o0.view(np.uint32))
    assert np.array_equal(g1.cpu().numpy().view(np.uint32), o1.view(np.uint32))
    rng = np.random.default_rng(1)
    ra3 = rng.integers(0, 2**32, 1 << 20, dtype=np.uint64).astype(np.uint32)
    rb3 = rng.integers(0, 2**32, 1 << 20, dtype=np.uint64).astype(np.uint32)
    g0, g1 = qt.box_muller(torch.from_numpy(ra3.view(np.int32)).cuda(),
                           torch.from_numpy(rb3.view(np.int32)).cuda())
    o0, o1 = O.box_muller_bulk(ra3, rb3)
    assert np.array_equal(g0.cpu().numpy().view(np.uint32), o0.view(np.uint32))
    assert np.array_equal(g1.cpu().numpy().view(np.uint32), o1.view(np.uint32))


MODELS = {
    "bm1": lambda: synth.bm_model(1, 7, T=1.5),
    "bm2": lambda: synth.bm_model(2, 5, T=1.0, rho=0.3),
    "ou2": lambda: synth.ou_model(6, alpha=(0.5, 8.0), sig=(0.7, 1.3), rho=-0.6),
    "bm3": lambda: synth.bm_model(3, 4, T=2.0, rho=-0.2),
}
SHAPES = {
    "bm1": [1, 37, 64, 100, 1, 129, 500, 2],
    "bm2": [1, (5, 6), (8, 8), 1, (10, 10), (3, 41)],
    "ou2": [1, (6, 6), (7, 7), (8, 8), (9, 9), (10, 10), (11, 11)],
    "bm3": [1, (3, 3, 3), (4, 4, 4), (2, 3, 5), (5, 5, 5)],
}


@pytest.fixture(scope="module", params=list(MODELS))
def small_case(request):
    spec = MODELS[request.param]()
    grid, N = synth.layer_grids(spec, SHAPES[request.param])
    return request.param, spec, grid, N, _plan(spec, grid, N)


def test_layer_samples_bitwise(small_case):
    name, spec, grid, N, plan = small_case
    _print_case(f"layer_samples {name}")
    mdl = _omodel(spec)
    for k in (0, spec["n"] // 2, spec["n"] - 1):
        m0, count = 12_345, 70_001
        gx, gy = qt.layer_samples(plan, k, m0, count, seed=0x5EED0007, contract=3)
        ox, oy = O.layer_pairs(mdl, k, m0, count, seed=0x5EED0007, contract=3)
        assert np.array_equal(gx.cpu().numpy().view(np.uint32), ox.view(np.uint32)), k
        assert np.array_equal(gy.cpu().numpy().view(np.uint32), oy.view(np.uint32)), k


def test_cells_bitwise(small_case):
    name, spec, grid, N, plan = small_case
    _print_case(f"cells {name}")
    d = spec["d"]
    off = np.concatenate([[0], np.cumsum(N)])
    rng = np.random.default_rng(5)
    for k in range(spec["n"] + 1):
        g = grid[off[k]:off[k + 1]].reshape(-1, d)
        pts = [rng.standard_normal((20_000, d)).astype(np.float32) * (1.5 * np.abs(g).max() + 1)]
        if d == 1 and len(g) > 1:
            mids = (np.float32(0.5) * (g[1:, 0] + g[:-1, 0])).astype(np.float32)
            pts.append(mids.reshape(-1, 1))                         # exactly on a cell edge
            pts.append(np.nextafter(mids, np.float32(np.inf)).reshape(-1, 1))
        if d > 1:
            pts.append(g.astype(np.float32))                         # on the grid points
            pts.append(((g[:-1] + g[1:]) * 0.5).astype(np.float32))  # near-ties
        x = np.concatenate(pts).astype(np.float32)
        gc = qt.cells(plan, k, torch.from_numpy(x).cuda()).cpu().numpy()
        oc = O.cells_bulk(g, d, x)
        assert np.array_equal(gc, oc), k


@pytest.mark.parametrize("mode", [0, 1])
def test_counts_small_bitwise_and_schedule_free(small_case, mode):
    name, spec, grid, N, plan = small_case
    _print_case(f"counts {name} mode {mode}")
    mdl = _omodel(spec)
    M, m0, seed = 200_001, 7_777, 0x5EED0011
    ref = O.transitions(mdl, grid, N, M, seed=seed, contract=5, mode=mode, m0=m0,
                        nthreads=THREADS)
    for chunk, xmap, count, groups in ((0, 1, 0, 2), (0, 0, 2, 1), (2, 0, 1, 2), (4_098, 1, 1, 2),
                                       (65_536, 0, 1, 2), (333_333, 1, 1, 2), (0, 1, 2, 3),
                                       (0, 1, 2, 8)):
        plan.tune(chunk=chunk, xcd_map=xmap, count=count, groups=groups)
        got = plan.transitions(M, seed, contract=5, mode=mode, m0=m0).cpu().numpy()
        assert np.array_equal(got, ref), (chunk, xmap, count, groups)
    plan.tune(chunk=0, xcd_map=1, count=0, groups=0)


def test_counts_edge_sizes():
    _print_case("edge sizes")
    spec = synth.bm_model(1, 3)
    grid, N = synth.layer_grids(spec, [1, 5, 1, 9])
    plan = _plan(spec, grid, N)
    mdl = _omodel(spec)
    for M, m0 in ((0, 0), (1, 0), (1, 1), (2, 3), (513, 99)):
        for mode in (0, 1):
            got = plan.transitions(M, 42, mode=mode, m0=m0).cpu().numpy()
            ref = O.transitions(mdl, grid, N, M, seed=42, mode=mode, m0=m0) if M else \
                np.zeros(plan.entries, np.int32)
            assert np.array_equal(got, ref), (M, m0, mode)
    with pytest.raises(qt.QtreeError) as e:
        plan.transitions(2**31, 1)
    assert e.value.status == 3
    with pytest.raises(qt.QtreeError) as e:
        plan.transitions(10, 1, m0=2**32 - 5)
    assert e.value.status == 3


def test_counts_largest_layers():
    """Largest supported layers: 1-D 16384 points, 2-D 4096 points."""
    _print_case("largest layers")
    for d, shape in ((1, 16384), (2, (64, 64))):
        spec = synth.bm_model(d, 2, rho=0.25)
        grid, N = synth.layer_grids(spec, [1, shape, shape])
        plan = _plan(spec, grid, N)
        mdl = _omodel(spec)
        M = 30_001 if d == 1 else 4_001
        for mode in (0, 1):
            got = plan.transitions(M, 9, mode=mode).cpu().numpy()
            ref = O.transitions(mdl, grid, N, M, seed=9, mode=mode, nthreads=THREADS)
            assert np.array_equal(got, ref), (d, mode)


# ---------------------------------------------------------------- pricing

def test_payoff_matches_oracle(small_case):
    name, spec, grid, N, plan = small_case
    d = spec["d"]
    mix = np.tril(np.random.default_rng(5).uniform(0.5, 1.5, (d, d)))
    for kind in (0, 1, 2, 3):
        sig = [0.2, 0.3, 0.25][:d]
        for mx in (None, mix):
            got = plan.payoff(kind, 100.0, 95.0, 0.04, 1.3, sig, mix=mx).cpu().numpy()
            ref = O.payoff(kind, d, N, grid, 100.0, 95.0, 0.04, 1.3, sig, mix=mx)
            fin = np.isfinite(ref)
            assert np.array_equal(fin, np.isfinite(got))
            assert np.allclose(got[fin], ref[fin], rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("sizes,M", [([1, 30, 40, 50, 60, 70], 3_000),
                                     ([1, 1100, 1023, 1024, 2000, 1500], 1_500)])
def test_bdp_matches_oracle_with_edge_rows(sizes, M):
    """Few samples leave empty rows; the second shape's rows of 1023 to 2000
    columns take several rounds of the row walk's eight loads per lane."""
    _print_case(f"bdp edges {sizes}")
    spec = synth.bm_model(1, 5)
    grid, N = synth.layer_grids(spec, sizes)
    plan = _plan(spec, grid, N)
    counts = plan.transitions(M, 7).cpu().numpy()           # few samples: empty rows
    phis = []
    for kind in (0, 2):
        for K in (80.0, 100.0, 120.0):
            for sig in (0.1, 0.25, 0.4):
                phis.append(O.payoff(kind, 1, N, grid, 100.0, K, 0.05, 1.0, sig))
    phi = np.stack(phis)                                     # 18 payoffs: 3 passes of 8
    V0, V = plan.bdp(torch.from_numpy(counts).cuda(), torch.from_numpy(phi).cuda())
    rV0, rV, empty = O.bdp(counts, N, phi, want_all=True)
    assert empty > 0
    assert np.allclose(V0, rV0, rtol=1e-9, atol=0)
    Vh = V.cpu().numpy()
    fin = np.isfinite(rV)
    assert np.array_equal(fin, np.isfinite(Vh))
    scale = np.abs(rV[fin]).max()
    assert np.max(np.abs(Vh[fin] - rV[fin])) <= 1e-9 * scale


# ---------------------------------------------------------------- full-size workloads

def test_c1_pathwise_put_full():
    """1-D American put, n = 10, N = 100 Lloyd grid, M = 1e5 paths."""
    _print_case("C1 full")
    spec = synth.bm_model(1, 10, T=1.0)
    grid, N = synth.layer_grids(spec, [1] + [100] * 10, base=_lloyd)
    plan = _plan(spec, grid, N)
    counts = plan.transitions(100_000, synth.SEED_BASE, mode=qt.PATHWISE)
    ref = O.transitions(_omodel(spec), grid, N, 100_000, seed=synth.SEED_BASE, mode=1,
                        nthreads=THREADS)
    got = counts.cpu().numpy()
    assert np.array_equal(got, ref)
    phi = plan.payoff(qt.PUT, 100.0, 100.0, 0.05, 1.0, 0.2)
    V0, _ = plan.bdp(counts, phi)
    rV0, _, _ = O.bdp(ref, N, O.payoff(0, 1, N, grid, 100.0, 100.0, 0.05, 1.0, 0.2))
    assert abs(V0[0] - rV0[0]) <= 1e-9 * abs(rV0[0])


def test_c2_layerwise_full_size():
    """1-D, n = 50, N = 500, M = 1e7 pairs per layer (the benchmark workload,
    in its launch configuration): every layer sums to M, four whole layers
    recomputed by the oracle, the BDP over a sigma x K sweep."""
    _print_case("C2 full")
    n, Nn, M = 50, 500, 10_000_000
    spec = synth.bm_model(1, n, T=1.0)
    grid, N = synth.layer_grids(spec, [1] + [Nn] * n, base=_lloyd)
    plan = _plan(spec, grid, N)
    # the search the benchmark times: guide tables of 1024 buckets, K = 2
    assert plan.cell_search() == (2, 1024)
    counts = plan.transitions(M, synth.SEED_BASE)
    got = counts.cpu().numpy()
    off = plan.count_offsets()
    sums = np.add.reduceat(got.astype(np.int64), off[:-1])
    assert np.all(sums == M)
    mdl = _omodel(spec)
    for k in (0, 1, 25, n - 1):
        ref = O.layer_counts_one(mdl, grid, N, k, M, seed=synth.SEED_BASE, nthreads=THREADS)
        assert np.array_equal(got[off[k]:off[k + 1]].reshape(N[k], N[k + 1]), ref), k
    phis = np.stack([O.payoff(0, 1, N, grid, 100.0, 100.0 * kr, 0.05, 1.0, s)
                     for s in (0.1, 0.2, 0.3, 0.4) for kr in (0.8, 1.0, 1.2)])
    V0, _ = plan.bdp(counts, torch.from_numpy(phis).cuda())
    rV0, _, _ = O.bdp(got, N, phis)
    assert np.allclose(V0, rV0, rtol=1e-9, atol=0)


def test_c3_2d_full_size():
    """2-D max-call state, n = 30, N = 2000 (40 x 50 product of Lloyd grids
    mapped by sqrt(t_k) chol(R)), M = 1e7 pairs per layer, in the benchmark's
    launch configuration: every layer sums to M; the first, a middle and the
    last layer recomputed in full by the oracle and compared count by count
    (4e6 counts each for the later two); 4096 random samples of three layers
    checked one by one (sample and both cells)."""
    _print_case("C3 full")
    n, M = 30, 10_000_000
    spec = synth.bm_model(2, n, T=1.0, rho=0.3)
    grid, N = synth.layer_grids(spec, [1] + [(40, 50)] * n, base=_lloyd)
    plan = _plan(spec, grid, N)
    counts = plan.transitions(M, synth.SEED_BASE)
    got = counts.cpu().numpy()
    off = plan.count_offsets()
    sums = np.add.reduceat(got.astype(np.int64), off[:-1])
    assert np.all(sums == M)
    mdl = _omodel(spec)
    poff = plan.point_offsets()
    rng = np.random.default_rng(3)
    for k in (0, 15, n - 1):
        ms = np.sort(rng.choice(M, 4096, replace=False))
        for m in ms[:64]:
            gx, gy = qt.layer_samples(plan, k, int(m), 1, seed=synth.SEED_BASE)
            ox, oy = O.layer_pair(mdl, k, int(m), synth.SEED_BASE)
            assert np.array_equal(gx.cpu().numpy()[0].view(np.uint32), ox.view(np.uint32))
            assert np.array_equal(gy.cpu().numpy()[0].view(np.uint32), oy.view(np.uint32))
        xs = np.stack([O.layer_pair(mdl, k, int(m), synth.SEED_BASE)[0] for m in ms])
        ys = np.stack([O.layer_pair(mdl, k, int(m), synth.SEED_BASE)[1] for m in ms])
        gk = grid[poff[k]:poff[k + 1]]
        gk1 = grid[poff[k + 1]:poff[k + 2]]
        ci = qt.cells(plan, k, torch.from_numpy(xs).cuda()).cpu().numpy()
        cj = qt.cells(plan, k + 1, torch.from_numpy(ys).cuda()).cpu().numpy()
        assert np.array_equal(ci, O.cells_bulk(gk, 2, xs))
        assert np.array_equal(cj, O.cells_bulk(gk1, 2, ys))
        # every sampled transition is present in the counts
        blk = got[off[k]:off[k + 1]].reshape(N[k], N[k + 1])
        assert np.all(blk[ci, cj] > 0)
    for k in (0, 15, n - 1):
        ref = O.layer_counts_one(mdl, grid, N, k, M, seed=synth.SEED_BASE, nthreads=THREADS)
        assert np.array_equal(got[off[k]:off[k + 1]].reshape(N[k], N[k + 1]), ref), k


def test_chunked_accumulation_equals_one_call(small_case):
    """Counts over [0, M) == counts over [0, M1) plus [M1, M) added on top
    (resume by sample chunk), in both counting schemes."""
    name, spec, grid, N, plan = small_case
    for count in (1, 2):
        plan.tune(count=count)
        for mode in (0, 1):
            whole = plan.transitions(90_001, 31, mode=mode).cpu().numpy()
            c = plan.transitions(33_333, 31, mode=mode)
            plan.transitions_add(c, 90_001 - 33_333, 31, mode=mode, m0=33_333)
            assert np.array_equal(c.cpu().numpy(), whole), (name, mode, count)
    plan.tune(count=0)


def test_two_pass_tiny_scratch_many_passes():
    """A plan whose workspace holds 5000 samples per layer runs a larger M in
    many counting passes (odd m0), with identical counts; the trace event is
    recorded after the sampling pass."""
    _print_case("two-pass tiny scratch")
    for d, shapes in ((1, [1, 120, 130, 40]), (2, [1, (9, 9), (10, 11), (5, 5)])):
        spec = synth.bm_model(d, 3, rho=0.2)
        grid, N = synth.layer_grids(spec, shapes)
        plan = qt.Plan(spec, grid, N, batch_samples=5000)
        assert 0 < plan.batch_samples < 20_000
        ref = O.transitions(_omodel(spec), grid, N, 61_111, seed=5, m0=1, nthreads=THREADS)
        for groups in (1, 3):                # histograms on the plan's stream when 3
            plan.tune(groups=groups)
            ev = torch.cuda.Event(enable_timing=True)
            plan.trace(ev)
            got = plan.transitions(61_111, 5, m0=1).cpu().numpy()
            plan.trace(None)
            assert ev.query()
            assert np.array_equal(got, ref), (d, groups)


def test_payoff_batch_matches_single():
    spec = synth.bm_model(2, 4, rho=0.1)
    grid, N = synth.layer_grids(spec, [1, (5, 5), (6, 6), (7, 7), (8, 8)])
    plan = _plan(spec, grid, N)
    rng = np.random.default_rng(2)
    n = 40
    kinds = rng.integers(0, 4, n)
    S0, K = rng.uniform(80, 120, n), rng.uniform(80, 120, n)
    r, T = rng.uniform(0, 0.1, n), rng.uniform(0.25, 2, n)
    sig = rng.uniform(0.1, 0.4, (n, 2))
    mix = np.tril(rng.uniform(-1.0, 1.5, (n, 2, 2)))
    for mx in (None, mix):
        batch = plan.payoff_batch(kinds, S0, K, r, T, sig, mix=mx).cpu().numpy()
        for q in range(n):
            ref = O.payoff(int(kinds[q]), 2, N, grid, S0[q], K[q], r[q], T[q], sig[q],
                           mix=None if mx is None else mx[q])
            fin = np.isfinite(ref)
            assert np.array_equal(fin, np.isfinite(batch[q]))
            assert np.allclose(batch[q][fin], ref[fin], rtol=1e-13, atol=1e-12)


def test_two_pass_several_batches():
    """More samples than one scratch batch holds (2^22 per layer): the count
    tiles accumulate over batches; odd m0 splits a Philox pair at every batch
    boundary."""
    _print_case("two-pass batches")
    spec = synth.bm_model(1, 2)
    grid, N = synth.layer_grids(spec, [1, 300, 700])
    plan = _plan(spec, grid, N)
    mdl = _omodel(spec)
    M, m0 = 9_000_001, 3
    got = plan.transitions(M, 77, m0=m0).cpu().numpy()
    ref = O.transitions(mdl, grid, N, M, seed=77, m0=m0, nthreads=THREADS)
    assert np.array_equal(got, ref)


def test_pi_quarter_disc_counts_match_oracle():
    """The generator experiment of Table rngs: the GPU count of points in the
    quarter disc equals the oracle's, repetition by repetition (integers)."""
    _print_case("pi quarter disc")
    npts = 2_000_000
    got = qt.pi_quarter_disc(0x5EED0000, 3, 4, npts).cpu().numpy()
    for r in range(4):
        ref = O.pi_estimate(0x5EED0000, 3 + r, npts) * npts / 4.0
        assert got[r] == int(round(ref)), r
    small = qt.pi_quarter_disc(7, 0, 1, 2).cpu().numpy()
    assert small[0] == int(round(O.pi_estimate(7, 0, 2) * 2 / 4.0))
    with pytest.raises(qt.QtreeError):
        qt.pi_quarter_disc(7, 0, 1, 3)                    # odd count of points


def test_zero_midpoint_and_signed_zero_samples():
    """A midpoint that rounds to -0 (grid point -2^-149 next to 0) and samples
    that are exactly +0 or -0 (no noise, mean 0): the search counts the
    midpoints strictly below the sample, so a signed zero never counts as
    below the other zero."""
    _print_case("zero midpoint / signed zero samples")
    n = 3
    spec = synth.bm_model(1, n, T=1.0)
    spec["L"] = np.zeros_like(spec["L"])
    spec["T"] = np.zeros_like(spec["T"])
    # mean -0: fma(0, z, -0) is -0 for z < 0 and +0 for z > 0
    spec["mu"] = np.full_like(spec["mu"], -0.0)
    spec["b"] = np.full_like(spec["b"], -0.0)
    tiny = np.float32(np.ldexp(1.0, -149))
    layer = np.array([-tiny, 0.0, 1.0], np.float32)
    assert np.float32(0.5) * (layer[0] + layer[1]) == 0.0
    assert np.signbit(np.float32(0.5) * (layer[0] + layer[1]))
    grid = np.concatenate([[0.0], layer, layer, layer]).astype(np.float32).reshape(-1, 1)
    N = np.array([1, 3, 3, 3], np.int32)
    plan = qt.Plan(spec, grid, N)
    counts = plan.transitions(40_001, 0x5EED0011).cpu().numpy()
    ref = O.transitions(_omodel(spec), grid, N, 40_001, seed=0x5EED0011)
    assert np.array_equal(counts, ref)
    # every sample sits at a zero, below no midpoint: all mass in cell 0 -> 0
    assert counts[0] == 40_001 and counts[1:3].sum() == 0


@pytest.mark.parametrize("name", ["bm1", "bm2"])
def test_autotune_choice_and_every_candidate_give_the_same_counts(name):
    """qtree_plan_autotune times the candidate layer-group / tail /
    samples-per-lane configurations and keeps one; the counts under the
    chosen and under every candidate equal the oracle's."""
    _print_case(f"plan autotune {name}")
    spec = MODELS[name]()
    grid, N = synth.layer_grids(spec, SHAPES[name])
    plan = _plan(spec, grid, N)
    M, seed = 90_001, 0x5EED0071
    ref = O.transitions(_omodel(spec), grid, N, M, seed=seed, contract=3, nthreads=THREADS)
    got = plan.autotune(M, seed=seed)
    assert got["ms"] > 0.0
    assert np.array_equal(plan.transitions(M, seed, contract=3).cpu().numpy(), ref)
    cands = ([(1, 100, 8)] + [(g, t, 8) for g in (2, 4, 6, 8) for t in (100, 50, 33)]
             if spec["d"] == 1 else [(g, 100, s) for s in (8, 4) for g in (1, 2)])
    assert (got["groups"], got["tail"], got["nd_samples"]) in cands
    for g, t, s in cands:
        plan.tune(groups=g, tail=t, nd_samples=s)
        assert np.array_equal(plan.transitions(M, seed, contract=3).cpu().numpy(), ref), (g, t, s)
