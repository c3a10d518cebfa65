"""GPU checks of the batched path: many uneven contracts in one persistent
launch give the same counts (bit-exact) and values as one plan at a time;
graph replays reproduce the eager run; scratch groups and the tuner cache."""
import os

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1101_3228_amd as qt  # noqa: E402


def _contracts(count, shrink, M, seed=7):
    specs = synth.batch_contracts(count, seed=seed, M=M, shrink=shrink)
    items = []
    for i, sp in enumerate(specs):
        model = synth.bm_model(sp["d"], sp["n"], T=sp["T"], rho=sp["rho"])
        grid, N = synth.layer_grids(model, sp["sizes"])
        plan = qt.Plan(model, grid, N, batch_samples=1)
        kinds = [qt.PUT, qt.PUT | qt.EUROPEAN] if sp["d"] == 1 else [qt.MAX_CALL]
        phi = torch.stack([plan.payoff(k, 100.0, 100.0 * sp["K_over_S0"], sp["r"], sp["T"],
                                       [sp["sigma"], sp["sigma"] * 1.2]) for k in kinds])
        items.append(dict(plan=plan, M=sp["M"], seed=synth.SEED_BASE + i, contract_id=i,
                          counts=plan.new_counts(), phi=phi, V=torch.empty_like(phi),
                          model=model, grid=grid, N=N))
    return items


def _single(items):
    ref_counts, ref_v0 = [], []
    for it in items:
        plan = it["plan"]
        c = plan.transitions(it["M"], it["seed"], contract=it["contract_id"])
        V0, _ = plan.bdp(c, it["phi"])
        ref_counts.append(c.cpu().numpy().copy())
        ref_v0.append(V0)
    return ref_counts, np.concatenate(ref_v0)


def test_batch_equals_one_plan_at_a_time():
    print("[gpu-case] batch vs single", flush=True)
    items = _contracts(12, shrink=0.12, M=60_001)
    ref_counts, ref_v0 = _single(items)
    batch = qt.Batch(items)
    info = batch.info()
    assert info["units"] >= sum(it["plan"].n for it in items)
    V0 = batch.run()
    for it, rc in zip(items, ref_counts):
        assert np.array_equal(it["counts"][:it["plan"].entries].cpu().numpy(), rc)
    assert np.allclose(V0, ref_v0, rtol=1e-12, atol=0)
    assert info["per_cu_1d"] >= 1 and info["per_cu_nd"] >= 1
    # batches of one dimension only (the other sampling launch is empty)
    for sub in (slice(0, None, 2), slice(1, None, 2)):
        part = items[sub]
        for it in part:
            it["counts"].fill_(-1)
        V0p = qt.Batch(part).run()
        for it, rc in zip(part, ref_counts[sub]):
            assert np.array_equal(it["counts"][:it["plan"].entries].cpu().numpy(), rc)
        off = np.cumsum([0] + [it["phi"].shape[0] for it in items])
        want = np.concatenate([ref_v0[off[i]:off[i + 1]] for i in range(len(items))[sub]])
        assert np.allclose(V0p, want, rtol=1e-12, atol=0)
    # and against the oracle for two contracts (one 1-D, one 2-D)
    for it in items[:2]:
        sp = it["model"]
        mdl = O.Model(sp["d"], sp["n"], sp["A"], sp["b"], sp["T"], sp["mu"], sp["L"], sp["x0"])
        ref = O.transitions(mdl, it["grid"], it["N"], it["M"], seed=it["seed"],
                            contract=it["contract_id"], nthreads=8)
        assert np.array_equal(it["counts"][:it["plan"].entries].cpu().numpy(), ref)


@pytest.mark.parametrize("case", ["tables_off", "with_3d"])
def test_batch_scan_launches_equal_one_plan_at_a_time(case):
    """The d >= 2 launch without the bucketed search, whose LDS block holds
    the scan's grid records rather than (x, y) pairs: 2-D contracts whose
    plans have the bucket tables turned off, and a batch that adds 3-D
    contracts to the 2-D ones.  Counts bit-exact and values to 1e-12 against
    one plan at a time, under both samples-per-lane settings."""
    print(f"[gpu-case] batch scan launch, {case}", flush=True)
    items = _contracts(6, shrink=0.12, M=40_001, seed=21)
    if case == "tables_off":
        for it in items:
            if it["model"]["d"] == 2:
                it["plan"].tune(buckets=0)
    else:
        for j, sizes in enumerate(([1, (3, 3, 3), (4, 4, 4), (4, 5, 5)],
                                   [1, (2, 3, 5), (5, 5, 5)])):
            model = synth.bm_model(3, len(sizes) - 1, T=1.0, rho=-0.2)
            grid, N = synth.layer_grids(model, sizes)
            plan = qt.Plan(model, grid, N, batch_samples=1)
            phi = torch.stack([plan.payoff(qt.MAX_CALL, 100.0, 100.0, 0.05, 1.0,
                                           [0.2, 0.25, 0.3])])
            items.append(dict(plan=plan, M=40_001, seed=synth.SEED_BASE + 100 + j,
                              contract_id=100 + j, counts=plan.new_counts(), phi=phi,
                              V=torch.empty_like(phi), model=model, grid=grid, N=N))
    ref_counts, ref_v0 = _single(items)
    batch = qt.Batch(items)
    for code in (0, 1):  # 8, then 4 samples per lane in the d >= 2 launch
        batch.set_config(code)
        for it in items:
            it["counts"].fill_(-1)
        V0 = batch.run()
        for it, rc in zip(items, ref_counts):
            assert np.array_equal(it["counts"][:it["plan"].entries].cpu().numpy(), rc), code
        assert np.allclose(V0, ref_v0, rtol=1e-12, atol=0), code


def test_batch_scratch_groups_and_graph_replay(tmp_path):
    print("[gpu-case] batch groups + graph", flush=True)
    items = _contracts(9, shrink=0.1, M=40_000, seed=11)
    ref_counts, ref_v0 = _single(items)
    tuner = qt.Tuner(str(tmp_path / "tune.txt"))
    stream = torch.cuda.Stream()
    batch = qt.Batch(items, tuner=tuner, scratch_bytes=3 << 20, graph=True)
    assert batch.info()["groups"] > 1
    for rep in range(4):
        for it in items:                      # eager work between replays
            it["counts"].fill_(-1)
            it["V"].fill_(0.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            V0 = batch.run(stream=stream)
        for it, rc in zip(items, ref_counts):
            assert np.array_equal(it["counts"][:it["plan"].entries].cpu().numpy(), rc), rep
        assert np.allclose(V0, ref_v0, rtol=1e-12, atol=0), rep
    # the first run timed every candidate and kept the fastest
    tu = batch.tuning()
    assert tu["timed"] >= 2 and tu["ms"] > 0.0
    assert tuner.lookup(batch.signature) == tu["config"]
    assert os.path.exists(tmp_path / "tune.txt")
    again = qt.Tuner(str(tmp_path / "tune.txt"))
    assert again.lookup(batch.signature) == tu["config"]
    # a batch of the same shape takes the cached choice without timing
    same = qt.Batch(items, tuner=again, scratch_bytes=3 << 20)
    same.run()
    t2 = same.tuning()
    assert t2["config"] == tu["config"] and t2["timed"] == 0
    assert t2["ms"] == pytest.approx(tu["ms"], rel=1e-5)


def test_batch_counts_identical_under_every_configuration():
    """Every configuration the tuner may pick (samples per lane 8 / 4,
    serial or overlapped sampling launches, a capped occupancy) gives the
    same counts and values, eagerly and in a replayed graph."""
    print("[gpu-case] batch configurations", flush=True)
    items = _contracts(10, shrink=0.12, M=50_001, seed=13)
    ref_counts, ref_v0 = _single(items)
    batch = qt.Batch(items, graph=True)
    cap = max(1, batch.info()["per_cu_nd"] - 1)
    stream = torch.cuda.Stream()
    for code in (0, 1, 2, 3, cap << 8, (cap << 8) | 3):
        batch.set_config(code)
        assert batch.tuning()["config"] == code
        for rep in range(2):                  # the eager run, then a replay
            for it in items:
                it["counts"].fill_(-1)
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                V0 = batch.run(stream=stream)
            for it, rc in zip(items, ref_counts):
                assert np.array_equal(it["counts"][:it["plan"].entries].cpu().numpy(), rc), code
            assert np.allclose(V0, ref_v0, rtol=1e-12, atol=0), code
    with pytest.raises(qt.QtreeError):
        batch.set_config(1 << 20)


@pytest.mark.timeout(900)
def test_c4_full_batch_equals_one_plan_at_a_time():
    """The full batched workload: 256 contracts (d alternating 1 / 2, n in
    [10, 100], N_k in [50, 2000], M = 1e6 pairs per layer each, two payoffs
    each), one batched run.  Every contract's counts equal a single-plan
    forward bit for bit (compared on the device), every V_0 agrees within
    1e-12 relative, and the cheapest 1-D and 2-D contracts equal the oracle."""
    print("[gpu-case] C4 full batch", flush=True)
    specs = synth.batch_contracts(256, M=1_000_000)
    qcache = {}

    def q(Nv):
        if Nv not in qcache:
            qcache[Nv] = qt.gauss_quantizer(Nv)
        return qcache[Nv]
    items = []
    for i, sp in enumerate(specs):
        model = synth.bm_model(sp["d"], sp["n"], T=sp["T"], rho=sp["rho"])
        grid, N = synth.layer_grids(model, sp["sizes"], base=q)
        plan = qt.Plan(model, grid, N, batch_samples=1)
        kinds = [qt.PUT, qt.PUT | qt.EUROPEAN] if sp["d"] == 1 else \
            [qt.MAX_CALL, qt.MAX_CALL | qt.EUROPEAN]
        phi = plan.payoff_batch(kinds, 100.0, 100.0 * sp["K_over_S0"], sp["r"], sp["T"],
                                [[sp["sigma"], sp["sigma"] * 1.2]] * 2)
        items.append(dict(plan=plan, M=sp["M"], seed=synth.SEED_BASE + i, contract_id=i,
                          counts=plan.new_counts(), phi=phi, V=torch.empty_like(phi),
                          model=model, grid=grid, N=N, d=sp["d"]))
    batch = qt.Batch(items, scratch_bytes=40 << 30)
    V0 = batch.run()
    print(f"[gpu-case] C4 batch ran: {batch.info()}", flush=True)
    tmp = torch.empty(max(it["plan"].entries for it in items) + 4, dtype=torch.int32,
                      device="cuda")
    at = 0
    big2d = 0
    for it in items:
        plan, e = it["plan"], it["plan"].entries
        c = plan.transitions(it["M"], it["seed"], contract=it["contract_id"], counts=tmp)
        assert torch.equal(c[:e], it["counts"][:e]), it["contract_id"]
        v, _ = plan.bdp(c, it["phi"])
        assert np.allclose(V0[at:at + v.size], v, rtol=1e-12, atol=0), it["contract_id"]
        at += v.size
        big2d += it["d"] == 2 and int(np.max(it["N"])) >= 1000
    assert big2d >= 10
    cost = [(it["plan"].n * int(np.max(it["N"])) ** it["d"], j) for j, it in enumerate(items)]
    for dim in (1, 2):
        j = min(cj for cj in cost if items[cj[1]]["d"] == dim)[1]
        it = items[j]
        sp = it["model"]
        mdl = O.Model(sp["d"], sp["n"], sp["A"], sp["b"], sp["T"], sp["mu"], sp["L"], sp["x0"])
        ref = O.transitions(mdl, it["grid"], it["N"], it["M"], seed=it["seed"],
                            contract=it["contract_id"], nthreads=16)
        assert np.array_equal(it["counts"][:it["plan"].entries].cpu().numpy(), ref), j


def test_batch_plan_allocation_failures(monkeypatch):
    """QTREE_FAULT_ALLOC=k makes the k-th device allocation of
    qtree_batch_plan fail: every k up to the eight allocations of a batch
    with both kinds of contract returns ENOMEM and no batch; with the
    variable unset the same contracts plan and run to the counts of one plan
    at a time."""
    print("[gpu-case] batch forced allocation failures", flush=True)
    items = _contracts(4, shrink=0.08, M=20_000, seed=21)
    ref_counts, ref_v0 = _single(items)
    for k in range(1, 9):
        monkeypatch.setenv("QTREE_FAULT_ALLOC", str(k))
        with pytest.raises(qt.QtreeError) as err:
            qt.Batch(items)
        assert err.value.status == 2, k
    monkeypatch.delenv("QTREE_FAULT_ALLOC")
    for it in items:
        it["counts"].fill_(-1)
    V0 = qt.Batch(items).run()
    for it, rc in zip(items, ref_counts):
        assert np.array_equal(it["counts"][:it["plan"].entries].cpu().numpy(), rc)
    assert np.allclose(V0, ref_v0, rtol=1e-12, atol=0)
