"""Benchmark: Monte Carlo transition samples per second of the quantization-tree
forward step on one MI355X, with the FP64 backward step of a contract sweep.

Workload (one step): 1-D Brownian state (standardized log-price of the
Black-Scholes put), n = 50 layers of N = 500 Lloyd-optimal points, M = 1e7
pairs (X_k, X_{k+1}) per layer sampled time-layer parallel (Algorithm III),
counts rebuilt from scratch, then the obstacles and the quantized BDP for 12
American puts sharing the counts (sigma in {0.1, 0.2, 0.3, 0.4} x K/S0 in
{0.8, 1.0, 1.2}).  Inputs (grids, model, contract parameters) are resident on
the GPU before timing starts.  Steps are pipelined: the obstacles and BDP of
step s run on a second stream while step s+1 samples (counts are double
buffered), as a stream of pricing requests would.  The value is pairs per
second over whole steps, every step's BDP included.

Prints one JSON line.  Roofline of the dominant kernel (the sampling pass,
fwd_keys_1d_guide): algorithmic VALU lane-slots per pair (the fixed arithmetic of
one pair, see ALG_SLOTS_PER_PAIR) times the pairs of one step, divided by the
time of the step's sampling launches measured with HIP events on their
stream (from the start of the step to a trace event the library records
after the last of them; the 1-D forward runs its layers in 4 groups, one
sampling launch each, back to back on that stream, with the histogram
passes on a second stream), against the MI355X VALU peak of 256 CUs x 128
lanes x 2.4 GHz lane-slots per second (the FP32 vector rate of 157.3 TFLOP/s
at 2 flops per FMA lane).  `traffic` is the HBM bytes of the same
launches per step from the committed counter profile.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def log(msg: str) -> None:
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_LAYERS, N_POINTS, M_PAIRS = 50, 500, 10_000_000
SIGMAS = (0.1, 0.2, 0.3, 0.4)
K_RATIOS = (0.8, 1.0, 1.2)
S0, RATE, MATURITY = 100.0, 0.05, 1.0

# ALU roofline.  Peak: 256 CUs x 128 lanes x 2.4 GHz = 78.6e12 lane-slots/s,
# the published FP32 vector rate (157.3 TFLOP/s at 2 flops per FMA lane).
# gfx950 issues all-VGPR FP32 fma/add/mul, integer add/sub, bitwise ops and
# right shifts at up to 128 lanes per clock per CU (measured 104-117), every
# other VALU op (compares, selects, min/max, left shifts, 3-input and 32x32
# multiplies, conversions, FP64) at 64 (58-63), and FP32 transcendentals at
# 32 (profiles/valu_op_rates.md).  An algorithmic operation is therefore
# priced at its issue cost in slots of the 128-lane peak: F = 1 for the
# full-rate class, H = 2 for the half-rate class, TR = 4 for a
# transcendental (in mixes a half-rate op measured between 1.3 and 2.3 slots:
# min + add 110 lanes/clock, mad_u64 + xor 78).  The operations counted are
# those the method needs, each in its cheapest gfx950 form; sorting keys for
# the count is not counted (the paper's count is one atomic increment).
F, H, TR = 1, 2, 4
# Philox4x32-10, one call: 10 rounds x (two 32x32->64 products, four xors)
PHILOX_CALL = 10 * (2 * H + 4 * F)                                       # 80
# ln(K 2^-24) by the fixed FP32 sequence: word split (shift, +1) 2F, convert
# H, exponent (shift, bias) 2F, mantissa (and, or) 2F, fold (compare, two
# selects) 3H, t F, Horner 12F, t^2 and r 2F, e - 24 and convert F + H,
# Cody-Waite 2F
LN_U24 = 2 * F + H + 2 * F + 2 * F + 3 * H + F + 12 * F + 2 * F + F + H + 2 * F  # 34
# correctly rounded sqrt: v_sqrt TR, predecessor F, successor F, two
# residual fmas 2F, two sign shifts 2F, two adds 2F
SQRT_RN = TR + F + F + 2 * F + 2 * F + 2 * F                             # 12
# sin and cos of 2 pi J 2^-24: word and quadrant splits 3F, reflection
# (compare, subtract, select) 2H + F, convert and scale H + F, y^2 F, sine
# 5F, cosine 5F, swap 2H, quadrant (and, compare, two selects) F + 3H, sign
# words (and, shift; add, and, shift) 3F + 2H, sign xors 2F
SINCOS = 3 * F + 2 * H + F + H + F + F + 5 * F + 5 * F + 2 * H + F + 3 * H + 3 * F + 2 * H + 2 * F  # 42
BOX_MULLER = LN_U24 + F + SQRT_RN + SINCOS + 2 * F                       # 91
KEY_INCR = H + F          # flat count index i N_{k+1} + j, one count increment
# 1-D guide-table search with K candidate midpoints: bucket fma F, clamp
# (med3) H, convert H, table and candidate addresses 2H, K x (subtract,
# sign shift, add) 3F
def guide_search(K: int) -> int:
    return F + H + H + 2 * H + 3 * F * K
# breadth-first binary search, per step: subtract, shift, and, add (4F) and
# the shift-add of the child address (H)
BFS_STEP = 4 * F + H
# d >= 2 exact argmin, per grid point and sample: two fmas 2F and half of a
# 3-input minimum H/2
ND_POINT = 2 * F + H / 2                                                 # 3
# One 1-D pair at N = 500 (the guide tables of these grids add K = 2
# midpoints per bucket): half a Philox call, one Box-Muller, three AR(1)
# fmas, two guide searches, index and increment
ALG_SLOTS_PER_PAIR = PHILOX_CALL // 2 + BOX_MULLER + 3 * F + 2 * guide_search(2) + KEY_INCR  # 167
# one d = 2 pair besides its searches: a Philox call, two Box-Muller, the
# AR(1) rows (2 x 2 for X_k, 2 x 4 for X_{k+1}: 12F), index and increment
ALG_SLOTS_2D_PAIR = PHILOX_CALL + 2 * BOX_MULLER + 12 * F + KEY_INCR     # 277
ALG_SLOTS_2D_POINT = ND_POINT
# d = 2 bucketed search (the bucket holding the point lists every grid point
# that can win there), in the issue classes above (compares, selects,
# conversions and 3-input ops at half rate): bucket coordinates (two fmas
# 2F), box test (four compares 4H; their conjunction is scalar), two
# conversions 2H, bucket index (a 24-bit multiply-add H, the layer's offset
# F) and the row address H; per listed candidate: index unpack F, record
# address (shift and add) 2F, key 2F, compare H, best key and index selects
# 2H; a point outside the box or in a full bucket scans all N points (key
# 2F, compare H, two selects 2H).
BUCKET_LOCATE = 2 * F + 4 * H + 2 * H + H + F + H                        # 19
BUCKET_CAND = F + 2 * F + 2 * F + H + 2 * H                              # 11
SCAN_POINT = 2 * F + H + 2 * H                                           # 8
# The same pair with every operation priced 1 (transcendental 4): the
# unweighted count reported beside the weighted one.
ALG_SLOTS_PER_PAIR_UNWEIGHTED = 30 + 71 + 3 + 2 * 11 + 2
PEAK_SLOTS = 256 * 128 * 2.4e9         # lane-slots per second

# Algorithmic VALU lane-slots of one surrogate query (the matrix products run
# on the MFMA units): 768 SiLU = 768 x (3 ops + exp and reciprocal, 4 each)
# = 8448; 512 bias adds (layers 2, 3); 256 head FMAs;
# 256 packed BF16 conversions of the 512 MFMA-layer inputs.
MLP_SLOTS_PER_QUERY = 768 * 11 + 512 + 256 + 256


def _measured_traffic(kernel: str = "fwd_keys_1d_guide"):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    runs (profiles/<kernel>_traffic.json), or None when the kernel's sources
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for src in rec["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
        return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["sha256"] else None
    except (OSError, KeyError, ValueError):
        return None


def _inputs():
    import paper_1101_3228_amd as qt
    import synth
    spec = synth.bm_model(1, N_LAYERS, T=MATURITY)
    base = qt.gauss_quantizer(N_POINTS)
    grid, N = synth.layer_grids(spec, [1] + [N_POINTS] * N_LAYERS, base=lambda n: base)
    return spec, grid, N


def cpu_baseline(spec, grid, N, pairs_per_layer: int):
    """The oracle (plain C, one thread per host core over layers) on a bounded
    sample: every layer with `pairs_per_layer` pairs."""
    import oracle as O
    threads = min(os.cpu_count() or 1, N_LAYERS)
    mdl = O.Model(spec["d"], spec["n"], spec["A"], spec["b"], spec["T"], spec["mu"], spec["L"],
                  spec["x0"])
    t0 = time.perf_counter()
    O.transitions(mdl, grid, N, pairs_per_layer, seed=0x5EED0000, nthreads=threads)
    dt = time.perf_counter() - t0
    pairs = pairs_per_layer * N_LAYERS
    return {"value": pairs / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"all {N_LAYERS} layers x {pairs_per_layer} pairs "
                      f"({pairs:.3g} pairs, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c3", action="store_true",
                    help="default run: skip the 2-D workload's nested line")
    ap.add_argument("--c3-steps", type=int, default=10,
                    help="default run: timed steps of the 2-D workload")
    ap.add_argument("--cpu-pairs", type=int, default=7_000_000,
                    help="pairs per layer in the oracle sample")
    ap.add_argument("--workload", choices=("c2", "c3", "batch", "c5", "c1", "p1", "swing",
                                           "rng", "nn", "lloyd", "strat"),
                    default="c2",
                    help="c2 (default): the 1-D time-layer workload of the headline metric; "
                         "c3: 2-D max-call, n=30, N=2000, M=1e7; batch: 256 uneven "
                         "1-D/2-D contracts, M=1e6 each, one batched run per step; c5: the "
                         "put surrogate, 1e6 queries per step after training on 1e5 tree "
                         "prices; c1: 1-D pathwise put, n=10, N=100, M=1e5 paths (latency); "
                         "p1: the paper's 2-D shape, n=365, N=100/250/500, M=1e5, both "
                         "algorithms, counts copied to the host; swing: the paper's swing "
                         "contract shape, 2-D OU, n=365, N=100 and 500, M=1e5, volume "
                         "constraints (100, 250); rng: the quarter-disc experiment, 500 x "
                         "1e9 Philox points; nn: 36.5M brute-force 2-D searches, N=100/250/500; "
                         "lloyd: randomized Lloyd grid optimization, d=2, N=500, 1e6 samples "
                         "x 20 steps; strat: stratified 1-D counts, the c2 shape with 2e4 "
                         "samples per cell")
    ap.add_argument("--epochs", type=int, default=6000, help="c5 training epochs")
    ap.add_argument("--tail", type=int, default=100,
                    help="c2/c3 with --groups: the last layer group's share in percent")
    ap.add_argument("--groups", type=int, default=0,
                    help="c2/c3: layer groups of the two-pass forward (0: library default)")
    ap.add_argument("--act-terms", type=int, default=1, choices=(1, 2),
                    help="c5: BF16 terms per activation entering the MFMA layers")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES between two device buffers three times (the "
                         "reference kernel for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.ones(args.calibrate_copy // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copied_bytes": src.numel() * 4, "copies": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; the quantization-tree "
                                   "forward step is measured on a single MI355X "
                                   "(multi-GPU sharding is a design note only)"}))
        sys.exit(2)

    if args.workload == "c3":
        return run_c3(args)
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "c5":
        return run_c5(args)
    if args.workload == "c1":
        return run_c1(args)
    if args.workload == "p1":
        return run_p1(args)
    if args.workload == "swing":
        return run_swing(args)
    if args.workload == "rng":
        return run_rng(args)
    if args.workload == "nn":
        return run_nn(args)
    if args.workload == "lloyd":
        return run_lloyd(args)
    if args.workload == "strat":
        return run_strat(args)

    import torch
    import paper_1101_3228_amd as qt

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    spec, grid, N = _inputs()
    plan = qt.Plan(spec, grid, N, device="cuda:0", batch_samples=M_PAIRS)
    assert plan.batch_samples >= M_PAIRS, "counting scratch must hold one layer's samples"
    if args.groups:
        plan.tune(groups=args.groups, tail=args.tail)
        tuning = {"fixed": plan.tuning()}
    else:
        # the library's autotuner picks the layer groups (untimed warm-up)
        tuning = plan.autotune(M_PAIRS, seed=0x5EED00FF)
    contracts = [(s, kr) for s in SIGMAS for kr in K_RATIOS]
    nc = len(contracts)
    kinds = np.full(nc, qt.PUT, np.int32)
    c_S0 = np.full(nc, S0)
    c_K = np.array([S0 * kr for _, kr in contracts])
    c_r = np.full(nc, RATE)
    c_T = np.full(nc, MATURITY)
    c_sig = np.array([[s] for s, _ in contracts])
    counts = [plan.new_counts(), plan.new_counts()]
    phi = [torch.empty((nc, plan.points), dtype=torch.float64, device=dev) for _ in range(2)]
    V = [torch.empty((nc, plan.points), dtype=torch.float64, device=dev) for _ in range(2)]
    s_fwd = torch.cuda.current_stream()
    s_bdp = torch.cuda.Stream()
    fwd_done = [torch.cuda.Event() for _ in range(2)]
    bdp_done = [torch.cuda.Event() for _ in range(2)]
    for e in bdp_done:
        e.record(s_bdp)

    def step(i, ev=None):
        b = i % 2
        s_fwd.wait_event(bdp_done[b])              # counts[b] free again
        if ev is not None:
            ev[0].record(s_fwd)
        done = fwd_done[b] if ev is None else ev[1]
        plan.transitions(M_PAIRS, 0x5EED0000 + i, counts=counts[b], stream=s_fwd)
        done.record(s_fwd)
        s_bdp.wait_event(done)
        plan.payoff_batch(kinds, c_S0, c_K, c_r, c_T, c_sig, out=phi[b], stream=s_bdp)
        plan.bdp(counts[b], phi[b], V=V[b], want_v0=False, stream=s_bdp)
        bdp_done[b].record(s_bdp)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    # per step: start, after the sampling pass (recorded by the library), end
    evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3))
           for _ in range(args.steps)]
    for e in evs:
        e[1].record(s_fwd)          # create the event so its handle can be passed down
    torch.cuda.synchronize()
    t_start.record(s_fwd)
    for i in range(args.steps):
        plan.trace(evs[i][1])
        step(i, (evs[i][0], evs[i][2]))
    plan.trace(None)
    s_fwd.wait_stream(s_bdp)
    t_end.record(s_fwd)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    fwd_ms = float(np.mean([e[0].elapsed_time(e[2]) for e in evs]))
    keys_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    V = V[(args.steps - 1) % 2]
    V0 = V[:, 0].cpu().numpy()
    pairs = N_LAYERS * M_PAIRS
    achieved = ALG_SLOTS_PER_PAIR * pairs / (keys_ms * 1e-3)
    hist = histogram_pass(plan, counts[0], s_fwd, pairs, max(3, args.steps // 4))
    out = {
        "metric": "MC transition samples/s (cell search+count)",
        "value": pairs / (ms_step * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 samples, int32 counts, f64 BDP",
        "data": "synthetic",
        "config": {"workload": "1-D Bermudan put tree, time-layer parallel: n=50 layers, "
                               "N=500 Lloyd points/layer, M=1e7 pairs/layer, "
                               "12-contract sigma x K BDP sweep",
                   "layers": N_LAYERS, "points_per_layer": N_POINTS, "pairs_per_layer": M_PAIRS,
                   "contracts": len(contracts), "mode": "layerwise"},
        "forward_ms": fwd_ms,
        "sampling_pass_ms": keys_ms,
        "histogram_pass_ms": fwd_ms - keys_ms,
        "forward_pairs_per_s": pairs / (fwd_ms * 1e-3),
        "V0_atm_sigma0.2": float(V0[contracts.index((0.2, 1.0))]),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
                     "unit": "Tlane-slot/s", "frac": achieved / PEAK_SLOTS,
                     "traffic": _measured_traffic(),
                     "kernel": "fwd_keys_1d_guide<2, 4>",
                     "alg_slots_per_pair": ALG_SLOTS_PER_PAIR,
                     "frac_unweighted": ALG_SLOTS_PER_PAIR_UNWEIGHTED * pairs
                     / (keys_ms * 1e-3) / PEAK_SLOTS,
                     "alg_slots_per_pair_unweighted": ALG_SLOTS_PER_PAIR_UNWEIGHTED},
        "histogram_pass": hist,
        "tuning": tuning,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, grid, N, args.cpu_pairs)
    del plan, counts, phi, V
    torch.cuda.empty_cache()
    if not args.no_c3:
        log("2-D workload")
        out["c3"] = measure_c3(args.c3_steps, 2, not args.no_cpu_baseline)
    print(json.dumps(out), flush=True)


# LDS atomic peak: one 32-bit atomic per LDS bank per clock, 32 banks per CU
# (128 bytes per clock), 256 CUs at 2.4 GHz.
LDS_ATOMIC_PEAK = 256 * 32 * 2.4e9


def histogram_pass(plan, counts, stream, pairs: int, reps: int) -> dict:
    """The counting pass of the 1-D forward on its own: forwards with one
    layer group, so the sampling launch and the histogram launch follow each
    other on one stream, with the library's trace event between them.  The
    histogram pass does one LDS atomic per pair, reads the 2-byte keys and the
    segment tables and stores the count blocks once."""
    import torch
    plan.tune(groups=1)
    evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(reps + 1)]
    for e in evs:
        e[1].record(stream)
    torch.cuda.synchronize()
    for i, e in enumerate(evs):
        e[0].record(stream)
        plan.trace(e[1])
        plan.transitions(M_PAIRS, 0x5EED0100 + i, counts=counts, stream=stream)
        e[2].record(stream)
    plan.trace(None)
    plan.tune(groups=0)
    torch.cuda.synchronize()
    keys_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs[1:]]))
    hist_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs[1:]]))
    # algorithmic bytes: the 2-byte keys and every chunk's segment table
    # (tiles + 1 words, tiles = ceil(N_k N_{k+1} / 4096)) are read, the
    # count blocks written once
    chunks = (M_PAIRS // 2 + 2048) // 2048
    tiles = (N_POINTS * N_POINTS + 4095) // 4096
    read = 2 * pairs + 4 * N_LAYERS * chunks * (tiles + 1)
    written = 4 * plan.entries
    rate = pairs / (hist_ms * 1e-3)
    return {"ms": hist_ms, "sampling_ms_alone": keys_ms, "lds_atomics_per_s": rate,
            "lds_atomic_peak": LDS_ATOMIC_PEAK, "lds_atomic_frac": rate / LDS_ATOMIC_PEAK,
            "hbm_read_bytes": read, "hbm_written_bytes": written,
            "hbm_GBps": (read + written) / (hist_ms * 1e-3) / 1e9,
            "count_flush_GBps": written / (hist_ms * 1e-3) / 1e9,
            "kernel": "count_tiles (one layer group, one stream)"}


def alg_slots_pair(d: int, Nk: int, Nk1: int, guide_k: int = 2) -> float:
    """Algorithmic lane-slots of one pair from layer k (Nk points) to k+1:
    1-D with guide-table searches adding guide_k midpoints (guide_k < 0: the
    breadth-first binary search of the layers' depths), d = 2 as
    ALG_SLOTS_2D_PAIR plus ND_POINT per grid point of both layers."""
    if d == 1:
        if guide_k >= 0:
            search = 2 * guide_search(guide_k)
        else:
            search = BFS_STEP * sum(max(0, int(np.ceil(np.log2(max(Nv, 1)))))
                                    for Nv in (Nk, Nk1))
        return PHILOX_CALL // 2 + BOX_MULLER + 3 * F + search + KEY_INCR
    return ALG_SLOTS_2D_PAIR + ALG_SLOTS_2D_POINT * (Nk + Nk1)


def bucketed_search_slots(plan, k: int, x, cache: dict | None = None) -> float:
    """Mean algorithmic lane-slots of the d = 2 bucketed search of device
    points x [count, 2] in layer k: the bucket is found in FP32 as the
    kernel finds it, then priced by its listed candidates (not the padding
    to groups of 8); outside the box or in a full bucket, the full scan."""
    lo, sc, B = plan.buckets(k)
    n_k = int(plan.N[k])
    if B[0] == 0:
        return BUCKET_LOCATE + SCAN_POINT * n_k
    if cache is not None and k in cache:
        cnt = cache[k]
    else:
        cnt = plan.bucket_counts(k).astype(np.int64)
        if cache is not None:
            cache[k] = cnt
    xf = x.cpu().numpy().astype(np.float32)
    f = ((xf - lo.astype(np.float32)) * sc.astype(np.float32)).astype(np.float32)
    inside = np.all((f >= 0) & (f < B.astype(np.float32)), axis=1)
    fi = np.where(inside[:, None], f, 0).astype(np.int64)
    c = cnt[fi[:, 0], fi[:, 1]]
    listed = inside & (c != 0xFFFF)
    per = np.where(listed, BUCKET_CAND * c, SCAN_POINT * n_k)
    return BUCKET_LOCATE + float(per.mean())


def bucketed_pair_slots(plan, samples: int = 65_536, seed: int = 0x5EED0C00) -> list:
    """Algorithmic lane-slots of one d = 2 pair from each layer k of the
    plan (ALG_SLOTS_2D_PAIR plus both searches), the searches priced on
    the layer samples 0..samples-1 of the given seed."""
    import paper_1101_3228_amd as qt
    out, cache = [], {}
    for k in range(plan.n):
        xs, ys = qt.layer_samples(plan, k, 0, samples, seed)
        out.append(ALG_SLOTS_2D_PAIR + bucketed_search_slots(plan, k, xs, cache)
                   + bucketed_search_slots(plan, k + 1, ys, cache))
        cache.pop(k, None)
    return out


def _batch_tuning(batch) -> dict:
    """The batch's configuration in use, its code decoded (bit 0: 4 samples
    per lane in the d >= 2 launch, else 8; bit 1: the 1-D launch overlapped
    on a side stream; bits 8-15: a cap on that launch's workgroups per CU)."""
    t = batch.tuning()
    c = t["config"]
    return {**t, "nd_samples": 4 if c & 1 else 8, "overlap": bool(c & 2),
            "nd_cap": (c >> 8) & 0xFF}


C3_LAYERS, C3_SHAPE, C3_M = 30, (40, 50), 10_000_000


def measure_c3(steps: int, warmup: int, with_cpu: bool, groups: int = 0,
               tail: int = 100) -> dict:
    """2-D max-call state, n = 30, N = 2000 (40 x 50 product of Lloyd grids
    mapped by sqrt(t_k) chol(R)), rho = 0.3, M = 1e7 pairs per layer; BDP of
    the American and European max-call (sigma 0.2 / 0.3).  One step = the
    forward (sampling and histogram passes), the obstacles and the BDP,
    pipelined as in the 1-D workload: step s's obstacles and BDP run on a
    second stream while step s+1 samples (counts double-buffered)."""
    import torch
    import paper_1101_3228_amd as qt
    import synth
    torch.cuda.set_device(0)
    n, M = C3_LAYERS, C3_M
    spec = synth.bm_model(2, n, T=MATURITY, rho=0.3)
    grid, N = synth.layer_grids(spec, [1] + [C3_SHAPE] * n, base=qt.gauss_quantizer)
    plan = qt.Plan(spec, grid, N, device="cuda:0", batch_samples=M)
    counts = [plan.new_counts(), plan.new_counts()]
    if groups:
        plan.tune(groups=groups, tail=tail)
        tuning = {"fixed": plan.tuning()}
    else:
        tuning = plan.autotune(M, seed=0x5EED00FF, counts=counts[0])
    dev = counts[0].device
    s_fwd = torch.cuda.current_stream()
    s_bdp = torch.cuda.Stream()
    phi = [torch.empty((2, plan.points), dtype=torch.float64, device=dev) for _ in range(2)]
    Vb = [torch.empty((2, plan.points), dtype=torch.float64, device=dev) for _ in range(2)]
    fwd_done = [torch.cuda.Event() for _ in range(2)]
    bdp_done = [torch.cuda.Event() for _ in range(2)]
    for e in bdp_done:
        e.record(s_bdp)

    def step(i, ev=None):
        b = i % 2
        s_fwd.wait_event(bdp_done[b])              # counts[b] free again
        if ev is not None:
            ev[0].record(s_fwd)
        plan.transitions(M, 0x5EED0000 + i, counts=counts[b], stream=s_fwd)
        done = fwd_done[b] if ev is None else ev[2]
        done.record(s_fwd)
        s_bdp.wait_event(done)
        plan.payoff_batch([qt.MAX_CALL, qt.MAX_CALL | qt.EUROPEAN], S0, S0, RATE, MATURITY,
                          [[0.2, 0.3], [0.2, 0.3]], out=phi[b], stream=s_bdp)
        plan.bdp(counts[b], phi[b], V=Vb[b], want_v0=False, stream=s_bdp)
        bdp_done[b].record(s_bdp)
        return Vb[b]

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(steps)]
    for e in evs:
        e[1].record(s_fwd)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(s_fwd)
    for i in range(steps):
        plan.trace(evs[i][1])
        V = step(i, evs[i])
    plan.trace(None)
    s_fwd.wait_stream(s_bdp)
    t1.record(s_fwd)
    torch.cuda.synchronize()
    ms_step = t0.elapsed_time(t1) / steps
    keys_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    fwd_ms = float(np.mean([e[0].elapsed_time(e[2]) for e in evs]))
    pairs = n * M
    points = sum(int(N[k]) + int(N[k + 1]) for k in range(n)) * M
    bucketed = plan.tuning()["buckets"] > 0
    if bucketed:
        per_layer = bucketed_pair_slots(plan)
        alg = M * float(np.sum(per_layer))
        # the bucketed kernel takes 2 samples per lane and round for the
        # tuning's 8; for 4, one, in its six-waves-per-SIMD instance
        kernel = ("fwd_keys_nd<2, 2, true>" if plan.tuning()["nd_samples"] == 8
                  else "fwd_keys_nd_bk1")
    else:
        alg = ALG_SLOTS_2D_PAIR * pairs + ALG_SLOTS_2D_POINT * points
        kernel = f"fwd_keys_nd<2, {plan.tuning()['nd_samples']}, false>"
    achieved = alg / (keys_ms * 1e-3)
    V0 = V[:, 0].cpu().numpy()
    out = {
        "workload": "2-D max-call tree, time-layer parallel: n=30 layers, N=2000 (40x50 "
                    "Lloyd product) points/layer, M=1e7 pairs/layer",
        "value": pairs / (ms_step * 1e-3), "unit": "pairs/s", "steps": steps,
        "ms_per_step": ms_step, "forward_ms": fwd_ms, "sampling_pass_ms": keys_ms,
        "histogram_pass_ms": fwd_ms - keys_ms,
        "paper_convention_gflops": 6.0 * points / (keys_ms * 1e-3) / 1e9,
        "V0_american_european": [float(V0[0]), float(V0[1])],
        "tuning": tuning,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
                     "unit": "Tlane-slot/s", "frac": achieved / PEAK_SLOTS,
                     "traffic": _measured_traffic("fwd_keys_nd"),
                     "kernel": kernel,
                     "alg_slots_per_pair_avg": alg / pairs},
    }
    if with_cpu:
        import oracle as O
        Mc = 400_000
        threads = min(os.cpu_count() or 1, n)
        mdl = O.Model(spec["d"], spec["n"], spec["A"], spec["b"], spec["T"], spec["mu"],
                      spec["L"], spec["x0"])
        tc = time.perf_counter()
        O.transitions(mdl, grid, N, Mc, seed=0x5EED0000, nthreads=threads)
        dt = time.perf_counter() - tc
        out["cpu_baseline"] = {"value": Mc * n / dt, "unit": "pairs/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"all {n} layers x {Mc} pairs ({Mc * n:.3g} pairs, "
                                         f"{dt:.1f} s)"}
    return out


def run_c3(args):
    """The 2-D workload as its own line (see measure_c3)."""
    r = measure_c3(args.steps, args.warmup, not args.no_cpu_baseline, args.groups, args.tail)
    out = {
        "metric": "MC transition samples/s (cell search+count)",
        "value": r["value"], "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 samples, int32 counts, f64 BDP", "data": "synthetic",
        "config": {"workload": r["workload"], "layers": C3_LAYERS, "points_per_layer": 2000,
                   "pairs_per_layer": C3_M},
    }
    out.update({k: v for k, v in r.items() if k not in ("workload", "value", "unit", "steps",
                                                        "ms_per_step")})
    print(json.dumps(out), flush=True)


def run_batch(args):
    """256 contracts with uneven n in [10, 100] and N_k in [50, 2000], d
    alternating 1 / 2, M = 1e6 pairs per layer each, two payoffs per contract;
    one batched run (sampling launches, histogram launch, BDP launch,
    replayed as a hipGraph) per step."""
    import torch
    import paper_1101_3228_amd as qt
    import synth
    torch.cuda.set_device(0)
    t_prep = time.perf_counter()
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
        plan = qt.Plan(model, grid, N, device="cuda:0", batch_samples=1)
        kinds = [qt.PUT, qt.PUT | qt.EUROPEAN] if sp["d"] == 1 else \
            [qt.MAX_CALL, qt.MAX_CALL | qt.EUROPEAN]
        phi = plan.payoff_batch(kinds, S0, S0 * sp["K_over_S0"], sp["r"], sp["T"],
                                [[sp["sigma"], sp["sigma"] * 1.2]] * 2)
        items.append(dict(plan=plan, M=sp["M"], seed=0x5EED0000 + i, contract_id=i,
                          counts=plan.new_counts(), phi=phi, V=torch.empty_like(phi)))
        if (i + 1) % 32 == 0:
            log(f"prepared {i + 1}/{len(specs)} contracts ({time.perf_counter() - t_prep:.1f} s)")
    tuner = qt.Tuner(os.environ.get("QTREE_TUNE_CACHE"))
    stream = torch.cuda.Stream()
    batch = qt.Batch(items, tuner=tuner, scratch_bytes=40 << 30, graph=True)
    prep_s = time.perf_counter() - t_prep
    log(f"batch planned ({prep_s:.1f} s)")
    with torch.cuda.stream(stream):
        for w in range(max(args.warmup, 2)):     # first run tunes and captures the graph
            batch.run(want_v0=False, stream=stream)
            torch.cuda.synchronize()
            log(f"warm-up run {w + 1} done")
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(args.steps):
            batch.run(want_v0=False, stream=stream)
        t1.record(stream)
        torch.cuda.synchronize()
        V0 = batch.run(want_v0=True, stream=stream)
    ms_step = t0.elapsed_time(t1) / args.steps
    pairs = sum(sp["n"] * sp["M"] for sp in specs)
    options = sum(it["phi"].shape[0] for it in items)
    info = batch.info()
    alg = 0.0
    log("pricing the step's algorithmic work")
    for i, (sp, it) in enumerate(zip(specs, items)):
        if (i + 1) % 64 == 0:
            log(f"priced {i + 1}/{len(specs)} contracts")
        Ns = [int(np.prod(v)) for v in sp["sizes"]]
        if sp["d"] == 2 and it["plan"].tuning()["buckets"] > 0:
            # the batch searches d = 2 contracts through their bucket tables
            alg += sp["M"] * float(np.sum(bucketed_pair_slots(it["plan"], samples=4096)))
        else:
            alg += sp["M"] * sum(alg_slots_pair(sp["d"], Ns[k], Ns[k + 1])
                                 for k in range(sp["n"]))
    achieved = alg / (ms_step * 1e-3)
    out = {
        "metric": "MC transition samples/s (cell search+count); options/s (tree)",
        "value": pairs / (ms_step * 1e-3), "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 samples, int32 counts, f64 BDP", "data": "synthetic",
        "config": {"workload": "batch of 256 contracts, d alternating 1/2, n in [10,100], "
                               "N_k in [50,2000], M=1e6 pairs/layer each, 2 payoffs each",
                   "contracts": len(items), "pairs": pairs, "options": options},
        "options_per_s": options / (ms_step * 1e-3),
        "batch": info, "prep_s": prep_s,
        "tuning": _batch_tuning(batch),
        "V0_mean": float(np.mean(V0)),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
                     "unit": "Tlane-slot/s", "frac": achieved / PEAK_SLOTS, "traffic": None,
                     "kernel": "whole step (batch_keys_nd + batch_keys_1d + batch_count + "
                               "bdp_batch_kernel); the per-kernel split is in the profile"},
    }
    if not args.no_cpu_baseline:
        # the oracle on the host cores over a sample of the contracts: the
        # contracts in order (d alternating) at 1e5 pairs per layer until
        # about 10 s of host time
        import oracle as O
        threads = min(os.cpu_count() or 1, 16)
        Mc, done, t_cpu, used = 100_000, 0, 0.0, 0
        for sp in specs:
            if t_cpu >= 10.0:
                break
            used += 1
            model = synth.bm_model(sp["d"], sp["n"], T=sp["T"], rho=sp["rho"])
            grid, N = synth.layer_grids(model, sp["sizes"], base=q)
            mdl = O.Model(model["d"], model["n"], model["A"], model["b"], model["T"],
                          model["mu"], model["L"], model["x0"])
            tc = time.perf_counter()
            O.transitions(mdl, grid, N, Mc, seed=7, nthreads=threads)
            t_cpu += time.perf_counter() - tc
            done += sp["n"] * Mc
        out["cpu_baseline"] = {"value": done / t_cpu, "unit": "pairs/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"the first {used} contracts (d alternating 1, 2) "
                                         f"at {Mc} pairs per layer: {done:.3g} pairs in "
                                         f"{t_cpu:.1f} s"}
    print(json.dumps(out), flush=True)


def tree_band_fmas(plan, pi) -> int:
    """Multiply-adds of one contract's backward recursion on a tree: the sum
    over the rows of every layer of the width of the row's nonzero band (the
    band table that qtree_pi writes after the layer offsets)."""
    import torch
    n = plan.n
    base, _ = pi._qtree_pi
    off = base - pi.data_ptr()
    band_at = off + ((8 * n + 255) // 256) * 256
    rows = int(plan.point_offsets()[n])
    b = pi[band_at:band_at + 8 * rows].view(torch.int32).view(rows, 2).cpu().numpy()
    return int(np.sum(b[:, 1] - b[:, 0]))


def run_c5(args):
    """The put surrogate (6-256-256-256-1, BF16 weights, two activation
    terms): labels from the tree (N = 100 optimal points per layer, counts
    shared per n, M = 2e6 pairs per layer), training on 1e5 of them (not
    timed), then one step = inference of 1e6 queries of which 5 % lie
    outside the box.  Reported beside it: the tree's options/s on the same
    queries (counts cached), the rate with the out-of-box 5 % sent to the
    tree, and the held-out accuracy."""
    import torch
    import synth
    from paper_1101_3228_amd import surrogate as S
    torch.cuda.set_device(0)
    lo, hi = synth.PUT_BOX_LO, synth.PUT_BOX_HI
    t_prep = time.perf_counter()
    pricer = S.PutTreePricer(N=100, M=2_000_000, device="cuda:0")
    xtr = synth.box_queries(100_000, 0x5EED0000)
    ytr = pricer.price(xtr)
    log(f"labels: {time.perf_counter() - t_prep:.1f} s")
    sur = S.Surrogate(pricer, lo, hi, synth.mlp_init(0x5EED0001), out_scale=0.05,
                      act_terms=args.act_terms, max_batch=4096, baseline=1, device="cuda:0")
    t_fit = time.perf_counter()
    hist = sur.fit(xtr, ytr, epochs=args.epochs, lr=2e-3, lr_final=1e-6,
                   log=lambda e, l: e % 500 == 0 and log(f"epoch {e}: loss {l:.3e}"))
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t_fit
    xte = synth.box_queries(20_000, 0x5EED0002)
    yte = pricer.price(xte)
    yp, _ = sur.price(xte)
    err = np.abs(yp - yte) / np.maximum(yte, 1e-2)

    Q = 1_000_000
    xq = synth.box_queries(Q, 0x5EED0003, frac_out=0.05)
    xd = torch.from_numpy(xq).cuda()
    y = torch.empty(Q, dtype=torch.float32, device="cuda:0")
    mask = torch.empty(Q, dtype=torch.uint8, device="cuda:0")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        sur.net.forward(xd, y, mask, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        sur.net.forward(xd, y, mask, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    value = Q / (ms * 1e-3)
    alg_flop = 2.0 * (6 * 256 + 2 * 256 * 256 + 256)      # per query
    achieved = alg_flop * Q / (ms * 1e-3) / 1e12

    # the tree on the same 1e6 queries: counts and transition weights cached
    # per n, contract records resident on the device; one qtree_bdp_many_trees
    # launch for every n (obstacles computed in the kernel), timed with HIP
    # events
    inside = mask.cpu().numpy().astype(bool)
    groups = pricer.specs(xq)
    vals = pricer.price_specs(groups, stream=stream)
    torch.cuda.synchronize()
    t_ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    t_ev[0].record(stream)
    reps = max(1, args.steps // 5)
    for _ in range(reps):
        pricer.price_specs(groups, out=vals, stream=stream)
    t_ev[1].record(stream)
    torch.cuda.synchronize()
    tree_ms = t_ev[0].elapsed_time(t_ev[1]) / reps
    tree_rate = Q / (tree_ms * 1e-3)
    # FP64 work of the tree side: one multiply-add per weight inside every
    # row's nonzero band, per contract (the band table of qtree_pi)
    band_fma = 0
    for n, rows in zip(groups["n"], groups["rows"]):
        plan, _, pi = pricer.tree(n)
        band_fma += rows.size * tree_band_fmas(plan, pi)
    tree_tflops = 2.0 * band_fma / (tree_ms * 1e-3) / 1e12
    out_groups = pricer.specs(xq[~inside])
    torch.cuda.synchronize()
    f_ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    f_ev[0].record(stream)
    pricer.price_specs(out_groups, stream=stream)
    f_ev[1].record(stream)
    torch.cuda.synchronize()
    fallback_s = f_ev[0].elapsed_time(f_ev[1]) * 1e-3
    blended = Q / (ms * 1e-3 + fallback_s)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import mlp as OM
        p = sur.net.params()
        xs = xq[:20_000]
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < 10.0:
            OM.forward(p, xs, lo, hi, 0.05, terms=args.act_terms, baseline=1)
            reps += 1
        el = time.perf_counter() - t0
        cpu = {"value": reps * xs.shape[0] / el, "unit": "options/s",
               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
               "kind": "oracle",
               "sample": f"FP64 numpy network on 20000 of the queries, {reps} passes"}
    out = {
        "metric": "options/s surrogate vs tree", "value": value, "unit": "options/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 weights, f32 accumulation", "data": "synthetic",
        "config": {"workload": "put surrogate 6-256-256-256-1 (Black-Scholes control "
                               "variate): 1e6 queries (5 % outside the training box) per "
                               "step; trained on 1e5 tree prices (N = 100, M = 2e6 "
                               "pairs/layer, n in [10, 100])",
                   "queries": Q, "act_terms": args.act_terms, "train_rows": int(xtr.shape[0]),
                   "epochs": args.epochs},
        "tree_options_per_s": tree_rate,
        "tree_ms": tree_ms,
        "tree_roofline": {"bound": "fp64", "achieved": tree_tflops, "peak": 78.6,
                          "unit": "TFLOP/s", "frac": tree_tflops / 78.6,
                          "kernel": "bdp_many_kernel (every tree in one launch, all "
                                    "layers, 64 contracts per workgroup; FLOP = 2 x the "
                                    "multiply-adds inside the rows' nonzero bands, obstacles "
                                    "not counted)"},
        "with_fallback_options_per_s": blended,
        "speedup_vs_tree": value / tree_rate,
        "accuracy_r19": {"mean": float(err.mean()), "median": float(np.median(err)),
                         "p99": float(np.quantile(err, 0.99)), "max": float(err.max()),
                         "frac_le_1e-3": float(np.mean(err <= 1e-3))},
        "train_s": fit_s, "final_loss": hist[-1],
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": achieved / 2500.0, "traffic": None,
                     "kernel": f"mlp_forward<{args.act_terms},false>"},
        # what binds this kernel in practice: SiLU on the vector ALUs
        "valu_view": {"alg_slots_per_query": MLP_SLOTS_PER_QUERY,
                      "achieved": MLP_SLOTS_PER_QUERY * value / 1e12,
                      "peak": PEAK_SLOTS / 1e12, "unit": "Tlane-slot/s",
                      "frac": MLP_SLOTS_PER_QUERY * value / PEAK_SLOTS},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def run_c1(args):
    """1-D put, n = 10, N = 100 Lloyd points per layer, M = 1e5 paths
    (pathwise, Algorithm II), S0 = K = 100, sigma = 0.2, r = 0.05, T = 1; one
    step = forward + obstacle + BDP with V_0 on the host (a latency figure)."""
    import torch
    import paper_1101_3228_amd as qt
    import synth
    torch.cuda.set_device(0)
    n, Nn, M = 10, 100, 100_000
    spec = synth.bm_model(1, n, T=1.0)
    grid, N = synth.layer_grids(spec, [1] + [Nn] * n, base=qt.gauss_quantizer)
    plan = qt.Plan(spec, grid, N, device="cuda:0")
    counts = plan.new_counts()
    phi = plan.payoff(qt.PUT, S0, 100.0, RATE, 1.0, 0.2)

    def step(i):
        plan.transitions(M, 0x5EED0000 + i, mode=qt.PATHWISE, counts=counts)
        return plan.bdp(counts, phi)[0]
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        V0 = step(i)
    el = time.perf_counter() - t0
    ms = el * 1e3 / args.steps
    print(json.dumps({
        "metric": "MC transition samples/s (cell search+count)", "value": M * n / (ms * 1e-3),
        "unit": "transitions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 samples, int32 counts, f64 BDP", "data": "synthetic",
        "config": {"workload": "1-D American put, pathwise: n=10, N=100, M=1e5 paths; "
                               "forward + BDP + V0 to host per step (latency bound)"},
        "V0": float(V0[0]), "roofline": None,
        "roofline_note": "1e6 transitions per step: launch latency, not a throughput bound",
    }), flush=True)


def run_p1(args):
    """The paper's own shape (context): 2-D Ornstein-Uhlenbeck state,
    n = 365, N = 100 / 250 / 500 per layer, M = 1e5; time-layer parallel
    (Algorithm III, pairs per layer) and pathwise (Algorithm II); each run
    includes copying the counts to the host, as the paper's timings do."""
    import torch
    import paper_1101_3228_amd as qt
    import synth
    torch.cuda.set_device(0)
    n, M = 365, 100_000
    spec = synth.ou_model(n)
    res = {}
    for Nn in (100, 250, 500):
        grid, N = synth.layer_grids(spec, [1] + [Nn] * n, base=qt.gauss_quantizer)
        plan = qt.Plan(spec, grid, N, device="cuda:0", batch_samples=M)
        counts = plan.new_counts()
        host = torch.empty(counts.shape, dtype=counts.dtype, pin_memory=True)
        for mode, name in ((qt.LAYERWISE, "alg3"), (qt.PATHWISE, "alg2")):
            for i in range(args.warmup):
                plan.transitions(M, 7 + i, mode=mode, counts=counts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(args.steps):
                plan.transitions(M, 7 + i, mode=mode, counts=counts)
                host.copy_(counts)
            torch.cuda.synchronize()
            s_run = (time.perf_counter() - t0) / args.steps
            res[f"{name}_N{Nn}"] = {"s": s_run, "transitions_per_s": M * n / s_run}
        log(f"N={Nn} done")
    cpu = None
    if not args.no_cpu_baseline:
        # the paper's serial figure (Algorithm I on one core): the oracle on
        # one thread, pathwise, the whole N = 100 run (1e5 paths)
        import oracle as O
        grid, N = synth.layer_grids(spec, [1] + [100] * n, base=qt.gauss_quantizer)
        mdl = O.Model(spec["d"], spec["n"], spec["A"], spec["b"], spec["T"], spec["mu"],
                      spec["L"], spec["x0"])
        t0 = time.perf_counter()
        O.transitions(mdl, grid, N, M, seed=7, mode=O.PATHWISE, nthreads=1)
        dt = time.perf_counter() - t0
        cpu = {"value": M * n / dt, "unit": "transitions/s", "cores": 1, "kind": "oracle",
               "sample": f"Algorithm I (pathwise), N = 100, all {M} paths, one thread: "
                         f"{dt:.1f} s (paper, serial, i7 at 2.8 GHz: 30 s)"}
    print(json.dumps({
        "metric": "MC transition samples/s (cell search+count)",
        "value": res["alg3_N500"]["transitions_per_s"], "unit": "transitions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["alg3_N500"]["s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 samples, int32 counts", "data": "synthetic",
        "config": {"workload": "paper shape (context): 2-D OU, n=365, N=100/250/500, M=1e5, "
                               "Algorithms III and II, counts copied to the host per run"},
        "runs": res,
        "paper_context_gtx480_s": {"alg3": {"N100": 0.21, "N250": 0.50, "N500": 0.99},
                                   "alg2": {"N100": 0.11, "N250": 0.30, "N500": 0.63}},
        "roofline": None,
        "cpu_baseline": cpu,
    }), flush=True)


PEAK_FP64 = 78.6e12  # MI355X FP64 vector FLOP/s


def run_swing(args):
    """The swing contract of the paper's own workload shape (Sec. 3): 2-D
    Ornstein-Uhlenbeck factors (alpha = 1 and 5, rho = -0.4), n = 365 daily
    dates, N = 100 (10 x 10) and 500 (20 x 25) points per layer, M = 1e5
    pairs per layer (time-layer parallel), forward on the factor sum
    (sigma = 0.7 / 1.4, S0 = K = 20), volume in [100, 250].  One step =
    forward step + obstacle + swing BDP with P0 on the host."""
    import torch
    import paper_1101_3228_amd as qt
    import synth
    torch.cuda.set_device(0)
    n, M, Qmin, Qmax = 365, 100_000, 100, 250
    spec = synth.ou_model(n, alpha=(1.0, 5.0), sig=(1.0, 1.0), rho=-0.4)
    runs = {}
    for Nn, side in ((100, (10, 10)), (500, (20, 25))):
        grid, N = synth.layer_grids(spec, [1] + [side] * n, base=qt.gauss_quantizer)
        plan = qt.Plan(spec, grid, N, device="cuda:0", batch_samples=M)
        counts = plan.new_counts()
        v = torch.empty(plan.points, dtype=torch.float64, device="cuda:0")
        P = torch.empty((plan.points, Qmax + 1), dtype=torch.float64, device="cuda:0")
        stream = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

        def step(i, timed=False):
            if timed:
                ev[0].record(stream)
            plan.transitions(M, 0x5EED0000 + i, counts=counts)
            plan.payoff_forward(20.0, 20.0, 0.0, 1.0, [0.7, 1.4], out=v)
            if timed:
                ev[1].record(stream)
            p0, _ = plan.swing(counts, v, Qmin, Qmax, P=P, want_p0=False)
            if timed:
                ev[2].record(stream)
        for i in range(args.warmup):
            step(i)
        torch.cuda.synchronize()
        fwd_ms = bdp_ms = 0.0
        t0 = time.perf_counter()
        for i in range(args.steps):
            step(i, timed=True)
            torch.cuda.synchronize()
            fwd_ms += ev[0].elapsed_time(ev[1])
            bdp_ms += ev[1].elapsed_time(ev[2])
        wall = (time.perf_counter() - t0) / args.steps
        P0, _ = plan.swing(counts, v, Qmin, Qmax, P=P)
        nnz = int((counts != 0).sum().item())
        flop = 2.0 * nnz * (Qmax + 1)
        runs[f"N{Nn}"] = {"fwd_ms": fwd_ms / args.steps, "swing_bdp_ms": bdp_ms / args.steps,
                          "step_ms": wall * 1e3, "transitions_per_s": M * n / (fwd_ms / args.steps * 1e-3),
                          "P0": P0, "nnz_counts": nnz,
                          "swing_fp64_frac": flop / (bdp_ms / args.steps * 1e-3) / PEAK_FP64}
        log(f"N={Nn} done")
    r5 = runs["N500"]
    print(json.dumps({
        "metric": "MC transition samples/s (cell search+count)",
        "value": r5["transitions_per_s"], "unit": "transitions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r5["step_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 samples, int32 counts, f64 swing BDP", "data": "synthetic",
        "config": {"workload": "swing contract, paper shape: 2-D OU, n=365, N=100/500, M=1e5 "
                               "pairs/layer, volume in [100, 250]; forward + obstacle + swing BDP"},
        "runs": runs,
        "roofline": {"bound": "alu", "achieved": 2.0 * r5["nnz_counts"] * (Qmax + 1)
                     / (r5["swing_bdp_ms"] * 1e-3) / 1e12, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s (FP64)", "frac": r5["swing_fp64_frac"], "traffic": None,
                     "kernel": "swing_layer_kernel (2 FLOP per nonzero count and volume level)"},
        "paper_context_gtx480_s": {"alg3_estimation": {"N100": 0.21, "N500": 0.99}},
    }), flush=True)


def run_rng(args):
    """The generator comparison of the paper (Table rngs): estimate pi from
    1e9 points in the unit square, 500 repetitions, Philox4x32-10 uniforms."""
    import torch
    import paper_1101_3228_amd as qt
    torch.cuda.set_device(0)
    npts, reps = 1_000_000_000, 500
    inside = torch.zeros(reps, dtype=torch.int64, device="cuda:0")
    qt.pi_quarter_disc(0x5EED0000, 0, 4, npts, inside=inside[:4])     # warm-up
    inside.zero_()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    qt.pi_quarter_disc(0x5EED0000, 0, reps, npts, inside=inside)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    est = 4.0 * inside.cpu().numpy().astype(np.float64) / npts
    # one Philox call + two points x (two shifts 2F, two 48-bit squares as
    # 32x32->64 products 2H, the 64-bit sum 2F, the 64-bit compare H, the
    # count F)
    slots = PHILOX_CALL + 2 * (5 * F + 3 * H)
    achieved = slots * (npts / 2) * reps / (ms * 1e-3)
    print(json.dumps({
        "metric": "Philox points/s (quarter-disc experiment)", "value": npts * reps / (ms * 1e-3),
        "unit": "points/s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "pi from 1e9 points in the unit square, 500 repetitions"},
        "ms_per_1e9_points": ms / reps, "mean": float(est.mean()),
        "std": float(est.std(ddof=1)), "std_theory": float(4 * np.sqrt(np.pi / 4 * (1 - np.pi / 4) / npts)),
        "paper_context_gtx480_s_per_1e9": {"drand48": 0.2562, "MRG32k3a": 0.2573, "XORWOW": 0.2085},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS / 1e12,
                     "unit": "Tlane-slot/s", "frac": achieved / PEAK_SLOTS, "traffic": None,
                     "kernel": f"pi_quarter_disc_kernel ({slots} lane-slots per Philox block)"},
    }), flush=True)


def run_nn(args):
    """The search benchmark of the paper (Table nn): 36.5e6 brute-force
    nearest-neighbour searches of N(0, I_2) points in 2-D grids of N = 100,
    250, 500 points (products of Lloyd quantizers), exact lowest-index argmin."""
    import torch
    import paper_1101_3228_amd as qt
    import synth
    torch.cuda.set_device(0)
    Q = 36_500_000
    rng = np.random.default_rng(0x5EED0000)
    x = torch.from_numpy(rng.standard_normal((Q, 2)).astype(np.float32)).cuda()
    cell = torch.empty(Q, dtype=torch.int32, device="cuda:0")
    out = {}
    for Nn in (100, 250, 500):
        spec = synth.bm_model(2, 1, T=1.0)
        grid, N = synth.layer_grids(spec, [1, Nn], base=qt.gauss_quantizer)
        plan = qt.Plan(spec, grid, N, device="cuda:0")
        qt.cells(plan, 1, x[:1000])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            lib_cells = qt.lib().qtree_cells(plan.handle, 1, x.data_ptr(), Q, cell.data_ptr(),
                                             qt._stream_handle(None))
            assert lib_cells == 0
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        out[f"N{Nn}"] = {"ms": ms, "searches_per_s": Q / (ms * 1e-3),
                         "paper_convention_gflops": 6.0 * Q * Nn / (ms * 1e-3) / 1e9}
        slots = ALG_SLOTS_2D_POINT * Q * Nn / (ms * 1e-3)
    print(json.dumps({
        "metric": "brute-force 2-D nearest-neighbour searches/s", "value": out["N500"]["searches_per_s"],
        "unit": "searches/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": out["N500"]["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "36.5e6 searches of N(0, I) points, grids of N = 100 / 250 / 500"},
        "runs": out, "paper_context_gtx480_s": {"N100": 0.09, "N250": 0.23, "N500": 0.41},
        "roofline": {"bound": "alu", "achieved": slots / 1e12, "peak": PEAK_SLOTS / 1e12,
                     "unit": "Tlane-slot/s", "frac": slots / PEAK_SLOTS, "traffic": None,
                     "kernel": "cells_kernel<2> at N = 500 (3 lane-slots per query and "
                               "grid point: 2 FMA + half of a 3-input min at its issue "
                               "cost)"},
    }), flush=True)


def run_lloyd(args):
    """Grid optimization (Sec. 2, eq. Qerr): randomized Lloyd steps for the
    2-D Gaussian N(0, L L^T), L = chol([[1, 0.3], [0.3, 1]]) (the correlation
    of the 2-D max-call workload), N = 500 points from a 20 x 25 product of
    N(0, 1) quantile grids, 1e6 fresh samples per step, 20 steps."""
    import torch
    import paper_1101_3228_amd as qt
    import synth
    torch.cuda.set_device(0)
    d, N, M, steps = 2, 500, 1_000_000, 20
    L = np.linalg.cholesky(np.array([[1.0, 0.3], [0.3, 1.0]]))
    a, b = synth.quantile_grid_1d(20), synth.quantile_grid_1d(25)
    g0 = (np.stack(np.meshgrid(a, b, indexing="ij"), axis=-1).reshape(-1, 2) @ L.T)
    g0 = g0.astype(np.float32)
    grid = torch.empty((N, d), dtype=torch.float32, device="cuda:0")
    dist = torch.zeros(steps, dtype=torch.float64, device="cuda:0")
    ws = torch.empty(qt.lib().qtree_lloyd_workspace_size(d, N), dtype=torch.uint8, device="cuda:0")
    qt.lloyd(d, g0, L, M, 2, 0x5EED0000, grid=grid, distortion=dist, workspace=ws)  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    qt.lloyd(d, g0, L, M, steps, 0x5EED0000, grid=grid, distortion=dist, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    dd = dist.cpu().numpy()
    value = M * steps / (ms * 1e-3)
    # search + Philox + two Box-Muller + L z (4 fma)
    alg = ALG_SLOTS_2D_POINT * N + PHILOX_CALL + 2 * BOX_MULLER + 4 * F
    out = {
        "metric": "Lloyd samples/s (grid optimization, eq. Qerr)", "value": value,
        "unit": "samples/s", "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": ms / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 samples, int64 cell sums", "data": "synthetic",
        "config": {"workload": "randomized Lloyd, d=2, N=500, N(0, [[1,0.3],[0.3,1]]), "
                               "1e6 samples/step, 20 steps"},
        "distortion_first_last": [float(dd[0]), float(dd[-1])],
        "roofline": {"bound": "alu", "achieved": alg * value / 1e12, "peak": PEAK_SLOTS / 1e12,
                     "unit": "Tlane-slot/s", "frac": alg * value / PEAK_SLOTS, "traffic": None,
                     "kernel": f"lloyd_accum_kernel<2> ({ALG_SLOTS_2D_POINT} lane-slots per "
                               f"sample and grid point + {alg - ALG_SLOTS_2D_POINT * N:.0f} per "
                               "sample)"},
    }
    if not args.no_cpu_baseline:
        import oracle as O
        t0 = time.perf_counter()
        Mc = 200_000
        O.lloyd(d, g0, L, Mc, 1, 0x5EED0000)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": Mc / dt, "unit": "samples/s", "cores": 1,
                               "kind": "oracle", "sample": f"one step of {Mc} samples ({dt:.1f} s)"}
    print(json.dumps(out), flush=True)


# Algorithmic lane-slots of one stratified pair: one Philox call, one
# Box-Muller, the normal quantile's central branch in FP64 (two degree-7
# Horner polynomials, q^2, r, product and the quotient's reciprocal and two
# Newton steps: 45 FP64 operations, each H), u and p (6 FP64 operations, H),
# AR(1) 3F, one guide search (K = 2), index and increment.
ALG_SLOTS_STRAT = PHILOX_CALL + BOX_MULLER + 45 * H + 6 * H + 3 * F + guide_search(2) + KEY_INCR


def run_strat(args):
    """Stratified time-layer counts on the 1-D workload's shape (n = 50,
    N = 500 Lloyd points per layer), proportional allocation of 1e7 samples
    per layer (every row exact to its sample count); the plain time-layer
    forward on the same plan and budget is timed beside it, and both price
    the at-the-money put; the spread of that price over 8 seeds is compared
    at a budget of 2e5 samples per layer (plain, proportional, equal)."""
    import torch
    import paper_1101_3228_amd as qt
    torch.cuda.set_device(0)
    spec, grid, N = _inputs()
    plan = qt.Plan(spec, grid, N, device="cuda:0")
    Mk = M_PAIRS
    pairs = sum(plan.strat_row(k, i, Mk, 1) for k in range(N_LAYERS) for i in range(N[k]))
    c_s = plan.new_counts()
    c_p = plan.new_counts()
    plan.transitions_stratified(Mk, 0x5EED0000, counts=c_s)
    plan.transitions(M_PAIRS, 0x5EED0000, counts=c_p)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        plan.transitions_stratified(Mk, 0x5EED0000, counts=c_s)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    e0.record()
    for _ in range(args.steps):
        plan.transitions(M_PAIRS, 0x5EED0000, counts=c_p)
    e1.record()
    torch.cuda.synchronize()
    ms_plain = e0.elapsed_time(e1) / args.steps
    phi = plan.payoff(qt.PUT, S0, S0, RATE, MATURITY, 0.2)
    # spread of the at-the-money put over seeds at 2e5 samples per layer
    # (not timed)
    spread = {"plain": [], "proportional": [], "equal": []}
    for r in range(8):
        seed = 0x5EED0100 + r
        plan.transitions(200_000, seed, counts=c_p)
        spread["plain"].append(float(plan.bdp(c_p, phi)[0][0]))
        plan.transitions_stratified(200_000, seed, alloc=1, counts=c_s)
        spread["proportional"].append(float(plan.bdp(c_s, phi)[0][0]))
        plan.transitions_stratified(200_000 // N_POINTS, seed, alloc=0, counts=c_s)
        spread["equal"].append(float(plan.bdp(c_s, phi)[0][0]))
    plan.transitions_stratified(Mk, 0x5EED0000, counts=c_s)
    plan.transitions(M_PAIRS, 0x5EED0000, counts=c_p)
    V_s, _ = plan.bdp(c_s, phi)
    V_p, _ = plan.bdp(c_p, phi)
    value = pairs / (ms * 1e-3)
    out = {
        "metric": "MC transition samples/s (stratified, 1-D)", "value": value,
        "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 samples, f64 quantile, int32 counts", "data": "synthetic",
        "config": {"workload": "stratified 1-D time-layer counts, n=50, N=500 Lloyd points, "
                               "proportional allocation of 1e7 samples per layer"},
        "plain_forward_ms_same_pairs": ms_plain,
        "V0_atm_put_sigma0.2": {"stratified": float(V_s[0]), "plain": float(V_p[0])},
        "V0_std_over_8_seeds_at_2e5_per_layer": {k: float(np.std(v, ddof=1))
                                                  for k, v in spread.items()},
        "roofline": {"bound": "alu", "achieved": ALG_SLOTS_STRAT * value / 1e12,
                     "peak": PEAK_SLOTS / 1e12, "unit": "Tlane-slot/s",
                     "frac": ALG_SLOTS_STRAT * value / PEAK_SLOTS, "traffic": None,
                     "kernel": f"strat_kernel_guide<2, 4> ({ALG_SLOTS_STRAT} lane-slots per pair)"},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
