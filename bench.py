"""Benchmark: exact batched evaluation of candidate mappings on one MI355X.

Workload (default): a 3-D stencil launch domain of 512^3 points on a machine of
16 nodes x 8 GPUs; every ordered 3-factorization of the 128 processors (36, from
decompose's enumeration) under 6 transformation chains = 216 candidate mappings;
7-point-axis star stencil of halo 2 with 8-byte cells.  One step evaluates every
candidate exactly (processor of each of the 216 x 134,217,728 launch points, and
the distinct-owner ghost volume with its intra/inter-node split), selects the
cheapest by (bytes, inter-node bytes, index), and materialises the selected
candidate's int32 processor map (512 MiB), all in one graph replay; consecutive steps
run round-robin on three streams (a plan and outputs each), so a step's evaluation
overlaps the previous step's map write.  Inputs (candidate descriptors) are
resident on the device before timing starts.  The ghost volume of a candidate is
counted exactly over its coordinate classes (runs of coordinates with the same
contribution and neighbour offsets along each launch dim), so the counting work is
its class tuples, not its points; the map is written point by point.

The metric's second part -- candidates ranked per second by the learned ranker vs
exhaustive exact evaluation, at the exhaustive optimum -- is the "search" object of
the same line (trained on 1M exact costs from the random-chain generator, evaluated
on ~1M candidates of 457 search instances; --no-search skips it).  Also by default:
"c3" (the 4,096-candidate random batch, one plan) and "c4" (the matmul batch).
Optional legs: --study (decompose vs Alg. A1 volumes), --two-level (hierarchical
decompositions), --transpose (all-to-all transposes), --c3-cyclic.

Prints one JSON line (see the keys below).  Only one GPU is supported.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "mapping point-evals/sec; candidates ranked/sec surrogate vs exhaustive at =opt"
PEAK_LANE_OPS = 256 * 64 * 2.4e9      # 32-bit VALU lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz
# Integer operations of one exact cell evaluation for a 3-D halo-2 star: one owner
# lookup, up to 2 * sum(h) = 12 neighbour lookups, compares and the de-duplication of
# a small set -- about 50 to 70; the midpoint prices one class-tuple evaluation (a
# class tuple is evaluated exactly like one of its cells).
OPS_PER_TUPLE = 60
PEAK_HBM = 8.0e12                     # bytes/s

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes (scaled by
# reference kernels' readings: reads x2.000 as a copy, writes x1.000 as a fill), valid only for the kernel
# sources they were taken on (hash of the files below); see
# profiles/c2_512cube_hbm_traffic.txt.
KERNEL_SOURCES = ["paper_2507_17087_amd/csrc/tm_kernels.hip", "paper_2507_17087_amd/csrc/tm_chain.h",
                  "paper_2507_17087_amd/csrc/tm_internal.h"]
TRAFFIC_SOURCE_HASH = "8f383901c5ebc06f"
TRAFFIC_BYTES = {"k_map": 537.05e6}


def measured_traffic(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return TRAFFIC_BYTES.get(kernel) if h.hexdigest()[:16] == TRAFFIC_SOURCE_HASH else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--streams", type=int, default=3,
                    help="streams the timed steps are issued on, round-robin (one plan and output set each)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--extent", type=int, default=512, help="cube side of the launch domain")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=min(16, os.cpu_count() or 1),
                    help="host threads for the oracle baseline (one candidate each)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--launch", type=int, nargs=2, metavar=("CELLS_PER_ITEM", "WG_PER_CU"),
                    help="fixed counting launch configuration instead of autotuning (e.g. for profiling)")
    ap.add_argument("--search", dest="search", action="store_true", default=True,
                    help="run the learned-ranker search leg (the default: the metric's second part)")
    ap.add_argument("--no-search", dest="search", action="store_false", help="skip the search leg")
    ap.add_argument("--study", action="store_true", help="also run the decompose-vs-Alg.-A1 volume study")
    ap.add_argument("--two-level", action="store_true", help="also run the two-level decomposition leg")
    ap.add_argument("--transpose", action="store_true", help="also run the all-to-all transpose leg")
    ap.add_argument("--c3", dest="c3", action="store_true", default=True,
                    help="run the 4,096-candidate random batch (the default)")
    ap.add_argument("--no-c3", dest="c3", action="store_false", help="skip the random batch")
    ap.add_argument("--c4", dest="c4", action="store_true", default=True, help="run the matmul batch (the default)")
    ap.add_argument("--no-c4", dest="c4", action="store_false", help="skip the matmul batch")
    ap.add_argument("--c3-cyclic", action="store_true",
                    help="also run the random batch with 25%% of projections cyclic")
    ap.add_argument("--search-train", type=int, default=1_000_000, help="training candidates (exact costs)")
    ap.add_argument("--search-eval", type=int, default=1_000_000, help="evaluation candidates")
    ap.add_argument("--search-epochs", type=int, default=8)
    ap.add_argument("--search-eval-seed", type=int, default=2, help="seed of the evaluation instances")
    ap.add_argument("--search-prefilter", type=int, default=256,
                    help="candidates per instance the network keeps (first stage)")
    ap.add_argument("--search-topk", type=int, default=32,
                    help="of those, candidates per instance the block-model estimates send to exact evaluation")
    ap.add_argument("--search-train-source", choices=("c3", "menu"), default="c3",
                    help="training candidates: the random-chain generator (c3 recipe, rank 3, seed 1) or "
                         "chain-menu instances (seed 1)")
    ap.add_argument("--search-octaves", type=int, nargs=2, default=[5, 9])
    ap.add_argument("--copy-probe", action="store_true",
                    help="a 256 MiB fill, copy and reduction before timing (references for the HBM counters)")
    return ap.parse_args()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cands, st, extent, threads, gpu_costs):
    """The oracle (plain C, single-threaded per call) on `threads` full-size candidates
    of the workload, one per host thread (ctypes releases the GIL during each call),
    then one of them alone on one thread; the oracle's results are compared with the
    GPU's cost rows of the same candidates."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    picks = [(i * 37) % len(cands) for i in range(threads)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(lambda i: oracle.stencil_cost(cands[i], st), picks))
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    one = oracle.stencil_cost(cands[picks[0]], st)
    dt1 = time.perf_counter() - t1
    pts = threads * extent ** 3
    equal = sum(1 for i, r in zip(picks, res) if tuple(int(x) for x in gpu_costs[i]) == r)
    return {"value": pts / dt, "unit": "point-evals/s", "cores": threads, "kind": "oracle",
            "single_thread_value": extent ** 3 / dt1, "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(),
            "sample": f"{threads} of the {len(cands)} candidates (indices {picks[0]}, {picks[1] if threads > 1 else ''}"
                      f"... step 37 mod {len(cands)}) on the full {extent}^3 domain, one oracle call per "
                      f"host thread: {pts} point-evals in {dt:.2f} s; then candidate {picks[0]} alone on one "
                      f"thread in {dt1:.2f} s",
            "parity": {"checked": len(picks), "equal": equal, "single_thread_equal": one == res[0]}}


def instances_with(tm, W, seed, target, octaves, min_cands=1024):
    """Search instances (c3's domain and machine distribution, launch rank 3) whose
    candidate lists (factorizations x 32 chains) have at least min_cands entries,
    until `target` candidates are reached."""
    inst, fls, total, first = [], [], 0, 0
    while total < target:
        for ext, n, g in W.random_instances(256, seed=seed, first=first, octaves=tuple(octaves)):
            fs = tm.tm_enumerate_factorizations(n * g, 3)
            if len(fs) * 32 >= min_cands:
                inst.append((ext, n, g))
                fls.append(fs)
                total += len(fs) * 32
                if total >= target:
                    break
        first += 256
    cands, seg = W.instance_batch(inst, fls)
    return cands, seg, inst


def search_leg(args, tm, W):
    """Learned ranker: train on exact costs of 1M candidates (by default from the
    random-chain generator, seed 1), then search the candidates of seed-2 chain-menu
    instances in two stages (the network keeps --search-prefilter per instance, their
    block-model estimates send --search-topk to exact evaluation) and compare with
    exhaustive exact evaluation of every candidate (both timed after a warm-up call)."""
    import torch
    st = W.c3_stencil(3)
    t0 = time.perf_counter()
    if args.search_train_source == "c3":
        tc = W.random_candidates(args.search_train, seed=1, ranks=(3,), octaves=tuple(args.search_octaves))
    else:
        tc, _, _ = instances_with(tm, W, 1, args.search_train, args.search_octaves)
    plan = tm.Plan(len(tc), 1)
    plan.load(tc, st)
    costs = torch.empty((len(tc), 4), dtype=torch.int64, device="cuda")
    plan.run(costs)
    feat = tm.tm_ranker_features(plan)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r = tm.Ranker(seed=1)
    losses = r.train(feat, costs, epochs=args.search_epochs, batch=4096, lr=2e-3, seed=1)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    del feat, costs
    plan.close()
    ec, seg, einst = instances_with(tm, W, args.search_eval_seed, args.search_eval, args.search_octaves)
    plan = tm.Plan(len(ec), 1)
    plan.load(ec, st)
    tm.tm_search(plan, None, seg)  # warm-up
    torch.cuda.synchronize()
    reps = 3
    e0 = time.perf_counter()
    for _ in range(reps):
        b_ex, c_ex = tm.tm_search(plan, None, seg)
    torch.cuda.synchronize()
    e1 = time.perf_counter()
    K1, K = args.search_prefilter, args.search_topk
    tm.tm_search(plan, r, seg, topk=K, prefilter=K1)  # warm-up
    torch.cuda.synchronize()
    e2 = time.perf_counter()
    for _ in range(reps):
        b_rk, c_rk = tm.tm_search(plan, r, seg, topk=K, prefilter=K1)
    torch.cuda.synchronize()
    e3 = time.perf_counter()
    ce, cr = c_ex.cpu().numpy(), c_rk.cpu().numpy()
    ok = (ce[:, 2] == cr[:, 2]) & (ce[:, 3] == cr[:, 3])
    # a score margin: of the second stage's top-K, only candidates estimated within
    # 0.05 (log2 units, ~3.5 %) of the instance's best are evaluated exactly
    tm.tm_search(plan, r, seg, topk=K, prefilter=K1, margin=0.05)
    torch.cuda.synchronize()
    m0 = time.perf_counter()
    for _ in range(reps):
        _, c_mg = tm.tm_search(plan, r, seg, topk=K, prefilter=K1, margin=0.05)
    torch.cuda.synchronize()
    m1 = time.perf_counter()
    cm = c_mg.cpu().numpy()
    okm = (ce[:, 2] == cm[:, 2]) & (ce[:, 3] == cm[:, 3])
    # ablation: the same search with an all-zero network, whose first stage ranks by
    # the descriptor estimate alone (the method without the network); and the share
    # of instances whose optimum the first stage's cut keeps (single-stage top-k, k up
    # to the prefilter), trained vs all-zero, with that search's throughput
    r0 = tm.Ranker(seed=1)
    r0.set_params(torch.zeros(tm.tm_ranker_param_count(), dtype=torch.float32, device="cuda"))
    _, c_0 = tm.tm_search(plan, r0, seg, topk=K, prefilter=K1)
    c0 = c_0.cpu().numpy()
    ok0 = (ce[:, 2] == c0[:, 2]) & (ce[:, 3] == c0[:, 3])
    curve = {}
    k99 = None
    for k in (1, 4, 16, 64, 256):
        row = {}
        for name, rr in (("trained", r), ("estimate_only", r0)):
            tm.tm_search(plan, rr, seg, topk=k)
            torch.cuda.synchronize()
            k0 = time.perf_counter()
            _, ck = tm.tm_search(plan, rr, seg, topk=k)
            torch.cuda.synchronize()
            k1 = time.perf_counter()
            ck = ck.cpu().numpy()
            row[name] = {"opt_rate": float(((ce[:, 2] == ck[:, 2]) & (ce[:, 3] == ck[:, 3])).mean()),
                         "ranked_candidates_per_s": len(ec) / (k1 - k0)}
        curve[str(k)] = row
        if k99 is None and row["trained"]["opt_rate"] >= 0.99:
            k99 = k
    r0.close()
    # the paper's choice without search: decompose's argmin factorization (Sec. 4.3)
    # under the better of the two machine orders, evaluated exactly
    base = []
    for ext, nn, g in einst:
        f = tm.tm_decompose_argmin(nn * g, ext, (1, 1, 1))
        base.append(W.candidate(ext, nn, g, [W.merge(0, 1), W.decompose(0, f)]))
        base.append(W.candidate(ext, nn, g, [W.swap(0, 1), W.merge(0, 1), W.decompose(0, f)]))
    cb = tm.tm_eval_stencil_batch(W.batch(base), st).cpu().numpy()
    ev, od = cb[0::2], cb[1::2]
    first_le = (ev[:, 2] < od[:, 2]) | ((ev[:, 2] == od[:, 2]) & (ev[:, 3] <= od[:, 3]))
    cd = np.where(first_le[:, None], ev, od)
    better = (cr[:, 2] < cd[:, 2]) | ((cr[:, 2] == cd[:, 2]) & (cr[:, 3] < cd[:, 3]))
    n = len(ec)
    ex_rate = n / ((e1 - e0) / reps)
    rk_rate = n / ((e3 - e2) / reps)
    plan.close()
    r.close()
    return {"instances": int(len(seg) - 1), "candidates": int(n), "prefilter": K1, "topk": K,
            "exact_evaluations": int((len(seg) - 1) * K),
            "opt_rate": float(ok.mean()), "estimate_only_opt_rate": float(ok0.mean()),
            "single_stage_curve": curve, "smallest_single_stage_topk_at_99": k99,
            "with_margin_0.05": {"opt_rate": float(okm.mean()),
                                 "ranked_candidates_per_s": len(ec) / ((m1 - m0) / reps),
                                 "speedup": (len(ec) / ((m1 - m0) / reps)) / ex_rate},
            "vs_decompose": {"better_instances": float(better.mean()),
                             "bytes_reduction": float(1 - cr[:, 2].sum() / cd[:, 2].sum()),
                             "inter_bytes_reduction": float(1 - cr[:, 3].sum() / max(1, cd[:, 3].sum()))},
            "ranked_candidates_per_s": rk_rate,
            "exhaustive_candidates_per_s": ex_rate, "speedup": rk_rate / ex_rate,
            "train_candidates": int(len(tc)), "train_source": args.search_train_source,
            "train_epochs": args.search_epochs,
            "train_loss_first_last": [losses[0], losses[-1]] if losses else None,
            "exact_costs_s": t1 - t0, "train_s": t2 - t1,
            "extents": f"octaves {args.search_octaves[0]}..{args.search_octaves[1]} per dim (log-uniform)"}


def study_leg(tm, W):
    """Sec. 6.3's decompose-vs-Alg.-A1 comparison as exact communication volumes:
    180 2-D stencil configurations x {decompose's F, Alg. A1's F} x {node-major,
    GPU-major machine order}, halo 1, 8-B cells, all evaluated in one plan."""
    import torch
    cf = W.study_configs(long_last=True) + W.study_configs(long_last=False)
    fd = [tm.tm_decompose_argmin(g, ext, (1, 1)) for a, s, g, ext, n, gp in cf]
    fg = [tm.tm_greedy_grid(g, 2) for a, s, g, ext, n, gp in cf]
    cands = W.study_candidates(cf, fd, fg)
    st = W.stencil((1, 1), 8)
    plan = tm.Plan(len(cands), 1)
    plan.load(cands, st)
    out = torch.empty((len(cands), 4), dtype=torch.int64, device="cuda")
    plan.run(out)
    torch.cuda.synchronize()
    ts = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.run(out)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    _, _, pts = plan.info()
    plan.close()
    c = out.cpu().numpy().reshape(len(cf), 2, 2, 4)  # config, (decompose, A1), (node-major, GPU-major)

    def gm(x):
        return float(np.exp(np.mean(np.log(x))))

    def ratios(col, order):
        g, d = c[:, 1, order, col].astype(np.float64), c[:, 0, order, col].astype(np.float64)
        ok = d > 0
        return np.where(ok, g / np.where(ok, d, 1), 1.0)

    res = {"configs": len(cf), "candidates": int(len(cands)), "point_evals": int(pts),
           "gpu_ms": min(ts), "point_evals_per_s": pts / (min(ts) * 1e-3),
           "differs": int(sum(1 for a, b in zip(fd, fg) if tuple(a) != tuple(b)))}
    half = len(cf) // 2
    for orient, rows in (("long_dim_last", slice(0, half)), ("long_dim_first", slice(half, len(cf)))):
        sub_cf = cf[rows]
        res[orient] = {}
        for name, col, order in (("bytes", 2, 0), ("inter_bytes_node_major", 3, 0),
                                 ("inter_bytes_gpu_major", 3, 1)):
            r = ratios(col, order)[rows]
            by = {}
            for key, idx in (("aspect", 0), ("size_per_node", 1), ("gpus", 2)):
                vals = sorted(set(x[idx] for x in sub_cf))
                by[key] = {str(v): gm(r[[i for i, x in enumerate(sub_cf) if x[idx] == v]]) - 1 for v in vals}
            res[orient][name] = {"A1_over_decompose_geomean_minus_1": gm(r) - 1, "max": float(r.max() - 1),
                                 "min": float(r.min() - 1), **by}
    return res


def two_level_leg(tm, W):
    """Two-level decompositions (App. A.1's hierarchical mappers) of the benchmark
    domain: every node grid of the 16 nodes x every GPU grid of the 8 GPUs per node,
    hierarchical block and node-block / GPU-cyclic (300 candidates), against the
    benchmark's flat candidates; per-processor costs and the node-level exchange
    volume (a node receives each remote cell once)."""
    import torch
    L = 512
    fam = W.two_level_candidates((L, L, L), 16, 8, tm.tm_enumerate_factorizations(16, 3),
                                 tm.tm_enumerate_factorizations(8, 3))
    flat = W.c2_candidates(tm.tm_enumerate_factorizations(128, 3), extent=(L, L, L))
    st = W.c2_stencil()
    res = {"candidates": int(len(fam)), "flat_candidates": int(len(flat))}
    for name, cands in (("two_level", fam), ("flat", flat)):
        tm.tm_eval_stencil_batch(cands, st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        proc = tm.tm_eval_stencil_batch(cands, st).cpu().numpy()
        t1 = time.perf_counter()
        node = tm.tm_eval_stencil_node_batch(cands, st).cpu().numpy()
        t2 = time.perf_counter()
        pts = len(cands) * L ** 3
        bi = int(np.lexsort((np.arange(len(cands)), proc[:, 3], proc[:, 2]))[0])
        res[name] = {"best_bytes": int(proc[bi, 2]), "best_inter_bytes": int(proc[bi, 3]),
                     "min_inter_bytes": int(proc[:, 3].min()), "min_node_level_bytes": int(node[:, 2].min()),
                     "node_level_bytes_of_best": int(node[bi, 2]),
                     "point_evals_per_s_host_inclusive": [pts / (t1 - t0), pts / (t2 - t1)]}
    return res


def transpose_leg(tm, W, reps=3):
    """Transposes by all-to-all exchanges (App. A.3) on the benchmark domain: for
    every decompose candidate of 128 processors, the exact halo-2 ghost transfers and
    the exact cells moved by a transpose along each dim in T (to the pencil-transposed
    image split along the next dim), for T = {0} and T = {0, 1}.  Reports decompose's
    plain pick, the transpose-aware objective's pick and the exact optimum of
    ghost + moved transfers, and the redistribution kernel's throughput."""
    import torch
    L = 512
    ext = (L, L, L)
    facs = tm.tm_enumerate_factorizations(128, 3)
    cands = W.batch([W.candidate(ext, 16, 8, [W.merge(0, 1), W.decompose(0, f)]) for f in facs])
    st = W.c2_stencil()
    ghost = tm.tm_eval_stencil_batch(cands, st).cpu().numpy()
    src, dst = [], []
    for c in cands:
        for n in range(3):
            src.append(c)
            dst.append(tm.tm_transpose_target(c, n, (n + 1) % 3))
    src, dst = W.batch(src), W.batch(dst)
    tm.tm_eval_redistribution_batch(src, dst, 8)
    torch.cuda.synchronize()
    ts, tg = [], []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        moved = tm.tm_eval_redistribution_batch(src, dst, 8)
        e1.record()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        tg.append(e0.elapsed_time(e1))
    moved = moved.cpu().numpy().reshape(len(facs), 3, 4)
    pts = len(src) * L ** 3
    res = {"pairs": int(len(src)), "points": int(pts), "ms_host_inclusive": 1e3 * float(np.median(ts)),
           "gpu_ms": float(np.median(tg)), "point_evals_per_s_host_inclusive": pts / float(np.median(ts)),
           "point_evals_per_s_gpu": pts / (float(np.median(tg)) * 1e-3)}
    plain = facs.index(tm.tm_decompose_argmin(128, ext, (2, 2, 2)))
    for T in ((0,), (0, 1)):
        tot = ghost[:, 2] + sum(moved[:, n, 2] for n in T)
        inter = ghost[:, 3] + sum(moved[:, n, 3] for n in T)
        aware = facs.index(tm.tm_decompose_argmin_transpose(128, ext, (2, 2, 2), T))
        best = int(np.lexsort((np.arange(len(facs)), inter, tot))[0])
        res["T=" + "".join(str(n) for n in T)] = {
            "decompose": {"F": list(facs[plain]), "bytes": int(tot[plain]), "inter_bytes": int(inter[plain])},
            "transpose_aware": {"F": list(facs[aware]), "bytes": int(tot[aware]), "inter_bytes": int(inter[aware])},
            "exact_best": {"F": list(facs[best]), "bytes": int(tot[best]), "inter_bytes": int(inter[best])}}
    return res


def c3_leg(tm, W, reps=20, cyclic_pct=0):
    """The batched workload: 4,096 random candidates (seed 17087; launch ranks 2 and 3
    mixed, extents log-uniform 32..1023, 1..64 nodes x {1,2,4,8} GPUs, 0-4 random
    transformations), halo 1, in one plan (one counting launch), autotuned, timed as
    graph replays of the whole evaluation (reset, tables, counting, selection) with
    HIP events on the plan's stream.  cyclic_pct: the share of projections drawn
    cyclic (the coverage variant)."""
    import torch
    cs = W.c3_candidates(4096, cyclic_pct=cyclic_pct)
    plan = tm.Plan(len(cs), 1)
    plan.load(cs, W.c3_stencil(3))  # a rank-2 candidate takes the first two halo widths
    out = torch.empty((len(cs), 4), dtype=torch.int64, device="cuda")
    best = torch.empty(1, dtype=torch.int64, device="cuda")
    plan.run(out, best)
    cpi, wg = plan.autotune(out)
    plan.run(out, best)
    torch.cuda.synchronize()
    ts, tc = [], []
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record()
        plan.run_stage(0, out, best)
        e[1].record()
        plan.run_stage(1, out, best)
        e[2].record()
        plan.run_stage(2, out, best)
        e[3].record()
        torch.cuda.synchronize()
        ts.append(e[0].elapsed_time(e[3]))
        tc.append(e[1].elapsed_time(e[2]))
    _, items, pts = plan.info()
    tuples = plan.class_tuples()
    plan.close()
    ms, cms = float(np.median(ts)), float(np.median(tc))
    ach = OPS_PER_TUPLE * tuples / (cms * 1e-3)
    return {"candidates": int(len(cs)), "ranks": sorted(int(k) for k in set(cs["lrank"])), "points": int(pts),
            "ms": ms, "ms_spread": [float(min(ts)), float(max(ts))], "point_evals_per_s": pts / (ms * 1e-3),
            "count_ms": cms, "class_tuples": int(tuples), "work_items": int(items),
            "tuples_per_item": cpi, "wg_per_cu": wg,
            "roofline_count": {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                               "unit": "Tlane-op/s", "frac": ach / PEAK_LANE_OPS, "kernel": "k_count",
                               "ops_per_tuple": OPS_PER_TUPLE}}


def c4_leg(tm, W, reps=10):
    """The matmul workload: 256^3 task points on 16 nodes x 4 GPUs, every
    3-factorization of 64 (with and without swap(0,1)) plus the hierarchical Cannon
    mapper: 57 candidates, 8 MiB tiles; one call per evaluation, timed on the host
    (validation, upload, tables, counting) and with HIP events on the call's stream.
    The counting runs over pairs of coordinate classes (a few to a few thousand per
    matrix here, not 65,536 tiles), so the call is bound by its launches and copies,
    not by arithmetic: no roofline is claimed for it."""
    import torch
    fs = tm.tm_enumerate_factorizations(64, 3)
    mc = W.c4_candidates(fs)
    tm.tm_eval_matmul_batch(mc, W.C4_TILE_BYTES)
    torch.cuda.synchronize()
    ts, tg = [], []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        tm.tm_eval_matmul_batch(mc, W.C4_TILE_BYTES)
        e1.record()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        tg.append(e0.elapsed_time(e1))
    dt, gms = float(np.median(ts)), float(np.median(tg))
    pts = len(mc) * 256 ** 3
    return {"candidates": int(len(mc)), "task_points": int(pts), "ms_host_inclusive": dt * 1e3,
            "gpu_ms": gms, "point_evals_per_s": pts / dt, "point_evals_per_s_gpu": pts / (gms * 1e-3)}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library evaluates mappings on a single MI355X "
              "(multi-GPU sharding is described in the design notes, not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2507_17087_amd as tm
    import workloads as W

    torch.cuda.set_device(0)
    L = args.extent
    # decompose's search space, from the library
    fs = tm.tm_enumerate_factorizations(128, 3)
    cands = W.c2_candidates(fs, extent=(L, L, L))
    st = W.c2_stencil()
    n = len(cands)
    points = n * L ** 3

    plan = tm.Plan(n, 1)
    plan.load(cands, st)
    out = torch.empty((n, 4), dtype=torch.int64, device="cuda")
    best = torch.empty(1, dtype=torch.int64, device="cuda")
    pmap = torch.empty(L ** 3, dtype=torch.int32, device="cuda")
    if args.copy_probe:
        a = torch.ones(64 << 20, dtype=torch.int32, device="cuda")  # a fill: writes 256 MiB
        b = torch.empty_like(a)
        b.copy_(a)
        s_ = a.sum()  # a reduction: reads 256 MiB
        torch.cuda.synchronize()
        del a, b, s_
    tuned = (0, 0)
    if args.launch:
        tuned = tuple(args.launch)
        plan.set_launch(*tuned)
    elif not args.no_autotune:
        tuned = plan.autotune(out)
    _, items, _ = plan.info()

    # A step: one graph replay -- the evaluation (tables and classes, counting, bytes
    # + selection) and then the map of the selected candidate, with no host step in
    # between.  The timed steps are issued round-robin on `--streams` streams, each
    # with its own plan (the same batch) and its own outputs, so that one step's
    # evaluation (latency-bound) overlaps the previous step's map write (HBM-bound);
    # every step is a whole pass.  Events around each replay on its stream.
    ns = max(1, args.streams)
    lanes = [(plan, out, best, pmap, torch.cuda.current_stream())]
    for _ in range(ns - 1):
        p2 = tm.Plan(n, 1)
        p2.load(cands, st)
        p2.set_launch(*tuned)
        lanes.append((p2, torch.empty_like(out), torch.empty_like(best), torch.empty_like(pmap),
                      torch.cuda.Stream()))

    def step(k):
        p_, o_, b_, m_, s_ = lanes[k % ns]
        with torch.cuda.stream(s_):
            p_.run_map(o_, b_, m_)

    for k in range(args.warmup * ns):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    lanes_agree = all(bool(torch.equal(lanes[i][1], out)) and bool(torch.equal(lanes[i][2], best)) and
                      bool(torch.equal(lanes[i][3], pmap)) for i in range(ns))
    # the same steps on one stream (one step at a time), for comparison; then once more
    # with events around each replay for the per-step GPU time
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for k in range(args.steps):
        plan.run_map(out, best, pmap)
    torch.cuda.synchronize()
    ms_step_one = (time.perf_counter() - t2) * 1e3 / args.steps
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    for k in range(args.steps):
        evs[k][0].record()
        plan.run_map(out, best, pmap)
        evs[k][1].record()
    torch.cuda.synchronize()
    step_gpu = np.array([evs[k][0].elapsed_time(evs[k][1]) for k in range(args.steps)])
    # breakdown (second and third passes over the same steps; not part of `value`):
    # the evaluation graph and the map launch with events between them, then the
    # evaluation one stage graph at a time
    mev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    for k in range(args.steps):
        mev[k][0].record()
        plan.run(out, best)
        mev[k][1].record()
        plan.materialize(pmap, d_index=best)
        mev[k][2].record()
    sev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    for k in range(args.steps):
        sev[k][0].record()
        for stage in range(3):
            plan.run_stage(stage, out, best)
            sev[k][stage + 1].record()
    torch.cuda.synchronize()
    evalk = np.mean([mev[k][0].elapsed_time(mev[k][1]) for k in range(args.steps)])
    mapk = np.mean([mev[k][1].elapsed_time(mev[k][2]) for k in range(args.steps)])
    prep = np.mean([sev[k][0].elapsed_time(sev[k][1]) for k in range(args.steps)])
    count = np.mean([sev[k][1].elapsed_time(sev[k][2]) for k in range(args.steps)])
    sel = np.mean([sev[k][2].elapsed_time(sev[k][3]) for k in range(args.steps)])

    costs = out.cpu().numpy()
    b = int(best.cpu()[0])
    tuples = plan.class_tuples()
    value = points / (ms_step * 1e-3)
    cnt_ach = OPS_PER_TUPLE * tuples / (count * 1e-3)
    map_bw = 4.0 * L ** 3 / (mapk * 1e-3)
    roof_map = {"bound": "hbm", "achieved": map_bw / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": map_bw / PEAK_HBM, "traffic": measured_traffic("k_map"), "kernel": "k_map",
                "bytes_per_point": 4, "kernel_ms": mapk}
    roof_count = {"bound": "alu", "achieved": cnt_ach / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                  "unit": "Tlane-op/s", "frac": cnt_ach / PEAK_LANE_OPS, "traffic": measured_traffic("k_count"),
                  "kernel": "k_count", "class_tuples": tuples, "ops_per_tuple": OPS_PER_TUPLE, "kernel_ms": count}
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "point-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"3-D stencil {L}^3 on 16 nodes x 8 GPUs: 36 factorizations x 6 chains "
                               f"= {n} candidates, star halo 2, 8-B cells; exact ghost volume of every "
                               f"candidate + selection + int32 map of the winner",
                   "candidates": n, "points_per_candidate": L ** 3, "halo": 2,
                   "machine": [16, 8], "work_items": items,
                   "tuples_per_item": tuned[0], "wg_per_cu": tuned[1]},
        # the step's dominant kernel (largest mean time of the stages)
        "roofline": roof_map if mapk >= max(count, prep) else roof_count,
        "roofline_map": roof_map,
        "roofline_count": roof_count,
        "stages_ms": {"evaluate": evalk, "map": mapk, "tables": prep, "count": count, "select": sel},
        "step_gpu_ms": {"median": float(np.median(step_gpu)), "min": float(step_gpu.min()),
                        "max": float(step_gpu.max())},
        "streams": ns,
        "streams_agree": lanes_agree,
        "ms_per_step_one_stream": ms_step_one,
        "value_one_stream": points / (ms_step_one * 1e-3),
        "count_point_evals_per_s": points / (count * 1e-3),
        "count_class_tuples_per_s": tuples / (count * 1e-3),
        "map_points_per_s": L ** 3 / (mapk * 1e-3),
        "selected": {"index": b, "factorization": list(fs[b // 6]), "chain": b % 6,
                     "bytes": int(costs[b][2]), "inter_bytes": int(costs[b][3])},
    }
    for ln in lanes:
        ln[0].close()
    del pmap, lanes
    if args.search:
        res["search"] = search_leg(args, tm, W)
    if args.study:
        res["study"] = study_leg(tm, W)
    if args.two_level:
        res["two_level"] = two_level_leg(tm, W)
    if args.transpose:
        res["transpose"] = transpose_leg(tm, W)
    if args.c3:
        res["c3"] = c3_leg(tm, W)
    if args.c3_cyclic:
        res["c3_cyclic"] = c3_leg(tm, W, cyclic_pct=25)
    if args.c4:
        res["c4"] = c4_leg(tm, W)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(cands, st, L, args.cpu_threads, costs)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
