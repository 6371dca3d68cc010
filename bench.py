"""Benchmark: exact batched evaluation of candidate mappings on one MI355X.

Workload (default): a 3-D stencil launch domain of 512^3 points on a machine of
16 nodes x 8 GPUs; every ordered 3-factorization of the 128 processors (36, from
decompose's enumeration) under 6 transformation chains = 216 candidate mappings;
7-point-axis star stencil of halo 2 with 8-byte cells.  One step evaluates every
candidate exactly (processor of each of the 216 x 134,217,728 launch points, and
the distinct-owner ghost volume with its intra/inter-node split), selects the
cheapest by (bytes, inter-node bytes, index), and materialises the selected
candidate's int32 processor map (512 MiB).  Inputs (candidate descriptors) are
resident on the device before timing starts.

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
OPS_PER_POINT = 2                     # table read + boundary test: the least any point costs
PEAK_HBM = 8.0e12                     # bytes/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--extent", type=int, default=512, help="cube side of the launch domain")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    return ap.parse_args()


def cpu_baseline(cands, st, extent):
    """The oracle (plain C, one thread) on one full-size candidate of the workload."""
    import oracle
    from workloads import c2_candidates
    c = c2_candidates([(4, 4, 8)], extent=(extent,) * 3)[0]
    t0 = time.perf_counter()
    oracle.stencil_cost(c, st)
    dt = time.perf_counter() - t0
    pts = extent ** 3
    return {"value": pts / dt, "unit": "point-evals/s", "cores": 1, "kind": "oracle",
            "sample": f"1 of the 216 candidates (F=(4,4,8), identity chain) on the full {extent}^3 "
                      f"domain: {pts} point-evals in {dt:.2f} s, single thread"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build evaluates mappings on a single MI355X "
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
    tuned = (0, 0)
    if not args.no_autotune:
        tuned = plan.autotune(out)
    _, items, _ = plan.info()

    def step(ev=None):
        plan.run_stage(0, out, best)
        if ev:
            ev[0].record()
        plan.run_stage(1, out, best)
        if ev:
            ev[1].record()
        plan.run_stage(2, out, best)
        if ev:
            ev[2].record()
        plan.materialize(pmap, d_index=best)
        if ev:
            ev[3].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    e_start = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        e_start[k].record()
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    prep = np.mean([e_start[k].elapsed_time(evs[k][0]) for k in range(args.steps)])
    count = np.mean([evs[k][0].elapsed_time(evs[k][1]) for k in range(args.steps)])
    sel = np.mean([evs[k][1].elapsed_time(evs[k][2]) for k in range(args.steps)])
    mapk = np.mean([evs[k][2].elapsed_time(evs[k][3]) for k in range(args.steps)])

    costs = out.cpu().numpy()
    b = int(best.cpu()[0])
    value = points / (ms_step * 1e-3)
    ach = OPS_PER_POINT * points / (count * 1e-3)
    map_bw = 4.0 * L ** 3 / (mapk * 1e-3)
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
                   "cells_per_item": tuned[0], "wg_per_cu": tuned[1]},
        "roofline": {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "Tlane-op/s", "frac": ach / PEAK_LANE_OPS, "traffic": None,
                     "kernel": "k_count<3,2>", "ops_per_point": OPS_PER_POINT,
                     "kernel_ms": count},
        "roofline_map": {"bound": "hbm", "achieved": map_bw / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                         "frac": map_bw / PEAK_HBM, "traffic": None, "kernel": "k_map",
                         "bytes_per_point": 4, "kernel_ms": mapk},
        "stages_ms": {"tables": prep, "count": count, "select": sel, "map": mapk},
        "count_point_evals_per_s": points / (count * 1e-3),
        "map_points_per_s": L ** 3 / (mapk * 1e-3),
        "selected": {"index": b, "factorization": list(fs[b // 6]), "chain": b % 6,
                     "bytes": int(costs[b][2]), "inter_bytes": int(costs[b][3])},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(cands, st, L)
    plan.close()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
