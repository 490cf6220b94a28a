#!/usr/bin/env python3
"""Exact-betweenness throughput on one MI355X: compressed (shattered +
compressed, batched) vs plain, as GTEPS = sources x edges / second.

One step = one full exact-BC computation of the workload graph with every
input resident in HBM: zero the accumulators, drain every (piece, sources)
work item of every traversal kernel class (forward sweep, backward sweep,
accumulation), and gather the per-piece scores back to the original vertices.
The host preprocessing (degree-1 stripping, biconnected shattering, identical
vertices) runs once before the timed region and is reported separately.

Prints one JSON line (see the fields below).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402

METRIC = "exact-BC GTEPS (sources×edges/s) + HBM roofline %, compressed-batched vs plain"
PEAK_HBM_GBS = 8000.0
CLASS_NAMES = ["wave_lds", "wg_lds", "batch64", "wg_global", "team64"]
KERNEL_SYMBOLS = {0: "wg_kernel<64,*,*,LDS>", 1: "wg_kernel<256,*,*,LDS>", 2: "ms_kernel<WAVES,EU,*,*>",
                  3: "wg_kernel<256,*,*,global>", 4: "ms_team_kernel<WAVES,EU,*,*>"}

WORKLOADS = {
    "rmat17": ("R-MAT scale 17 (131,072 labels), edge factor 8, (a,b,c,d)=(.57,.19,.19,.05), symmetrised, "
               "loops/duplicates removed, + 5% twins (copied neighbour lists) + 25% pendants",
               lambda: gg.rmat_decorated()),
    "ba1500": ("Barabasi-Albert core n=1,500 (2 edges per new vertex) + 400 pendants + 100 hung triangles",
               lambda: gg.ba_pendant_triangles()),
    "grid512": ("512x512 grid, 12% of edges deleted, largest component", lambda: gg.grid_deleted()),
    "blocktree20000": ("block tree of 20,000 2-connected ER blocks (8..4,096 vertices, avg degree 6)",
                       lambda: gg.block_tree()),
}


def load_traffic(workload: str, kclass: int):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        e = d.get(workload, {}).get(CLASS_NAMES[kclass])
        from paper_1209_6007_amd import kernel_source_hash

        if not e or e.get("kernel_sha") != kernel_source_hash():
            return None
        return float(e["bytes_per_launch"])
    except Exception:
        return None


def timed_run(sbc, ctx, G, mode, steps, warmup, use_graph=False):
    plan = sbc.sbc_plan_create(ctx.h, G.h, mode)
    try:
        if use_graph:
            sbc.sbc_plan_use_graph(plan, True)
        for _ in range(warmup):
            sbc.sbc_plan_execute(plan)
            sbc.sbc_plan_sync(plan)
        stats = []
        t0 = time.perf_counter()
        for _ in range(steps):
            sbc.sbc_plan_execute(plan)
            stats.append(sbc.sbc_plan_sync(plan))
        t1 = time.perf_counter()
        n, _ = sbc.sbc_graph_info(G.h)
        result = sbc.sbc_plan_result(plan, n)
    finally:
        sbc.sbc_plan_destroy(plan)
    return (t1 - t0) / steps, stats, result


def cpu_baseline(g, seconds_target: float, threads: int):
    """Oracle (Algorithm 1, FP64) on a bounded random sample of sources."""
    import oracle

    oracle.build(force=False)
    r = gg.rng(99)
    probe = r.choice(g.n, size=min(g.n, 32), replace=False).astype(np.int32)
    t0 = time.perf_counter()
    oracle.bc_plain(g.n, g.row_ptr, g.col, sources=probe, threads=threads)
    dt = max(time.perf_counter() - t0, 1e-6)
    k = int(min(g.n, max(64, len(probe) * seconds_target / dt)))
    src = r.choice(g.n, size=k, replace=False).astype(np.int32)
    t0 = time.perf_counter()
    oracle.bc_plain(g.n, g.row_ptr, g.col, sources=src, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": k * g.m / dt / 1e9, "unit": "GTEPS", "cores": threads, "kind": "oracle",
            "sample": f"{k} uniformly sampled sources of the same graph (Algorithm 1, FP64, {threads} threads), "
                      f"{dt:.1f} s, scaled to sources x edges / s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat17", choices=sorted(WORKLOADS))
    ap.add_argument("--ops", default="odai", help="preprocessing letters (o: per-piece BFS order, Section 4.1)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--graph", action="store_true", help="replay a captured HIP graph")
    ap.add_argument("--param", action="append", default=[], help="key=value tuning knob")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--phases", action="store_true", help="one extra compressed run with in-kernel phase timers")
    ap.add_argument("--calibrate", action="store_true", help="also time a plain streaming copy (1 GiB)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU split of the work items is "
              "described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)

    import paper_1209_6007_amd as sbc  # no torch in this process: the library syncs its own streams

    desc, make = WORKLOADS[args.workload]
    g = make()
    params = {}
    for kv in args.param:
        k, v = kv.split("=")
        params[k] = int(v)
    ctx = sbc.Context(0, params)
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    t0 = time.perf_counter()
    prep = G.preprocess(args.ops)
    prep_s = time.perf_counter() - t0
    nm = float(g.n) * float(g.m)

    t_c, st_c, res_c = timed_run(sbc, ctx, G, sbc.SBC_COMPRESSED, args.steps, args.warmup, args.graph)
    out = {
        "metric": METRIC,
        "value": nm / t_c / 1e9,
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_c * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "n": g.n, "m": g.m, "ops": args.ops,
                   "parallelism": "single GPU", "hip_graph": bool(args.graph)},
    }
    last = st_c[-1]
    # dominant traversal kernel of the compressed step
    k_dom = int(np.argmax(last["ms_class"]))
    ms_dom = float(np.mean([s["ms_class"][k_dom] for s in st_c]))
    bytes_dom = last["bytes_class"][k_dom]
    achieved = bytes_dom / (ms_dom * 1e-3) / 1e9 if ms_dom > 0 else 0.0
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                       "frac": achieved / PEAK_HBM_GBS, "traffic": load_traffic(args.workload, k_dom),
                       "kernel": KERNEL_SYMBOLS[k_dom], "kernel_class": CLASS_NAMES[k_dom],
                       "launch_ms": ms_dom, "algo_bytes_per_launch": bytes_dom}
    out["compressed"] = {
        "effective_gteps": nm / t_c / 1e9,
        "raw_gteps": last["teps"] / t_c / 1e9,
        "kernel_ms": float(np.mean([s["ms_traverse"] for s in st_c])),
        "device_ms": float(np.mean([s["ms_device"] for s in st_c])),
        "preprocess_s": prep_s,
        "end_to_end_gteps_incl_preprocess": nm / (t_c + prep_s) / 1e9,
        "prep": {k: prep[k] for k in ("stripped", "blocks", "bridges", "twin_classes", "twins_merged", "pieces",
                                       "piece_vertices", "piece_arcs", "work_teps")},
        "class_ms": last["ms_class"], "class_items": last["items_class"], "class_grid": last["grid_class"],
    }
    if not args.no_plain:
        t_p, st_p, res_p = timed_run(sbc, ctx, G, sbc.SBC_PLAIN, args.steps, args.warmup, args.graph)
        nz = res_p != 0
        rel = float(np.max(np.abs(res_c[nz] - res_p[nz]) / np.abs(res_p[nz]))) if nz.any() else 0.0
        lp = st_p[-1]
        kp = int(np.argmax(lp["ms_class"]))
        out["plain"] = {"gteps": nm / t_p / 1e9, "ms_per_step": t_p * 1e3,
                        "kernel_class": CLASS_NAMES[kp],
                        "hbm_frac": lp["bytes_class"][kp] / (lp["ms_class"][kp] * 1e-3) / 1e9 / PEAK_HBM_GBS
                        if lp["ms_class"][kp] > 0 else 0.0}
        out["compressed_vs_plain"] = {"speedup": t_p / t_c, "max_rel_diff": rel,
                                      "zero_mismatch": int(np.sum((res_p == 0) != (res_c == 0)))}
    if args.calibrate:
        cb = sbc.sbc_copy_bandwidth(ctx.h, 1 << 30, 10)
        out["roofline"]["copy_kernel_gbs"] = cb
        out["roofline"]["frac_of_copy"] = out["roofline"]["achieved"] / cb if cb > 0 else None
    if args.phases:
        pctx = sbc.Context(0, dict(params, profile_phases=1))
        plan = sbc.sbc_plan_create(pctx.h, G.h, sbc.SBC_COMPRESSED)
        sbc.sbc_plan_execute(plan)
        pst = sbc.sbc_plan_sync(plan)
        out["phases"] = dict(sbc.sbc_plan_phase_profile(plan), kernel_ms=pst["ms_traverse"])
        sbc.sbc_plan_destroy(plan)
        pctx.close()
    if not args.no_cpu_baseline:
        threads = min(os.cpu_count() or 1, 16)
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_seconds, threads)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
