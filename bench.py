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
CLASS_NAMES = ["small_lds", "unused1", "batch64", "deep64", "team64"]
KERNEL_SYMBOLS = {0: "wave_kernel<WAVES,*,*>", 1: "", 2: "ms_kernel<WAVES,EU,*,*>",
                  3: "ms_kernel<WAVES,EU,*,*> (deep pieces)", 4: "ms_team_kernel<WAVES,EU,*,*>"}

WORKLOADS = {
    "rmat17": ("R-MAT scale 17 (131,072 labels), edge factor 8, (a,b,c,d)=(.57,.19,.19,.05), symmetrised, "
               "loops/duplicates removed, + 5% twins (copied neighbour lists) + 25% pendants",
               lambda: gg.rmat_decorated()),
    "ba1500": ("Barabasi-Albert core n=1,500 (2 edges per new vertex) + 400 pendants + 100 hung triangles",
               lambda: gg.ba_pendant_triangles()),
    "grid512": ("512x512 grid, 12% of edges deleted, largest component", lambda: gg.grid_deleted()),
    "blocktree20000": ("block tree of 20,000 2-connected ER blocks (8..4,096 vertices, avg degree 6)",
                       lambda: gg.block_tree()),
    "blocktree20000s": ("block tree of 20,000 2-connected ER blocks (8..256 vertices, avg degree 6): "
                        "small pieces only", lambda: gg.block_tree(max_size=256)),
}


def load_traffic(workload: str, kclass):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source (kclass: a traversal class index, or a
    name such as "far64" for the farness kernel)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        e = d.get(workload, {}).get(kclass if isinstance(kclass, str) else CLASS_NAMES[kclass])
        from paper_1209_6007_amd import kernel_source_hash

        if not e or e.get("kernel_sha") != kernel_source_hash():
            return None
        return float(e["bytes_per_launch"])
    except Exception:
        return None


def progress(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def timed_run(sbc, ctx, G, mode, steps, warmup, use_graph=False):
    name = "plain" if mode == sbc.SBC_PLAIN else "compressed"
    plan = sbc.sbc_plan_create(ctx.h, G.h, mode)
    try:
        if use_graph:
            sbc.sbc_plan_use_graph(plan, True)
        for i in range(warmup):
            sbc.sbc_plan_execute(plan)
            st = sbc.sbc_plan_sync(plan)
            progress(f"{name} warm-up {i}: {st['ms_device']:.1f} ms")
        stats = []
        t0 = time.perf_counter()
        for i in range(steps):
            sbc.sbc_plan_execute(plan)
            stats.append(sbc.sbc_plan_sync(plan))
            progress(f"{name} step {i}: {stats[-1]['ms_device']:.1f} ms")
        t1 = time.perf_counter()
        n, _ = sbc.sbc_graph_info(G.h)
        result = sbc.sbc_plan_result(plan, n)
    finally:
        sbc.sbc_plan_destroy(plan)
    return (t1 - t0) / steps, stats, result


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(g, sources_pool, seconds_target: float, threads: int, r):
    """Sources x edges per second of the oracle on about seconds_target of work."""
    import oracle

    probe = r.choice(sources_pool, size=min(len(sources_pool), 8 * threads), replace=False).astype(np.int32)
    t0 = time.perf_counter()
    oracle.bc_plain(g.n, g.row_ptr, g.col, sources=probe, threads=threads)
    dt = max(time.perf_counter() - t0, 1e-6)
    k = int(min(len(sources_pool), max(4 * threads, len(probe) * seconds_target / dt)))
    src = r.choice(sources_pool, size=k, replace=False).astype(np.int32)
    t0 = time.perf_counter()
    oracle.bc_plain(g.n, g.row_ptr, g.col, sources=src, threads=threads)
    dt = time.perf_counter() - t0
    return k * g.m / dt, k, dt


def cpu_baseline(g, seconds_target: float, threads: int):
    """Oracle (Algorithm 1, FP64) on bounded random samples of the graph's
    non-isolated sources: with `threads` threads, and with one thread (a
    per-core rate comparable with the paper's single-core runs)."""
    import oracle

    oracle.build(force=False)
    pool = np.flatnonzero(np.diff(g.row_ptr) > 0)
    rate, k, dt = oracle_rate(g, pool, seconds_target, threads, gg.rng(99))
    rate1, k1, dt1 = oracle_rate(g, pool, seconds_target / 3, 1, gg.rng(98))
    return {"value": rate / 1e9, "unit": "GTEPS", "cores": threads, "kind": "oracle",
            "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "single_thread_gteps": rate1 / 1e9,
            "sample": f"{k} sources drawn uniformly from the {len(pool)} non-isolated vertices of the same graph "
                      f"(Algorithm 1, FP64, {threads} threads, {dt:.1f} s), scaled to sources x edges / s; "
                      f"single thread: {k1} sources, {dt1:.1f} s"}


def serving(args, sbc):
    """Continuous batching of a Poisson stream of BC jobs (R-MAT or deleted-edge
    grid, fair coin): latency from arrival to result on the host."""
    import threading
    from concurrent.futures import ProcessPoolExecutor

    reqs = gg.serving_stream(n_requests=args.requests, rate_per_s=args.rate)
    progress(f"serving: generating {len(reqs)} request graphs")
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        graphs = list(ex.map(gg.request_graph, reqs, chunksize=4))
    # Jobs share the device, so none takes the team kernel (a cooperative
    # launch holds every CU); deep pieces (the grid jobs, which carry most of
    # the work) get their own launch shape from the library's deep class.
    params = {"team_min_vertices": 0}
    for kv in args.param:
        k, v = kv.split("=")
        params[k] = int(v)
    ctx = sbc.Context(0, params)
    Gs = [sbc.Graph(g.n, g.row_ptr, g.col) for g in graphs]
    srv = sbc.sbc_server_create(ctx.h, args.slots, 0)
    jobs = [None] * len(reqs)
    progress("serving: stream starts")
    t0 = time.perf_counter()

    def submit_all():
        for i, r in enumerate(reqs):
            d = t0 + r.arrival_s - time.perf_counter()
            if d > 0:
                time.sleep(d)
            jobs[i] = sbc.sbc_server_submit(srv, Gs[i].h, sbc.SBC_COMPRESSED)

    th = threading.Thread(target=submit_all)
    th.start()
    lat, work = [], 0.0
    by_kind = {"rmat": [], "grid": []}
    last_done = t0
    for i in range(len(reqs)):
        while jobs[i] is None:
            time.sleep(0.001)
        bc, st = sbc.sbc_job_wait(jobs[i], graphs[i].n)
        sbc.sbc_job_release(jobs[i])
        lat.append(st["latency_ms"])
        by_kind[reqs[i].kind].append(st["latency_ms"])
        work += float(graphs[i].n) * float(graphs[i].m)
        last_done = max(last_done, time.perf_counter())
        if i % 50 == 49:
            progress(f"serving: {i + 1} jobs done, p50 so far {np.percentile(lat, 50):.1f} ms")
    th.join()
    makespan = last_done - t0
    sbc.sbc_server_destroy(srv)
    ctx.close()
    span = reqs[-1].arrival_s - reqs[0].arrival_s
    offered = work / max(span, 1e-9) / 1e9
    out = {"metric": "serving latency (arrival to result on host) and aggregate GTEPS",
           "value": work / makespan / 1e9, "unit": "GTEPS", "n_gpus": 1, "higher_is_better": True,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "max_ms": float(np.max(lat)), "mean_ms": float(np.mean(lat)), "requests": len(reqs),
           "by_kind": {k: {"jobs": len(v), "p50_ms": float(np.percentile(v, 50)), "p99_ms": float(np.percentile(v, 99))}
                       for k, v in by_kind.items() if v},
           "rate_per_s": args.rate, "makespan_s": makespan, "offered_gteps": offered,
           "config": {"workload": f"Poisson stream at {args.rate}/s of {len(reqs)} jobs: R-MAT scale 10..15 "
                                  "(decorated) or deleted-edge grid side 32..256, fair coin", "slots": args.slots,
                      "params": params,
                      "order": ("least estimated work first" if params.get("server_order", 1) == 1
                                else "oldest first")},
           "data": "synthetic", "dtype": "f64"}
    print(json.dumps(out), flush=True)


def roofline_of(stats, args_graph: bool, workload: str):
    """Roofline of the dominant traversal kernel of a compressed step: the
    class with the most algorithmic bytes (the classes' launches overlap in
    time, so the longest launch need not be the one doing the work), its
    bytes over its mean launch duration from the plan's HIP events."""
    last = stats[-1]
    k_dom = int(np.argmax(last["bytes_class"]))
    ms_dom = float(np.mean([s["ms_class"][k_dom] for s in stats]))
    bytes_dom = last["bytes_class"][k_dom]
    timing = "HIP events around the kernel's launch on its stream"
    if ms_dom <= 0 and args_graph:
        # a replayed graph records no per-launch events: the whole traversal span instead
        ms_dom = float(np.mean([s["ms_traverse"] for s in stats]))
        bytes_dom = last["algo_bytes"]
        timing = "graph replay: every traversal launch together (no per-launch events)"
    achieved = bytes_dom / (ms_dom * 1e-3) / 1e9 if ms_dom > 0 else None
    return {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS if achieved else None, "traffic": load_traffic(workload, k_dom),
            "kernel": KERNEL_SYMBOLS[k_dom], "kernel_class": CLASS_NAMES[k_dom], "launch_ms": ms_dom,
            "algo_bytes_per_launch": bytes_dom, "timing": timing}


def active_sources(g) -> int:
    """Vertices with at least one edge: the sources that traverse anything."""
    return int(np.count_nonzero(np.diff(g.row_ptr) > 0))


def compressed_leg(sbc, params, name, steps, warmup, ops):
    """Compressed step of another workload, for the same JSON line."""
    desc, make = WORKLOADS[name]
    progress(f"leg {name}: generating")
    g = make()
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    t0 = time.perf_counter()
    prep = G.preprocess(ops)
    prep_s = time.perf_counter() - t0
    ctx = sbc.Context(0, params)
    try:
        t_c, st_c, _ = timed_run(sbc, ctx, G, sbc.SBC_COMPRESSED, steps, warmup)
    finally:
        ctx.close()
        G.close()
    na = active_sources(g)
    return {"workload": f"{name}: {desc}", "n": g.n, "m": g.m, "non_isolated": na, "steps": steps,
            "warmup": warmup, "ms_per_step": t_c * 1e3, "gteps": na * g.m / t_c / 1e9,
            "raw_gteps": st_c[-1]["teps"] / t_c / 1e9, "preprocess_s": prep_s, "pieces": prep["pieces"],
            "class_ms": st_c[-1]["ms_class"], "class_items": st_c[-1]["items_class"],
            "roofline": roofline_of(st_c, False, name)}


def farness_leg(sbc, params, name, steps, warmup):
    """Closeness on the same shattered pieces ("oda"): per step, the farness
    kernel's per-piece sums, their download and the host's block-cut-tree
    pass.  Roofline of the farness kernel: per (source, piece), the CSR
    (4 (n_p + 1) + 4 a_p bytes), a level read per arc (4 a_p), a level write
    and a reach read per vertex (8 n_p): 8 a_p + 12 n_p bytes."""
    desc, make = WORKLOADS[name]
    progress(f"farness {name}: generating")
    g = make()
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    ctx = sbc.Context(0, params)
    f, pst = sbc.sbc_far_create(G.h, "oda")
    try:
        ex = sbc.sbc_far_export(f)
        npc = np.diff(ex["vtx_off"]).astype(np.float64)
        apc = np.diff(ex["row"][ex["vtx_off"]]).astype(np.float64)
        algo_bytes = float(np.sum(npc * (8 * apc + 12 * npc + 4)))
        for i in range(warmup):
            sbc.sbc_far_run(ctx.h, f, g.n)
        runs = []
        t0 = time.perf_counter()
        for i in range(steps):
            runs.append(sbc.sbc_far_run(ctx.h, f, g.n)[2])
            progress(f"farness {name} step {i}: kernel {runs[-1]['ms_kernel']:.1f} ms, total {runs[-1]['ms_total']:.1f} ms")
        t = (time.perf_counter() - t0) / steps
    finally:
        sbc.sbc_far_destroy(f)
        ctx.close()
        G.close()
    ms_k = float(np.mean([r["ms_kernel"] for r in runs]))
    na = active_sources(g)
    achieved = algo_bytes / (ms_k * 1e-3) / 1e9 if ms_k > 0 else None
    return {"workload": f"{name}: {desc}", "ops": "oda", "n": g.n, "m": g.m, "non_isolated": na, "steps": steps,
            "warmup": warmup, "ms_per_step": t * 1e3, "gteps": na * g.m / t / 1e9,
            "kernel_ms": ms_k, "raw_gteps": runs[-1]["teps"] / 1e9, "host_prep_ms": pst["ms_prep"],
            "host_finish_ms": float(np.mean([r["ms_finish"] for r in runs])), "pieces": pst["pieces"],
            "items": runs[-1]["items"], "grid": runs[-1]["grid"],
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": achieved / PEAK_HBM_GBS if achieved else None,
                         "traffic": load_traffic(name, "far64"), "kernel_class": "far64",
                         "kernel": "far_kernel<WAVES,*>", "launch_ms": ms_k, "algo_bytes_per_launch": algo_bytes,
                         "timing": "HIP events around the kernel's launch on its stream"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat17", choices=sorted(WORKLOADS))
    ap.add_argument("--ops", default="odau",
                    help="preprocessing letters (o: per-piece BFS order, Section 4.1; u: identical vertices "
                         "merged whatever their reach)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--legs", default="blocktree20000,grid512",
                    help="comma-separated workloads timed after the main one (compressed only); '' for none")
    ap.add_argument("--far", default="rmat17",
                    help="comma-separated workloads whose farness/closeness is timed too ('' for none)")
    ap.add_argument("--leg-steps", type=int, default=3)
    ap.add_argument("--leg-warmup", type=int, default=1)
    ap.add_argument("--graph", action="store_true", help="replay a captured HIP graph")
    ap.add_argument("--param", action="append", default=[], help="key=value tuning knob")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--phases", action="store_true", help="one extra compressed run with in-kernel phase timers")
    ap.add_argument("--calibrate", action="store_true", help="also time a plain streaming copy (1 GiB)")
    ap.add_argument("--autotune", action="store_true", help="apply the autotuner's choice (tuned now unless cached)")
    ap.add_argument("--serving", action="store_true", help="run the Poisson serving stream instead")
    ap.add_argument("--requests", type=int, default=600)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--slots", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); splitting the work items over several "
              "GPUs is not built", file=sys.stderr)
        sys.exit(2)

    import paper_1209_6007_amd as sbc  # no torch in this process: the library syncs its own streams

    if args.serving:
        serving(args, sbc)
        return
    desc, make = WORKLOADS[args.workload]
    if args.workload.startswith("blocktree") and not args.no_plain:
        # plain Brandes on the whole block tree (millions of vertices as one
        # piece) runs for minutes to hours: only the compressed path is timed
        progress("plain run skipped on the block tree (whole graph as one piece)")
        args.no_plain = True
    g = make()
    params = {}
    for kv in args.param:
        k, v = kv.split("=")
        params[k] = int(v)
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    t0 = time.perf_counter()
    prep = G.preprocess(args.ops)
    prep_s = time.perf_counter() - t0
    tuned = None
    if args.autotune:
        from paper_1209_6007_amd import autotune

        tuned = autotune.tune(G, sbc.SBC_COMPRESSED, row_ptr=g.row_ptr, col=g.col, log=progress)
        params = dict(tuned, **params)
    ctx = sbc.Context(0, params)
    na = active_sources(g)
    # Sources x edges: every non-isolated vertex is a source that traverses
    # its component; isolated vertices do no work and are not counted.
    work = float(na) * float(g.m)

    t_c, st_c, res_c = timed_run(sbc, ctx, G, sbc.SBC_COMPRESSED, args.steps, args.warmup, args.graph)
    out = {
        "metric": METRIC,
        "value": work / t_c / 1e9,
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
        "config": {"workload": f"{args.workload}: {desc}", "n": g.n, "m": g.m, "non_isolated": na,
                   "isolated": g.n - na, "ops": args.ops, "parallelism": "single GPU", "hip_graph": bool(args.graph),
                   "params": params, "autotuned": tuned is not None,
                   "value_definition": "non-isolated vertices x undirected edges / step time"},
    }
    last = st_c[-1]
    out["roofline"] = roofline_of(st_c, args.graph, args.workload)
    out["compressed"] = {
        "effective_gteps": work / t_c / 1e9,
        "gteps_all_labels": float(g.n) * float(g.m) / t_c / 1e9,
        "raw_gteps": last["teps"] / t_c / 1e9,
        "kernel_ms": float(np.mean([s["ms_traverse"] for s in st_c])),
        "device_ms": float(np.mean([s["ms_device"] for s in st_c])),
        "preprocess_s": prep_s,
        "end_to_end_gteps_incl_preprocess": work / (t_c + prep_s) / 1e9,
        "prep": {k: prep[k] for k in ("stripped", "blocks", "bridges", "twin_classes", "twins_merged", "pieces",
                                       "piece_vertices", "piece_arcs", "work_teps")},
        "class_ms": last["ms_class"], "class_items": last["items_class"], "class_grid": last["grid_class"],
    }
    if not args.no_plain:
        t_p, st_p, res_p = timed_run(sbc, ctx, G, sbc.SBC_PLAIN, args.steps, args.warmup, args.graph)
        nz = res_p != 0
        rel = float(np.max(np.abs(res_c[nz] - res_p[nz]) / np.abs(res_p[nz]))) if nz.any() else 0.0
        lp = st_p[-1]
        kp = int(np.argmax(lp["bytes_class"]))
        out["plain"] = {"gteps": work / t_p / 1e9, "ms_per_step": t_p * 1e3,
                        "kernel_class": CLASS_NAMES[kp],
                        "hbm_frac": lp["bytes_class"][kp] / (lp["ms_class"][kp] * 1e-3) / 1e9 / PEAK_HBM_GBS
                        if lp["ms_class"][kp] > 0 else None}
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
    ctx.close()
    G.close()
    legs = [w for w in args.legs.split(",") if w and w != args.workload]
    if legs:
        out["legs"] = {}
        for w in legs:
            out["legs"][w] = compressed_leg(sbc, params, w, args.leg_steps, args.leg_warmup, args.ops)
            progress(f"leg {w}: {out['legs'][w]['ms_per_step']:.1f} ms per step")
    fars = [w for w in args.far.split(",") if w]
    if fars:
        out["closeness"] = {}
        for w in fars:
            out["closeness"][w] = farness_leg(sbc, params, w, args.leg_steps, args.leg_warmup)
            progress(f"farness {w}: {out['closeness'][w]['ms_per_step']:.1f} ms per step")
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle) starts")
        threads = min(os.cpu_count() or 1, 16)
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_seconds, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
