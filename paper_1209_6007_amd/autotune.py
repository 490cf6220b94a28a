"""Autotuner for the traversal kernels.

A workload is put in a bucket by its largest piece: a size class and a depth
class (breadth-first depth from the piece's highest-degree vertex, a lower
bound on the piece's diameter and at least half of it).  For each bucket the
tuner times a short run of every candidate configuration on the device and
keeps the fastest:

* which kernel runs the large pieces: the team kernel (all workgroups of an
  XCD share one 64-source batch) or one workgroup per batch, i.e. the
  small/large threshold ``team_min_vertices``, and ``team_max_levels``, which
  keeps deep pieces off the team kernel;
* the workgroup shape of one-workgroup batches (``batch_wg_waves``) and the
  number of teams (the team kernel keeps ``team_wg_waves``, whose 16 and 8
  waves measured within 2% of each other);
* then, with that choice fixed, whether small pieces run on the small-piece
  kernel (one source per wavefront, the piece in LDS) and its workgroup
  shape (``wave_max_vertices``, ``wave_wg_waves``), when the workload has
  pieces small enough for it;
* and, when its largest piece is deep (more levels than ``deep_min_levels``),
  the workgroup shape of the deep pieces' own launch (``deep_wg_waves``,
  ``deep_waves_per_eu``).

Runs are sampled (``sample_items``: an evenly spaced subset of the work
items, the same fraction of every kernel class) yet keep the device fully
loaded: eight rounds of the resident workgroups for one workgroup per batch,
four items per team for the team kernel.  The sampled time is scaled by the
number of items to estimate a full run.  Results are cached in a JSON file
per device (``$SBC_AUTOTUNE_CACHE`` or ``~/.cache/shatterbc/autotune.json``),
keyed by device name and bucket.

  python -m paper_1209_6007_amd.autotune --workload rmat17 [--force]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import (SBC_COMPRESSED, SBC_PLAIN, Context, Graph, sbc_context_device_name, sbc_context_get_param,
               sbc_graph_export, sbc_plan_create, sbc_plan_destroy, sbc_plan_execute, sbc_plan_sync)

SIZE_CLASSES = ((4096, "s"), (32768, "m"), (None, "l"))  # largest piece < bound -> class
DEEP_LEVELS = 32          # depth above this: "deep"
BATCH_ROUNDS = 8          # rounds of resident workgroups in a one-workgroup-per-batch run
WAVES_PER_CU = 32         # resident waves per compute unit at eight waves per SIMD
TEAM_ROUNDS = 4           # items per team in a team-kernel run

# Candidate configurations of the large pieces' kernels.  Every one sets
# every tuned key, so that the choice does not depend on the context it is
# applied to; the small-piece keys are at their defaults here.
_WAVE_DEFAULT = {"wave_max_vertices": 256, "wave_wg_waves": 4, "deep_wg_waves": 16, "deep_waves_per_eu": 0}
CANDIDATES = [dict(c, **_WAVE_DEFAULT) for c in (
    {"team_min_vertices": 0, "batch_wg_waves": 8, "batch_waves_per_eu": 8, "team_count": 64, "team_max_levels": 0},
    {"team_min_vertices": 0, "batch_wg_waves": 16, "batch_waves_per_eu": 8, "team_count": 64, "team_max_levels": 0},
    {"team_min_vertices": 0, "batch_wg_waves": 4, "batch_waves_per_eu": 8, "team_count": 64, "team_max_levels": 0},
    {"team_min_vertices": 4096, "batch_wg_waves": 8, "batch_waves_per_eu": 8, "team_count": 32, "team_max_levels": 0},
    {"team_min_vertices": 4096, "batch_wg_waves": 8, "batch_waves_per_eu": 8, "team_count": 64, "team_max_levels": 0},
    {"team_min_vertices": 4096, "batch_wg_waves": 8, "batch_waves_per_eu": 8, "team_count": 128, "team_max_levels": 0},
)]
TUNED_KEYS = sorted(CANDIDATES[0])
# Second stage: the small-piece kernel off, or on with 4 or 8 waves per
# workgroup and a lower size threshold.
SMALL_CANDIDATES = [
    {"wave_max_vertices": 0, "wave_wg_waves": 4},
    {"wave_max_vertices": 256, "wave_wg_waves": 4},
    {"wave_max_vertices": 256, "wave_wg_waves": 8},
    {"wave_max_vertices": 128, "wave_wg_waves": 8},
]
# Third stage, for workloads whose largest piece is deeper than the deep
# class's threshold: the deep launch's workgroup shape.
DEEP_MIN_LEVELS = 64  # the library's default deep_min_levels
DEEP_CANDIDATES = [
    {"deep_wg_waves": 16, "deep_waves_per_eu": 0},
    {"deep_wg_waves": 16, "deep_waves_per_eu": 8},
    {"deep_wg_waves": 8, "deep_waves_per_eu": 0},
    {"deep_wg_waves": 8, "deep_waves_per_eu": 8},
]


def cache_path() -> str:
    return os.environ.get("SBC_AUTOTUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "shatterbc",
                                                                 "autotune.json")


def bfs_depth(row_ptr: np.ndarray, col: np.ndarray) -> int:
    """Levels of a breadth-first search from the highest-degree vertex."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import breadth_first_order

    n = len(row_ptr) - 1
    if n <= 1:
        return 0
    start = int(np.argmax(np.diff(row_ptr)))
    a = csr_matrix((np.ones(len(col), np.int8), np.asarray(col), np.asarray(row_ptr)), shape=(n, n))
    order, pred = breadth_first_order(a, start, directed=True, return_predecessors=True)
    depth = np.zeros(n, np.int64)
    for v in order[1:]:  # predecessors come earlier in the order
        depth[v] = depth[pred[v]] + 1
    return int(depth[order].max())


def bucket_of(piece_vertices: int, depth: int) -> str:
    size = next(name for bound, name in SIZE_CLASSES if bound is None or piece_vertices < bound)
    return f"{size}-{'deep' if depth > DEEP_LEVELS else 'shallow'}"


def workload_bucket(graph: Graph, mode: int = SBC_COMPRESSED, n: int = 0, row_ptr=None, col=None) -> tuple:
    """(bucket, largest piece size, its depth) of a prepared graph (compressed
    mode) or of the whole graph (plain mode: pass row_ptr and col)."""
    if mode == SBC_PLAIN:
        rp, cl = np.asarray(row_ptr, np.int64), np.asarray(col, np.int64)
        depth = bfs_depth(rp, cl)
        return bucket_of(len(rp) - 1, depth), len(rp) - 1, depth
    ex = sbc_graph_export(graph.h)
    vo = ex["vtx_off"]
    if len(vo) < 2:
        return bucket_of(0, 0), 0, 0
    p = int(np.argmax(np.diff(vo)))
    vb, ve = int(vo[p]), int(vo[p + 1])
    rp = (ex["row"][vb:ve + 1] - ex["row"][vb]).astype(np.int64)
    cl = ex["col"][ex["row"][vb]:ex["row"][ve]].astype(np.int64)
    depth = bfs_depth(rp, cl)
    return bucket_of(ve - vb, depth), ve - vb, depth


def smallest_piece(graph: Graph, mode: int, n: int) -> int:
    """Vertices of the smallest piece with at least one source."""
    if mode == SBC_PLAIN:
        return n
    sizes = np.diff(sbc_graph_export(graph.h)["vtx_off"])
    sizes = sizes[sizes > 0]
    return int(sizes.min()) if len(sizes) else 0


def total_items(graph: Graph, mode: int, n: int) -> int:
    """(piece, 64 sources) items of a full run."""
    if mode == SBC_PLAIN:
        return (n + 63) // 64
    sizes = np.diff(sbc_graph_export(graph.h)["vtx_off"])
    return int(np.sum((sizes + 63) // 64))


def sample_for(params: dict, cus: int = 256) -> int:
    """Items of the largest kernel class in a sampled run (the other classes
    keep the same fraction of theirs): several rounds of the resident
    workgroups (a run of one or two rounds measures its slowest item, not the
    throughput), or TEAM_ROUNDS items per team."""
    if params.get("team_min_vertices", 0) > 0:
        return TEAM_ROUNDS * int(params.get("team_count", 64))
    waves = int(params.get("batch_wg_waves", 8))
    return BATCH_ROUNDS * cus * max(1, WAVES_PER_CU // waves)


def _time_candidate(params: dict, graph: Graph, mode: int, device: int, full_items: int, cus: int = 256) -> float:
    """Estimated milliseconds of a full run under params."""
    ctx = Context(device, dict(params, sample_items=sample_for(params, cus)))
    try:
        plan = sbc_plan_create(ctx.h, graph.h, mode)
        try:
            sbc_plan_execute(plan)
            st = sbc_plan_sync(plan)
            return float(st["ms_traverse"]) * full_items / max(1, int(st["items"]))
        finally:
            sbc_plan_destroy(plan)
    finally:
        ctx.close()


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save_cache(d: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cache_key(device_name: str, bucket: str, mode: int) -> str:
    return f"{device_name}|{'plain' if mode == SBC_PLAIN else 'compressed'}|{bucket}"


def tune(graph: Graph, mode: int = SBC_COMPRESSED, device: int = 0, row_ptr=None, col=None, force: bool = False,
         path: str | None = None, log=None) -> dict:
    """Best parameters for the graph's bucket (tuned now unless cached)."""
    bucket, np_max, depth = workload_bucket(graph, mode, row_ptr=row_ptr, col=col)
    probe = Context(device)
    name = sbc_context_device_name(probe.h)
    cus = int(sbc_context_get_param(probe.h, "cus"))
    probe.close()
    key = cache_key(name, bucket, mode)
    cache = load_cache(path)
    if key in cache and not force:
        return dict(cache[key]["params"])
    n = len(row_ptr) - 1 if row_ptr is not None else 0
    full = total_items(graph, mode, n)
    results = []
    for cand in CANDIDATES:
        t0 = time.perf_counter()
        ms = _time_candidate(cand, graph, mode, device, full, cus)
        results.append((ms, cand))
        if log:
            log(f"autotune {key}: {cand} -> {ms:.1f} ms estimated ({time.perf_counter() - t0:.1f} s)")
    ms, best = min(results, key=lambda r: r[0])
    small = []
    smin = smallest_piece(graph, mode, n)
    if 0 < smin <= max(c["wave_max_vertices"] for c in SMALL_CANDIDATES):
        for opt in SMALL_CANDIDATES:
            cand = dict(best, **opt)
            t0 = time.perf_counter()
            m = _time_candidate(cand, graph, mode, device, full, cus)
            small.append((m, cand))
            if log:
                log(f"autotune {key}: small pieces {opt} -> {m:.1f} ms estimated ({time.perf_counter() - t0:.1f} s)")
        ms, best = min(small, key=lambda r: r[0])
    deep = []
    if depth > DEEP_MIN_LEVELS:
        for opt in DEEP_CANDIDATES:
            cand = dict(best, **opt)
            t0 = time.perf_counter()
            m = _time_candidate(cand, graph, mode, device, full, cus)
            deep.append((m, cand))
            if log:
                log(f"autotune {key}: deep pieces {opt} -> {m:.1f} ms estimated ({time.perf_counter() - t0:.1f} s)")
        ms, best = min(deep, key=lambda r: r[0])
    cache[key] = {"params": best, "estimated_ms": ms, "piece_vertices": int(np_max), "depth": int(depth),
                  "items": full, "candidates": [{"params": c, "estimated_ms": m} for m, c in results],
                  "small_candidates": [{"params": c, "estimated_ms": m} for m, c in small],
                  "deep_candidates": [{"params": c, "estimated_ms": m} for m, c in deep]}
    save_cache(cache, path)
    return dict(best)


def apply(ctx: Context, params: dict) -> None:
    from . import sbc_context_set_param

    for k in TUNED_KEYS:
        if k in params:
            sbc_context_set_param(ctx.h, k, int(params[k]))


def main(argv=None):
    import graphgen as gg  # the seeded workload generators (repository root)

    ap = argparse.ArgumentParser(prog="python -m paper_1209_6007_amd.autotune")
    ap.add_argument("--workload", default="rmat17", choices=sorted(gg.WORKLOADS))
    ap.add_argument("--mode", default="compressed", choices=["compressed", "plain"])
    ap.add_argument("--ops", default="odau")
    ap.add_argument("--force", action="store_true")
    ap.add_argument("--cache")
    a = ap.parse_args(argv)
    g = gg.WORKLOADS[a.workload]()
    G = Graph(g.n, g.row_ptr, g.col)
    mode = SBC_COMPRESSED if a.mode == "compressed" else SBC_PLAIN
    if mode == SBC_COMPRESSED:
        G.preprocess(a.ops)
    best = tune(G, mode, row_ptr=g.row_ptr, col=g.col, force=a.force, path=a.cache, log=print)
    print(json.dumps({"workload": a.workload, "mode": a.mode, "params": best}))


if __name__ == "__main__":
    main()
