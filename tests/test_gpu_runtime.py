"""GPU: autotuner choices, sampled tuning plans and the serving loop, through
the C interface, against the oracle."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_1209_6007_amd as sbc
from paper_1209_6007_amd import autotune as at
from tests.helpers import assert_bc_close

pytestmark = pytest.mark.gpu
RTOL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def _oracle():
    oracle.build(force=False)


def test_autotune_choice_gives_exact_result(tmp_path):
    g = gg.rmat_decorated(scale=12, seed=31)
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    G.preprocess("odai")
    path = str(tmp_path / "tune.json")
    best = at.tune(G, sbc.SBC_COMPRESSED, row_ptr=g.row_ptr, col=g.col, path=path, log=print)
    entry = next(iter(at.load_cache(path).values()))
    assert len(entry["candidates"]) == len(at.CANDIDATES)
    assert entry["small_candidates"] == []  # one piece, far above the small-piece sizes
    assert entry["params"] == best and all(c["estimated_ms"] > 0 for c in entry["candidates"])
    # cached: no new timing
    assert at.tune(G, sbc.SBC_COMPRESSED, row_ptr=g.row_ptr, col=g.col, path=path) == best
    ctx = sbc.Context(0)
    at.apply(ctx, best)
    assert_bc_close(sbc.sbc_betweenness(ctx.h, G.h, sbc.SBC_COMPRESSED), oracle.bc(g), RTOL, "autotuned")
    ctx.close()


def test_autotune_small_piece_stage(tmp_path):
    """A block tree of small pieces: the second stage times the small-piece
    options with the first stage's choice, and its pick is exact."""
    g = gg.block_tree(n_pieces=200, max_size=300, seed=41)
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    G.preprocess("odai")
    path = str(tmp_path / "tune.json")
    best = at.tune(G, sbc.SBC_COMPRESSED, row_ptr=g.row_ptr, col=g.col, path=path, log=print)
    entry = next(iter(at.load_cache(path).values()))
    assert len(entry["small_candidates"]) == len(at.SMALL_CANDIDATES)
    assert entry["params"] == best and sorted(best) == at.TUNED_KEYS
    ctx = sbc.Context(0)
    at.apply(ctx, best)
    assert_bc_close(sbc.sbc_betweenness(ctx.h, G.h, sbc.SBC_COMPRESSED), oracle.bc(g), RTOL, "autotuned small")
    ctx.close()


def test_sampled_estimate_of_a_two_class_plan():
    """A block tree with small pieces (small-piece kernel) and larger ones
    (batch kernel): a sampled plan keeps the same fraction of both classes'
    items, and its scaled time estimates the full run's within 35%."""
    g = gg.block_tree(n_pieces=4000, max_size=2048, seed=47)
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    G.preprocess("odai")

    def run(params, reps):
        ctx = sbc.Context(0, params)
        plan = sbc.sbc_plan_create(ctx.h, G.h, sbc.SBC_COMPRESSED)
        try:
            ts = []
            for _ in range(reps):
                sbc.sbc_plan_execute(plan)
                st = sbc.sbc_plan_sync(plan)
                ts.append(st["ms_traverse"])
        finally:
            sbc.sbc_plan_destroy(plan)
            ctx.close()
        return st, float(np.median(ts))

    full, t_full = run({}, 3)
    assert full["items_class"][0] > 0 and full["items_class"][2] > 0, full["items_class"]
    keep = full["items_class"][2] // 4
    samp, t_samp = run({"sample_items": keep}, 3)
    for k in (0, 2):
        frac = samp["items_class"][k] / full["items_class"][k]
        assert abs(frac - 0.25) <= 1.0 / full["items_class"][k] + 0.01, (k, samp["items_class"], full["items_class"])
    est = t_samp * full["items"] / samp["items"]
    print(f"full {t_full:.2f} ms, sampled {t_samp:.2f} ms, estimate {est:.2f} ms", flush=True)
    assert 0.65 * t_full <= est <= 1.35 * t_full


@pytest.mark.parametrize("team", [0, 3])
def test_sampled_plan_runs_the_sample(team):
    """sample_items keeps an evenly spaced subset of each class's items (here 3
    of the plain piece's 64-source items)."""
    g = gg.rmat_decorated(scale=11, seed=5)
    ctx = sbc.Context(0, {"sample_items": 3, "team_min_vertices": team})
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    plan = sbc.sbc_plan_create(ctx.h, G.h, sbc.SBC_PLAIN)
    sbc.sbc_plan_execute(plan)
    st = sbc.sbc_plan_sync(plan)
    got = sbc.sbc_plan_result(plan, g.n)
    sbc.sbc_plan_destroy(plan)
    assert st["items"] == 3 and st["batched_sources"] == 3 * 64
    # a partial sum of Algorithm 1: nonnegative, finite, below the full result
    full = oracle.bc(g)
    assert np.all(np.isfinite(got)) and np.all(got >= 0) and got.sum() > 0
    assert np.all(got <= full * (1 + 1e-9) + 1e-9)
    ctx.close()


@pytest.mark.parametrize("deterministic", [False, True])
def test_server_mix_equals_alone(deterministic):
    """Jobs of different sizes and shapes served together give the results of
    the same jobs run alone (and the oracle's): bit for bit in deterministic
    mode, to 1e-12 otherwise (device atomics add in another order)."""
    graphs = [gg.rmat_decorated(scale=s, seed=40 + s) for s in (9, 10, 11)] + \
             [gg.grid_deleted(side=sd, seed=50 + sd) for sd in (20, 33, 47, 90)] + [gg.ba_pendant_triangles()]
    mode = "compressed+deterministic" if deterministic else "compressed"
    ctx = sbc.Context(0)
    alone = [sbc.betweenness(g.n, g.row_ptr, g.col, mode=mode, ops="odai", ctx=ctx) for g in graphs]
    Gs = [sbc.Graph(g.n, g.row_ptr, g.col) for g in graphs]
    srv = sbc.sbc_server_create(ctx.h, 3, 0)
    jobs = [sbc.sbc_server_submit(srv, G.h, sbc._mode(mode)) for G in Gs]
    for g, j, a in zip(graphs, jobs, alone):
        got, st = sbc.sbc_job_wait(j, g.n)
        sbc.sbc_job_release(j)
        assert st["latency_ms"] > 0
        if deterministic:
            np.testing.assert_array_equal(got, a)
        else:
            assert_bc_close(got, a, 1e-12, "mix vs alone")
        assert_bc_close(got, oracle.bc(g), RTOL, "mix vs oracle")
    sbc.sbc_server_destroy(srv)
    ctx.close()


@pytest.mark.parametrize("order", [0, 1])
def test_server_order(order):
    """One slot, busy with a deep grid job while two more grid jobs and two
    small R-MAT jobs arrive: least-estimated-work-first runs the small jobs
    before the waiting grid jobs; oldest-first runs them in arrival order.
    Every result equals the oracle's either way."""
    graphs = [gg.grid_deleted(side=120, seed=61), gg.grid_deleted(side=110, seed=62),
              gg.grid_deleted(side=100, seed=63), gg.rmat_decorated(scale=8, seed=64),
              gg.rmat_decorated(scale=8, seed=65)]
    ctx = sbc.Context(0, {"server_order": order})
    Gs = [sbc.Graph(g.n, g.row_ptr, g.col) for g in graphs]
    for G in Gs:
        G.preprocess("odai")  # before submission, so that the first job is still running at the last submit
    srv = sbc.sbc_server_create(ctx.h, 1, 0)
    jobs = [sbc.sbc_server_submit(srv, G.h, sbc.SBC_COMPRESSED) for G in Gs]
    starts = []
    for g, j in zip(graphs, jobs):
        got, st = sbc.sbc_job_wait(j, g.n)
        sbc.sbc_job_release(j)
        starts.append(st["submit_to_start_ms"])
        assert_bc_close(got, oracle.bc(g), RTOL, f"order {order}")
    sbc.sbc_server_destroy(srv)
    ctx.close()
    print("waits before start (ms):", [round(x, 1) for x in starts], flush=True)
    small_first = max(starts[3], starts[4]) < min(starts[1], starts[2])
    assert small_first == (order == 1), starts
