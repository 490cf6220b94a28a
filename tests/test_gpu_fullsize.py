"""GPU parity at the benchmark workloads' full sizes, in the launch
configuration bench.py times (default context), on outputs the oracle can
compute: sampled sources (Algorithm 1 restricted to them), single pieces of
the full shattered graph (Algorithm 2 with ident weights on the piece), and
properties that hold at any size (compressed equals plain)."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_1209_6007_amd as sbc
from tests.helpers import assert_bc_close

pytestmark = pytest.mark.gpu
RTOL = 1e-9


@pytest.fixture(scope="module")
def ctx():
    oracle.build(force=False)
    c = sbc.Context(0)
    yield c
    c.close()


def sampled_sources(ctx, g, k, seed):
    src = gg.rng(seed).choice(g.n, size=k, replace=False).astype(np.int32)
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    got = sbc.sbc_betweenness_sources(ctx.h, G.h, src)
    want = oracle.bc_plain(g.n, g.row_ptr, g.col, sources=src)
    return got, want


def test_rmat17_sampled_sources(ctx):
    """R-MAT scale 17 (the benchmark graph): 128 sampled sources through the
    plain path (one piece of 170,394 vertices on the team kernel)."""
    g = gg.rmat_decorated()
    got, want = sampled_sources(ctx, g, 128, 11)
    assert_bc_close(got, want, RTOL, "rmat17 sampled sources")


def test_rmat17_compressed_equals_plain(ctx):
    """Theorem 1 at full size: the compressed run (odai) equals the plain run."""
    g = gg.rmat_decorated()
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    G.preprocess("odai")
    comp = sbc.sbc_betweenness(ctx.h, G.h, sbc.SBC_COMPRESSED)
    plain = sbc.sbc_betweenness(ctx.h, G.h, sbc.SBC_PLAIN)
    assert_bc_close(comp, plain, RTOL, "rmat17 compressed vs plain")


def test_grid512_sampled_sources(ctx):
    """512x512 grid with 12% of edges deleted: 64 sampled sources, ~800 levels."""
    g = gg.grid_deleted()
    got, want = sampled_sources(ctx, g, 64, 12)
    assert_bc_close(got, want, RTOL, "grid512 sampled sources")


def test_grid_compressed_equals_plain(ctx):
    g = gg.grid_deleted(side=128, seed=21)
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    G.preprocess("odai")
    comp = sbc.sbc_betweenness(ctx.h, G.h, sbc.SBC_COMPRESSED)
    plain = sbc.sbc_betweenness(ctx.h, G.h, sbc.SBC_PLAIN)
    assert_bc_close(comp, plain, RTOL, "grid128 compressed vs plain")
    assert_bc_close(plain, oracle.bc(g), RTOL, "grid128 plain vs oracle")


def test_block_tree_full_run_and_sampled_pieces(ctx):
    """The 20,000-piece block tree in one persistent launch per kernel class;
    a sample of its pieces (as shattered, with reach) checked one by one
    against Algorithm 2 with ident weights on the oracle."""
    g = gg.block_tree()
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    st = G.preprocess("odai")
    print(f"block tree n={g.n} m={g.m} pieces={st['pieces']} piece_vertices={st['piece_vertices']}", flush=True)
    bc = sbc.sbc_betweenness(ctx.h, G.h, sbc.SBC_COMPRESSED)
    assert np.all(np.isfinite(bc)) and np.all(bc >= 0)
    deg = np.diff(g.row_ptr)
    assert np.all(bc[deg == 1] == 0)
    ex = sbc.sbc_graph_export(G.h)
    vo = ex["vtx_off"]
    sizes = np.diff(vo)
    r = gg.rng(13)
    picks = list(r.choice(len(sizes), size=6, replace=False)) + [int(np.argmax(sizes))]
    for p in picks:
        vb, ve = int(vo[p]), int(vo[p + 1])
        rp = (ex["row"][vb:ve + 1] - ex["row"][vb]).astype(np.int32)
        cl = ex["col"][ex["row"][vb]:ex["row"][ve]].astype(np.int32)
        reach, ident = ex["reach"][vb:ve], ex["ident"][vb:ve]
        got = sbc.sbc_piece_bc(ctx.h, ve - vb, rp, cl, reach, ident)
        want = oracle.bc_weighted(ve - vb, rp, cl, reach, ident)
        assert_bc_close(got, want, RTOL, f"block tree piece {p} (n={ve - vb})")


def test_block_tree_200_pieces_vs_oracle(ctx):
    """200 blocks of the same recipe: the whole compressed result against
    Algorithm 1 on the uncompressed graph."""
    g = gg.block_tree(n_pieces=200, seed=gg.SEED_BASE + 33)
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    G.preprocess("odai")
    got = sbc.sbc_betweenness(ctx.h, G.h, sbc.SBC_COMPRESSED)
    assert_bc_close(got, oracle.bc(g), RTOL, "block tree 200 pieces")


def test_small_piece_block_tree_full_run(ctx):
    """The 20,000-piece block tree of 8..256-vertex blocks (the small-piece
    workload), in the launch configuration the bench times: equal to the same
    run with every piece on the batch kernel, and a sample of its pieces
    checked one by one against Algorithm 2 with ident weights on the oracle."""
    g = gg.block_tree(max_size=256)
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    st = G.preprocess("odai")
    print(f"small-piece block tree n={g.n} m={g.m} pieces={st['pieces']}", flush=True)
    plan = sbc.sbc_plan_create(ctx.h, G.h, sbc.SBC_COMPRESSED)
    try:
        sbc.sbc_plan_execute(plan)
        rs = sbc.sbc_plan_sync(plan)
        bc = sbc.sbc_plan_result(plan, g.n)
    finally:
        sbc.sbc_plan_destroy(plan)
    assert rs["items_class"][0] > 0 and rs["items_class"][2] == 0, rs["items_class"]
    batch = sbc.Context(0, {"wave_max_vertices": 0})
    ref = sbc.sbc_betweenness(batch.h, G.h, sbc.SBC_COMPRESSED)
    batch.close()
    assert_bc_close(bc, ref, 1e-12, "small-piece kernel vs batch kernel")
    ex = sbc.sbc_graph_export(G.h)
    vo = ex["vtx_off"]
    sizes = np.diff(vo)
    r = gg.rng(17)
    picks = list(r.choice(len(sizes), size=8, replace=False)) + [int(np.argmax(sizes))]
    for p in picks:
        vb, ve = int(vo[p]), int(vo[p + 1])
        rp = (ex["row"][vb:ve + 1] - ex["row"][vb]).astype(np.int32)
        cl = ex["col"][ex["row"][vb]:ex["row"][ve]].astype(np.int32)
        reach, ident = ex["reach"][vb:ve], ex["ident"][vb:ve]
        got = sbc.sbc_piece_bc(ctx.h, ve - vb, rp, cl, reach, ident, kernel=5)
        want = oracle.bc_weighted(ve - vb, rp, cl, reach, ident)
        assert_bc_close(got, want, RTOL, f"small-piece block tree piece {p} (n={ve - vb})")
