"""Farness and closeness on the GPU against the oracle, bit for bit (all
values are exact int64): the device's per-piece sums against
oracle.farness_pieces on the exported pieces, and the farness of every vertex
after the host pass against oracle.farness on the original graph -- at small
sizes in every workgroup shape and preprocessing, with empty and edge-free
graphs, and at the benchmark workloads' full sizes (R-MAT scale 17, the
512x512 grid, the 20,000-piece block tree)."""
import time

import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_1209_6007_amd as sbc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    oracle.build(force=False)
    c = sbc.Context(0)
    yield c
    c.close()


def run(ctx, g, ops):
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    f, pst = sbc.sbc_far_create(G.h, ops)
    try:
        ex = sbc.sbc_far_export(f)
        far, clo, st, W = sbc.sbc_far_run(ctx.h, f, g.n, with_piece_sums=True)
    finally:
        sbc.sbc_far_destroy(f)
        G.close()
    return far, clo, st, W, ex, pst


def check_pieces(W, ex, what):
    if len(ex["vtx_off"]) > 1:
        want = oracle.farness_pieces(ex["vtx_off"], ex["row"], ex["col"], ex["reach"])
        bad = np.nonzero(W != want)[0]
        assert bad.size == 0, (what, bad[:5], W[bad[:5]], want[bad[:5]])


CASES = [
    ("decorated", lambda: gg.decorated_random(300, 0.01, 80, 20, 20, 11)),
    ("rmat12", lambda: gg.rmat_decorated(scale=12, seed=5)),
    ("grid60", lambda: gg.grid_deleted(side=60, seed=7)),
    ("blocks", lambda: gg.block_tree(n_pieces=120, max_size=300, seed=9)),
    ("er3000", lambda: gg.erdos_renyi(3000, 0.002, 4)),
    ("path200", lambda: gg.path(200)),
    ("K70", lambda: gg.complete(70)),
]


@pytest.mark.parametrize("waves", [4, 8, 16])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_farness_vs_oracle(name, make, waves):
    g = make()
    print(f"farness {name} n={g.n} waves={waves}", flush=True)
    c = sbc.Context(0, {"far_wg_waves": waves})
    want = oracle.farness(g.n, g.row_ptr, g.col)
    try:
        for ops in ("oda", "da", ""):
            far, clo, st, W, ex, _ = run(c, g, ops)
            check_pieces(W, ex, (name, ops))
            assert np.array_equal(far, want), (name, ops)
            assert st["flags"] == 0
    finally:
        c.close()


def test_slot_reuse_with_two_slots(ctx):
    """Many items through two resident workgroups: each item leaves its
    slot's masks clean for the next."""
    g = gg.block_tree(n_pieces=60, max_size=200, seed=3)
    c = sbc.Context(0, {"slots": 2})
    try:
        far, _, st, W, ex, _ = run(c, g, "oda")
        assert st["grid"] == 2 and st["items"] > 60
        check_pieces(W, ex, "two slots")
        assert np.array_equal(far, oracle.farness(g.n, g.row_ptr, g.col))
    finally:
        c.close()


def test_edge_free_and_empty_graphs(ctx):
    g = gg.csr_from_edges(5, np.zeros(0, np.int64), np.zeros(0, np.int64))
    far, clo, st, W, ex, _ = run(ctx, g, "oda")
    assert np.all(far == 0) and np.all(clo == 0) and W.size == 0
    g = gg.csr_from_edges(0, np.zeros(0, np.int64), np.zeros(0, np.int64))
    far, clo, st, W, ex, _ = run(ctx, g, "")
    assert far.size == 0


def test_closeness_values(ctx):
    g = gg.rmat_decorated(scale=11, seed=2)
    far, clo, _, _, _, _ = run(ctx, g, "oda")
    want = oracle.farness(g.n, g.row_ptr, g.col)
    comp = gg.components(g)
    size = np.bincount(comp)[comp]
    assert np.array_equal(far, want)
    assert np.array_equal(clo, np.where(want > 0, (size - 1) / np.maximum(want, 1), 0.0))


def timed(label, fn):
    t0 = time.perf_counter()
    out = fn()
    print(f"{label}: {time.perf_counter() - t0:.1f} s", flush=True)
    return out


@pytest.mark.parametrize("name", ["rmat17", "grid512"])
def test_full_size_vs_oracle(ctx, name):
    g = gg.rmat_decorated() if name == "rmat17" else gg.grid_deleted()
    far, _, st, W, ex, pst = timed(f"{name} device", lambda: run(ctx, g, "oda"))
    print(f"{name}: kernel {st['ms_kernel']:.1f} ms, {pst['pieces']} pieces", flush=True)
    check_pieces(W, ex, name)
    want = timed(f"{name} oracle", lambda: oracle.farness(g.n, g.row_ptr, g.col))
    assert np.array_equal(far, want)


def test_block_tree_full_size_piece_sums(ctx):
    g = gg.block_tree()
    far, _, st, W, ex, pst = timed("blocktree20000 device", lambda: run(ctx, g, "oda"))
    print(f"blocktree20000: kernel {st['ms_kernel']:.1f} ms, {pst['pieces']} pieces", flush=True)
    timed("blocktree20000 oracle pieces", lambda: check_pieces(W, ex, "blocktree20000"))
    # the whole-graph farness of sampled vertices: one search each over all
    # 13.1M vertices (every vertex of a block tree is in one component)
    src = gg.rng(31).choice(g.n, 32, replace=False).astype(np.int32)
    want = timed("blocktree20000 oracle samples", lambda: oracle.farness(g.n, g.row_ptr, g.col, sources=src))
    assert np.array_equal(far[src], want)
    assert np.all(far > 0)
