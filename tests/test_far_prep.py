"""Farness and closeness, host side (no GPU): the library's preparation of the
shattered pieces and its pass over the block-cut tree, fed with per-piece sums
that the oracle computes (oracle.farness_pieces on the exported pieces), must
give the oracle's farness of the whole graph exactly.

This checks the decomposition (degree-1 stripping, articulation shattering
with bridges as two-vertex blocks, the reach of copies and the
up-and-down pass) independently of the device kernel, which
test_gpu_far.py checks against the same oracle.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_1209_6007_amd as sbc

OPS = ["", "d", "a", "da", "oda", "o"]


def setup_module(_m):
    oracle.build(force=False)


def host_far(g, ops):
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    f, st = sbc.sbc_far_create(G.h, ops)
    try:
        ex = sbc.sbc_far_export(f)
        if len(ex["vtx_off"]) > 1:
            W = oracle.farness_pieces(ex["vtx_off"], ex["row"], ex["col"], ex["reach"], threads=1)
        else:
            W = np.zeros(0, np.int64)
        far, clo = sbc.sbc_far_finish(f, g.n, W)
        return far, clo, st, ex
    finally:
        sbc.sbc_far_destroy(f)
        G.close()


def test_all_six_vertex_graphs():
    """Every labelled graph on 6 vertices (2^15), shattered and stripped."""
    bad = []
    for idx, g in enumerate(gg.all_graphs(6)):
        want = oracle.farness(g.n, g.row_ptr, g.col, threads=1)
        for ops in ("da", ""):
            far, _, _, _ = host_far(g, ops)
            if not np.array_equal(far, want):
                bad.append((idx, ops))
    assert not bad, bad[:10]


@pytest.mark.parametrize("seed", range(12))
def test_random_decorated_graphs(seed):
    r = gg.rng(seed + 900)
    g = gg.decorated_random(int(r.integers(20, 120)), float(r.uniform(0.02, 0.12)), int(r.integers(0, 40)),
                            int(r.integers(0, 10)), int(r.integers(0, 10)), seed)
    want = oracle.farness(g.n, g.row_ptr, g.col)
    for ops in OPS:
        far, clo, _, _ = host_far(g, ops)
        assert np.array_equal(far, want), ops


@pytest.mark.parametrize("seed", range(4))
def test_block_trees_and_trees(seed):
    for g in (gg.block_tree(n_pieces=40, max_size=30, seed=seed + 1), gg.random_tree(80, seed),
              gg.binary_tree(31), gg.path(30), gg.star(9)):
        want = oracle.farness(g.n, g.row_ptr, g.col)
        for ops in OPS:
            far, _, _, _ = host_far(g, ops)
            assert np.array_equal(far, want), (g.name, ops)


def test_disconnected_graph_with_isolated_vertices_and_closeness():
    a = gg.erdos_renyi(30, 0.08, 7)
    b = gg.cycle(6)
    n = a.n + b.n + 3  # three isolated vertices at the end
    u = [int(x) for v in range(a.n) for x in [v] * int(a.row_ptr[v + 1] - a.row_ptr[v])]
    edges = [(u[e], int(a.col[e])) for e in range(len(a.col)) if u[e] < a.col[e]]
    edges += [(a.n + i, a.n + (i + 1) % 6) for i in range(6)]
    g = gg.csr_from_edges(n, np.array([e[0] for e in edges]), np.array([e[1] for e in edges]))
    want = oracle.farness(g.n, g.row_ptr, g.col)
    comp = gg.components(g)
    size = np.bincount(comp)[comp]
    for ops in OPS:
        far, clo, _, _ = host_far(g, ops)
        assert np.array_equal(far, want), ops
        want_c = np.where(want > 0, (size - 1) / np.maximum(want, 1), 0.0)
        assert np.array_equal(clo, want_c), ops
    assert np.all(far[-3:] == 0) and np.all(clo[-3:] == 0.0)


def test_copy_reach_sums_to_component_size():
    g = gg.rmat_decorated(scale=9, seed=4)
    comp = gg.components(g)
    size = np.bincount(comp)
    _, _, st, ex = host_far(g, "oda")
    assert st["pieces"] == len(ex["vtx_off"]) - 1 and st["blocks"] >= st["pieces"] and st["stripped"] > 0
    for p in range(len(ex["vtx_off"]) - 1):
        b, e = ex["vtx_off"][p], ex["vtx_off"][p + 1]
        assert int(ex["reach"][b:e].sum()) == int(size[comp[ex["orig"][b]]]), p


def test_rmat_and_grid_shattered():
    for g in (gg.rmat_decorated(scale=10, seed=8), gg.grid_deleted(side=40, seed=3)):
        want = oracle.farness(g.n, g.row_ptr, g.col)
        for ops in ("oda", "da", ""):
            far, _, _, _ = host_far(g, ops)
            assert np.array_equal(far, want), (g.name, ops)


def test_unknown_and_unsupported_letters_are_rejected():
    g = gg.cycle(5)
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    for ops in ("i", "dai", "s", "x"):
        with pytest.raises(sbc.SbcError) as e:
            sbc.sbc_far_create(G.h, ops)
        assert e.value.status == -1  # SBC_E_INVALID_ARG
    G.close()
