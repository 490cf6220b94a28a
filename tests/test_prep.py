"""Host preprocessing and the C interface, without a GPU.

The library's preprocessing (degree-1 stripping, biconnected shattering with
reach, identical-vertex merging) is exported piece by piece; the oracle's
Algorithm 2 with ident weights runs on every piece, and the Eq. (5) sum over
copies plus the exported host terms must equal the oracle's Algorithm 1 on the
original graph (Theorem 1 and its corollaries).
"""
import re
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_1209_6007_amd as sbc
from tests.helpers import assert_bc_close, map_back, member_reach

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OPS = ["", "d", "a", "i", "da", "di", "ai", "dai", "o", "odai", "s", "ds", "as", "si", "dasi", "odasi",
       "u", "du", "dau", "odau", "dasu"]


def setup_module(_m):
    oracle.build(force=False)
    sbc.lib()


def header_symbols():
    with open(os.path.join(ROOT, "include", "shatterbc.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sbc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = sbc.lib()
    syms = header_symbols()
    assert len(syms) >= 30
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(sbc.EXPORTED)


def test_no_device_means_error_not_fallback():
    """Without a GPU every compute entry point reports SBC_E_NO_DEVICE."""
    try:
        h = sbc.sbc_context_create(0)
    except sbc.SbcError as e:
        assert e.status == -12
        return
    sbc.sbc_context_destroy(h)
    pytest.skip("a GPU is visible")


def _gcreate(n, u, v):
    g = gg.csr_from_edges(n, np.array(u), np.array(v))
    return g


@pytest.mark.parametrize("case,status", [
    ("loop", -3), ("dup", -4), ("asym", -2), ("range", -5), ("rowptr", -1),
])
def test_validation_errors(case, status):
    rp = np.array([0, 1, 2], np.int32)
    col = np.array([1, 0], np.int32)
    n = 2
    if case == "loop":
        rp, col = np.array([0, 2, 3], np.int32), np.array([0, 1, 0], np.int32)
    elif case == "dup":
        rp, col = np.array([0, 2, 4], np.int32), np.array([1, 1, 0, 0], np.int32)
    elif case == "asym":
        rp, col = np.array([0, 1, 1], np.int32), np.array([1], np.int32)
    elif case == "range":
        col = np.array([5, 0], np.int32)
    elif case == "rowptr":
        rp = np.array([0, 2, 1], np.int32)
    with pytest.raises(sbc.SbcError) as ei:
        sbc.sbc_graph_create(n, rp, col)
    assert ei.value.status == status


def test_sanitize_repairs_input():
    rp = np.array([0, 3, 3, 4], np.int32)
    col = np.array([0, 2, 2, 1], np.int32)    # loop 0-0, duplicate 0->2, one-way 2->1
    h = sbc.sbc_graph_create(3, rp, col, sbc.SBC_SANITIZE)
    n, arcs = sbc.sbc_graph_info(h)
    assert (n, arcs) == (3, 4)                 # edges {0,2} and {1,2}
    sbc.sbc_graph_destroy(h)


def test_bad_ops_letter():
    g = gg.path(4)
    h = sbc.sbc_graph_create(g.n, g.row_ptr, g.col)
    with pytest.raises(sbc.SbcError):
        sbc.sbc_graph_preprocess(h, "dx")
    sbc.sbc_graph_destroy(h)


def compressed_via_oracle(g, ops, check_invariants=True):
    """Library preprocessing + oracle per piece + Eq. (5)."""
    h = sbc.sbc_graph_create(g.n, g.row_ptr, g.col)
    try:
        st = sbc.sbc_graph_preprocess(h, ops)
        ex = sbc.sbc_graph_export(h)
    finally:
        sbc.sbc_graph_destroy(h)
    V = ex["vtx_off"][-1]
    bcp = np.zeros(V)
    comp = gg.components(g) if check_invariants else None
    for p in range(len(ex["vtx_off"]) - 1):
        vb, ve = ex["vtx_off"][p], ex["vtx_off"][p + 1]
        np_ = ve - vb
        rp = (ex["row"][vb:ve + 1] - ex["row"][vb]).astype(np.int32)
        cl = ex["col"][ex["row"][vb]:ex["row"][ve]]
        assert np_ >= 3
        assert cl.min() >= 0 and cl.max() < np_
        k = int(ex["nside"][p])
        if k > 0:  # a side piece: Algorithm 3 for its side vertices 0..k-1, in that order
            assert "s" in ops and np.all(ex["ident"][vb:ve] == 1)
            bcp[vb:ve] = oracle.bc_side(np_, rp, cl, ex["reach"][vb:ve], np.arange(k, dtype=np.int32), threads=2)
        else:  # reach: the members' reach sum
            bcp[vb:ve] = oracle.bc_classes(np_, rp, cl, ex["reach"][vb:ve], ex["ident"][vb:ve], threads=2)
    out = ex["bcx"].copy()
    for v in range(g.n):
        for j in range(ex["map_off"][v], ex["map_off"][v + 1]):
            x = ex["map_idx"][j]
            out[v] += bcp[x] + ex["corr"][x]
    if check_invariants and len(ex["vtx_off"]) > 1 and "s" not in ops:
        # every piece represents its whole component: its reach sums = component size
        owner = {}
        for v in range(g.n):
            for j in range(ex["map_off"][v], ex["map_off"][v + 1]):
                owner[int(ex["map_idx"][j])] = v
        for p in range(len(ex["vtx_off"]) - 1):
            vb, ve = ex["vtx_off"][p], ex["vtx_off"][p + 1]
            tot = int(np.sum(ex["reach"][vb:ve].astype(np.int64)))
            some = owner[int(vb)]
            assert tot == int(np.sum(comp == comp[some])), (p, tot)
    return out, st


@pytest.mark.parametrize("ops", OPS)
def test_exhaustive_six_vertex_graphs_every_ops(ops):
    """Every labelled graph on 6 vertices (sampled 1 in 4 for the full sweep)."""
    pairs = [(i, j) for i in range(6) for j in range(i + 1, 6)]
    step = 1 if ops in ("dai", "dasi", "dau") else 4
    for mask in range(0, 1 << 15, step):
        es = [pairs[b] for b in range(15) if (mask >> b) & 1]
        u = np.array([e[0] for e in es], dtype=np.int64)
        v = np.array([e[1] for e in es], dtype=np.int64)
        g = gg.csr_from_edges(6, u, v)
        want = oracle.bc(g, threads=1)
        got, _ = compressed_via_oracle(g, ops, check_invariants=False)
        assert_bc_close(got, want, 1e-12, f"mask={mask} ops={ops}")


@pytest.mark.parametrize("seed", range(25))
def test_decorated_graphs_every_ops(seed):
    r = gg.rng(seed)
    g = gg.decorated_random(int(r.integers(8, 40)), float(r.uniform(0.05, 0.4)), int(r.integers(0, 12)),
                            int(r.integers(0, 10)), int(r.integers(0, 6)), 100 + seed)
    want = oracle.bc(g)
    for ops in OPS:
        got, _ = compressed_via_oracle(g, ops)
        assert_bc_close(got, want, 1e-10, f"seed={seed} ops={ops}")


def test_worked_examples_twins_with_reach():
    """K_{2,3} with pendants (open twins carrying reach) and a triangle with
    pendants (closed twins carrying reach): values derived pair by pair."""
    g = gg.csr_from_edges(7, np.array([0, 0, 0, 1, 1, 1, 0, 1]), np.array([2, 3, 4, 2, 3, 4, 5, 6]))
    got, st = compressed_via_oracle(g, "dai")
    np.testing.assert_allclose(got, [13, 13, 8 / 3, 8 / 3, 8 / 3, 0, 0], rtol=1e-12)
    assert st["stripped"] == 2 and st["twin_classes"] == 2
    g = gg.csr_from_edges(6, np.array([0, 1, 0, 0, 1, 2]), np.array([1, 2, 2, 3, 4, 5]))
    got, st = compressed_via_oracle(g, "dai")
    np.testing.assert_allclose(got, [8, 8, 8, 0, 0, 0], rtol=1e-12)
    assert st["pieces"] == 0                    # the triangle collapses to one class


def test_side_vertices_removed_with_algorithm3():
    """Side vertices (Section 3.3.2): a block with triangles and a K4 hung on
    it; 's' removes the side vertices, exports one side piece per block that
    had them (its side vertices first), and the result is exact."""
    # a 6-cycle 0..5 with chords 0-2 and 3-5 (vertices 1 and 4 become side
    # vertices of degree 2), a triangle 0-6-7 and a K4 {3, 8, 9, 10}
    u = [0, 1, 2, 3, 4, 5, 0, 3, 0, 0, 6, 3, 3, 3, 8, 8, 9]
    v = [1, 2, 3, 4, 5, 0, 2, 5, 6, 7, 7, 8, 9, 10, 9, 10, 10]
    g = gg.csr_from_edges(11, np.array(u), np.array(v))
    for ops in ("s", "as", "das", "dasi", "odasi"):
        got, st = compressed_via_oracle(g, ops)
        assert st["side_vertices"] > 0 and st["side_pieces"] > 0, (ops, st)
        assert_bc_close(got, oracle.bc(g), 1e-12, ops)


@pytest.mark.parametrize("name", ["ba", "blocks", "grid", "rmat", "trees"])
def test_workload_shapes_small(name):
    if name == "ba":
        g = gg.ba_pendant_triangles()
    elif name == "blocks":
        g = gg.block_tree(n_pieces=60, max_size=200, seed=5)
    elif name == "grid":
        g = gg.grid_deleted(side=24, seed=6)
    elif name == "rmat":
        g = gg.rmat_decorated(scale=9, seed=7)
    else:
        g = gg.random_tree(300, 8)
    want = oracle.bc(g)
    for ops in ("d", "da", "dai", "ai", "odai", "odasi", "s", "odau", "dasu"):
        got, st = compressed_via_oracle(g, ops)
        assert_bc_close(got, want, 1e-9, f"{name} ops={ops}")


def test_unequal_reach_twins_merge_more():
    """'u' merges the identical vertices that stripping left with different
    reach, which 'i' keeps apart: fewer piece vertices, the same result."""
    g = gg.rmat_decorated(scale=10, seed=12)
    want = oracle.bc(g)
    got_i, st_i = compressed_via_oracle(g, "odai")
    got_u, st_u = compressed_via_oracle(g, "odau")
    assert st_u["twins_merged"] > st_i["twins_merged"] and st_u["piece_vertices"] < st_i["piece_vertices"]
    assert_bc_close(got_u, want, 1e-9, "odau")
    assert_bc_close(got_i, want, 1e-9, "odai")


def test_worked_example_twins_of_unequal_reach():
    """C4 a-x-b-y with two pendants p, q on x: after stripping, x and y are
    open twins of reach 3 and 1, merged by 'u' only.  Pair by pair (ordered):
    x = 15 (p and q to each other and to a, b, y, both ways: 14; half of
    a<->b: 1), y = 1 (the other half), a = b = 3 (half of the pairs between
    y and x, p, q, both ways)."""
    # a=0, x=1, b=2, y=3, pendants 4, 5 on x
    g = gg.csr_from_edges(6, np.array([0, 1, 2, 3, 1, 1]), np.array([1, 2, 3, 0, 4, 5]))
    want = oracle.bc(g)
    got_u, st_u = compressed_via_oracle(g, "dau")
    got_i, st_i = compressed_via_oracle(g, "dai")
    assert st_u["twin_classes"] >= 1 and st_i["twin_classes"] < st_u["twin_classes"]
    np.testing.assert_array_equal(want, [3, 15, 3, 1, 0, 0])
    assert_bc_close(got_u, want, 1e-12, "dau")


@pytest.mark.parametrize("name", ["blocks", "rmat"])
def test_bc_pieces_mapped_back_is_the_oracle(name):
    """The check the full-size block tree uses on the GPU: the oracle's
    bc' of every exported piece (oracle.bc_pieces), mapped back with Eq. (5),
    equals Algorithm 1 on the original graph (Theorem 1)."""
    g = gg.block_tree(n_pieces=80, max_size=300, seed=15) if name == "blocks" else gg.rmat_decorated(scale=9, seed=8)
    h = sbc.sbc_graph_create(g.n, g.row_ptr, g.col)
    try:
        sbc.sbc_graph_preprocess(h, "odai")
        ex = sbc.sbc_graph_export(h)
    finally:
        sbc.sbc_graph_destroy(h)
    bcp = oracle.bc_pieces(ex["vtx_off"], ex["row"], ex["col"], member_reach(ex), ex["ident"], threads=4)
    assert_bc_close(map_back(ex, bcp), oracle.bc(g), 1e-9, name)


def test_block_tree_shatters_into_its_blocks():
    sizes = np.array([8, 20, 50, 9, 33])
    g = gg.block_tree(n_pieces=5, sizes=sizes, seed=11)
    h = sbc.sbc_graph_create(g.n, g.row_ptr, g.col)
    st = sbc.sbc_graph_preprocess(h, "a")
    sbc.sbc_graph_destroy(h)
    assert st["blocks"] == 5 and st["pieces"] == 5
    assert st["piece_vertices"] == int(sizes.sum())
