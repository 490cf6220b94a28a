"""Autotuner host logic (no GPU): depth estimate, buckets, sampling sizes and
the JSON cache."""
import json

import numpy as np

import graphgen as gg
import paper_1209_6007_amd as sbc
from paper_1209_6007_amd import autotune as at


def test_bfs_depth_closed_forms():
    # from the highest-degree vertex (the first of equal degree)
    assert at.bfs_depth(gg.path(10).row_ptr, gg.path(10).col) == 8      # vertex 1 -> vertex 9
    assert at.bfs_depth(gg.star(30).row_ptr, gg.star(30).col) == 1
    assert at.bfs_depth(gg.complete(7).row_ptr, gg.complete(7).col) == 1
    g = gg.grid2d(6, 9)
    d = at.bfs_depth(g.row_ptr, g.col)
    assert 7 <= d <= 13                                                   # eccentricity of an interior vertex
    assert at.bfs_depth(np.array([0]), np.array([], np.int32)) == 0


def test_depth_separates_workload_shapes():
    rm = gg.rmat_decorated(scale=11, seed=3)
    gr = gg.grid_deleted(side=64, seed=3)
    assert at.bfs_depth(rm.row_ptr, rm.col) <= at.DEEP_LEVELS
    assert at.bfs_depth(gr.row_ptr, gr.col) > at.DEEP_LEVELS


def test_buckets():
    assert at.bucket_of(100, 5) == "s-shallow"
    assert at.bucket_of(4095, 40) == "s-deep"
    assert at.bucket_of(4096, 3) == "m-shallow"
    assert at.bucket_of(32767, 33) == "m-deep"
    assert at.bucket_of(32768, 32) == "l-shallow"


def test_candidates_set_every_tuned_key_and_sample_sizes():
    for c in at.CANDIDATES:
        assert sorted(c) == at.TUNED_KEYS
        s = at.sample_for(c, cus=256)
        want = (at.TEAM_ROUNDS * c["team_count"] if c["team_min_vertices"] > 0
                else at.BATCH_ROUNDS * 256 * (at.WAVES_PER_CU // c["batch_wg_waves"]))
        assert s == want


def test_small_stage_keys_are_tuned_keys():
    for c in at.SMALL_CANDIDATES:
        assert set(c) <= set(at.TUNED_KEYS)
    assert any(c["wave_max_vertices"] == 0 for c in at.SMALL_CANDIDATES)  # the kernel off is a choice


def test_deep_stage_keys_are_tuned_keys():
    for c in at.DEEP_CANDIDATES:
        assert set(c) <= set(at.TUNED_KEYS)
    # the first stage runs the library's default deep shape
    assert all(c["deep_wg_waves"] == 16 and c["deep_waves_per_eu"] == 0 for c in at.CANDIDATES)


def test_smallest_piece():
    g = gg.block_tree(n_pieces=30, max_size=200, seed=5)
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    G.preprocess("odai")
    sizes = np.diff(sbc.sbc_graph_export(G.h)["vtx_off"])
    assert at.smallest_piece(G, sbc.SBC_COMPRESSED, g.n) == int(sizes[sizes > 0].min())
    assert at.smallest_piece(G, sbc.SBC_PLAIN, g.n) == g.n


def test_total_items_matches_pieces():
    g = gg.rmat_decorated(scale=10, seed=4)
    G = sbc.Graph(g.n, g.row_ptr, g.col)
    G.preprocess("odai")
    sizes = np.diff(sbc.sbc_graph_export(G.h)["vtx_off"])
    assert at.total_items(G, sbc.SBC_COMPRESSED, g.n) == int(np.sum((sizes + 63) // 64))
    assert at.total_items(G, sbc.SBC_PLAIN, g.n) == (g.n + 63) // 64
    b, npmax, depth = at.workload_bucket(G, sbc.SBC_COMPRESSED)
    assert npmax == int(sizes.max()) and b == at.bucket_of(npmax, depth)


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "sub" / "autotune.json")
    assert at.load_cache(p) == {}
    d = {at.cache_key("dev", "l-shallow", sbc.SBC_COMPRESSED): {"params": at.CANDIDATES[4], "estimated_ms": 1.0}}
    at.save_cache(d, p)
    assert at.load_cache(p) == json.loads(json.dumps(d))
    assert at.cache_key("dev", "s-deep", sbc.SBC_PLAIN) == "dev|plain|s-deep"
