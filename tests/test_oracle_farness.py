"""Pins of the oracle's farness (sum of shortest-path distances, the quantity
behind closeness centrality) against the mathematics, no GPU:

* closed forms: paths, cycles, stars, complete and complete bipartite graphs,
  and grids (distances add over the two axes);
* all-pairs distances by Floyd-Warshall (min-plus relaxation, no search) on
  random graphs, weighted and unweighted, connected or not;
* invariants: the farness sum is twice the Wiener index, which on a tree is
  the sum over edges of 2 s (n - s), s the size of one side;
* the packed-pieces form equals the one-graph form piece by piece.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle


def setup_module(_m):
    oracle.build(force=False)


def far(g, weight=None):
    return oracle.farness(g.n, g.row_ptr, g.col, weight)


def floyd_warshall(g):
    """All-pairs hop distances by min-plus relaxation; inf where unreachable."""
    n = g.n
    D = np.full((n, n), np.inf)
    np.fill_diagonal(D, 0.0)
    for v in range(n):
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            D[v, g.col[e]] = 1.0
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return D


def brute_farness(g, weight=None):
    D = floyd_warshall(g)
    w = np.ones(g.n) if weight is None else np.asarray(weight, dtype=np.float64)
    fin = np.isfinite(D)
    return np.array([int(round(float(np.sum(np.where(fin[x], D[x] * w, 0.0))))) for x in range(g.n)], dtype=np.int64)


def path_farness(n):
    i = np.arange(n, dtype=np.int64)
    return i * (i + 1) // 2 + (n - 1 - i) * (n - i) // 2


def test_path_cycle_star_closed_forms():
    for n in (1, 2, 3, 7, 50):
        assert np.array_equal(far(gg.path(n)), path_farness(n)), n
    for n in (3, 4, 9, 10, 31, 64):
        want = n * n // 4 if n % 2 == 0 else (n * n - 1) // 4
        assert np.all(far(gg.cycle(n)) == want), n
    for k in (1, 2, 5, 40):
        got = far(gg.star(k + 1))
        # the generator's centre is vertex 0
        assert got[0] == k and np.all(got[1:] == 1 + 2 * (k - 1)), (k, got)


def test_complete_and_bipartite_closed_forms():
    for n in (2, 3, 8, 33):
        assert np.all(far(gg.complete(n)) == n - 1)
    for a, b in ((1, 1), (2, 3), (4, 4), (3, 9)):
        got = far(gg.complete_bipartite(a, b))
        assert np.all(got[:a] == b + 2 * (a - 1)) and np.all(got[a:] == a + 2 * (b - 1)), (a, b, got)


def test_grid_distances_add_over_axes():
    for rows, cols in ((1, 5), (3, 4), (8, 8), (5, 17)):
        got = far(gg.grid2d(rows, cols))
        fr, fc = path_farness(rows), path_farness(cols)
        want = (fr[:, None] * cols + fc[None, :] * rows).reshape(-1)  # id = r * cols + c
        assert np.array_equal(got, want), (rows, cols)


@pytest.mark.parametrize("seed", range(25))
def test_random_graphs_vs_floyd_warshall(seed):
    r = gg.rng(seed + 500)
    n = int(r.integers(1, 14))
    g = gg.erdos_renyi(n, float(r.uniform(0.05, 0.6)), seed)
    assert np.array_equal(far(g), brute_farness(g))
    w = r.integers(1, 9, size=n).astype(np.int32)
    assert np.array_equal(far(g, w), brute_farness(g, w))


def test_wiener_index_on_trees_and_sum_invariant():
    for seed in range(6):
        t = gg.random_tree(int(gg.rng(seed).integers(2, 60)), seed)
        # side sizes of each edge by removing it
        total = 0
        for v in range(t.n):
            for e in range(t.row_ptr[v], t.row_ptr[v + 1]):
                w = int(t.col[e])
                if v < w:
                    seen = {w}
                    stack = [w]
                    while stack:
                        x = stack.pop()
                        for f in range(t.row_ptr[x], t.row_ptr[x + 1]):
                            y = int(t.col[f])
                            if y not in seen and not (x == w and y == v):
                                seen.add(y)
                                stack.append(y)
                    s = len(seen)
                    total += 2 * s * (t.n - s)
        assert int(far(t).sum()) == total, seed
    g = gg.erdos_renyi(40, 0.08, 3)
    D = floyd_warshall(g)
    assert int(far(g).sum()) == int(np.sum(D[np.isfinite(D)]))


def test_pieces_form_is_per_piece():
    gs = [gg.erdos_renyi(30, 0.1, 1), gg.cycle(9), gg.path(1), gg.grid2d(4, 6)]
    vtx_off, row, col, wts = [0], [0], [], []
    r = gg.rng(77)
    for g in gs:
        vtx_off.append(vtx_off[-1] + g.n)
        base = row[-1]
        row.extend((base + g.row_ptr[1:]).tolist())
        col.extend(g.col.tolist())
        wts.append(r.integers(1, 5, size=g.n).astype(np.int32))
    got = oracle.farness_pieces(np.array(vtx_off), np.array(row), np.array(col, np.int32), np.concatenate(wts))
    for p, g in enumerate(gs):
        assert np.array_equal(got[vtx_off[p]:vtx_off[p + 1]], far(g, wts[p])), p


def test_threads_agree():
    g = gg.erdos_renyi(300, 0.02, 4)
    a = oracle.farness(g.n, g.row_ptr, g.col, threads=1)
    b = oracle.farness(g.n, g.row_ptr, g.col, threads=7)
    assert np.array_equal(a, b)


def test_source_subset_is_the_same_searches():
    g = gg.erdos_renyi(200, 0.02, 9)
    w = gg.rng(3).integers(1, 6, size=g.n).astype(np.int32)
    src = np.array([5, 0, 199, 5, 77], np.int32)
    assert np.array_equal(oracle.farness(g.n, g.row_ptr, g.col, w, sources=src),
                          brute_farness(g, w)[src])
