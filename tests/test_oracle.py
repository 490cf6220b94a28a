"""Pins of the CPU oracle against the paper and the mathematics (no GPU).

* brute force of Eq. (1) over every labelled graph on 6 vertices and random
  graphs up to 12 vertices (walk counting, no Brandes recursion);
* closed forms: the binary-tree formula of Section 3.1, its general-tree form,
  paths, stars, cycles, complete and complete bipartite graphs;
* invariants: the score sum equals the sum of (d(s,t)-1) over ordered pairs;
  degree-1 vertices score 0; identical vertices score the same (Section 3.1);
* Algorithm 2 with reach == 1 equals Algorithm 1 (Section 3.2.1);
* Algorithm 2 with reach and ident weights equals Algorithm 1 on the graph the
  attributed piece stands for (pendants for reach, twin copies for ident).
"""
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import brute
from tests.helpers import assert_bc_close, expand_attributed, expand_classes, tree_closed_form, twin_corrections

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def setup_module(_m):
    oracle.build(force=False)


def test_exhaustive_six_vertex_graphs():
    """All 2^15 labelled graphs on 6 vertices: Algorithm 1 == Eq. (1)."""
    n = 6
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    B = 1 << len(pairs)
    adj = np.zeros((B, n, n), dtype=np.int64)
    masks = np.arange(B)
    for b, (i, j) in enumerate(pairs):
        bit = (masks >> b) & 1
        adj[:, i, j] = bit
        adj[:, j, i] = bit
    want = brute.bc_bruteforce_batch(adj)
    worst = 0.0
    for g_idx in range(B):
        a = adj[g_idx]
        rp = np.zeros(n + 1, dtype=np.int32)
        rp[1:] = np.cumsum(a.sum(1))
        col = np.nonzero(a)[1].astype(np.int32)
        got = oracle.bc_plain(n, rp, col, threads=1)
        err = np.max(np.abs(got - want[g_idx]))
        worst = max(worst, err)
        assert err <= 1e-12, (g_idx, got, want[g_idx])
    assert worst <= 1e-12


@pytest.mark.parametrize("seed", range(40))
def test_random_small_graphs_vs_bruteforce(seed):
    r = gg.rng(seed)
    n = int(r.integers(2, 13))
    p = float(r.uniform(0.1, 0.7))
    g = gg.erdos_renyi(n, p, seed + 1000)
    want = brute.bc_bruteforce(g.n, g.row_ptr, g.col)
    got = oracle.bc(g, threads=2)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_decorated_small_graphs_vs_bruteforce():
    for seed in range(12):
        g = gg.decorated_random(6, 0.5, 2, 2, 1, seed)
        if g.n > 14:
            continue
        want = brute.bc_bruteforce(g.n, g.row_ptr, g.col)
        np.testing.assert_allclose(oracle.bc(g, threads=1), want, rtol=1e-12, atol=1e-12)


def test_binary_tree_formula_section_3_1():
    """Section 3.1: bc[v] = 2(l_v r_v + (n - l_v - r_v - 1)(l_v + r_v))."""
    for n in (1, 2, 3, 7, 10, 31, 100):
        g = gg.binary_tree(n)
        sub = np.ones(n, dtype=np.int64)
        for v in range(n - 1, 0, -1):
            sub[(v - 1) // 2] += sub[v]
        want = np.zeros(n)
        for v in range(n):
            lv = sub[2 * v + 1] if 2 * v + 1 < n else 0
            rv = sub[2 * v + 2] if 2 * v + 2 < n else 0
            want[v] = 2 * (lv * rv + (n - lv - rv - 1) * (lv + rv))
        np.testing.assert_array_equal(oracle.bc(g, threads=2), want)


@pytest.mark.parametrize("seed", range(8))
def test_random_trees_closed_form(seed):
    n = 50 + 37 * seed
    g = gg.random_tree(n, seed)
    np.testing.assert_array_equal(oracle.bc(g, threads=3), tree_closed_form(g))


def test_path_and_star_closed_forms():
    for n in (2, 3, 5, 17, 64):
        got = oracle.bc(gg.path(n))
        i = np.arange(n)
        np.testing.assert_array_equal(got, 2 * i * (n - 1 - i))      # unordered i(n-1-i)
        s = oracle.bc(gg.star(n))
        assert s[0] == (n - 1) * (n - 2)                              # unordered (n-1)(n-2)/2
        assert np.all(s[1:] == 0)


def test_cycle_complete_bipartite_closed_forms():
    for n in range(3, 26):
        got = oracle.bc(gg.cycle(n))
        want = (n - 1) * (n - 3) / 4 if n % 2 else (n - 2) ** 2 / 4   # ordered
        np.testing.assert_allclose(got, want, rtol=1e-13)
        np.testing.assert_array_equal(oracle.bc(gg.complete(n)), np.zeros(n))
    for a, b in [(1, 5), (2, 3), (3, 3), (4, 7), (5, 2)]:
        got = oracle.bc(gg.complete_bipartite(a, b))
        # ordered: side A gets b(b-1)/a, side B gets a(a-1)/b
        np.testing.assert_allclose(got[:a], b * (b - 1) / a, rtol=1e-13)
        np.testing.assert_allclose(got[a:], a * (a - 1) / b, rtol=1e-13)


def test_golden_fixtures():
    """Hand-derived values stored under tests/golden (each with its source)."""
    with open(os.path.join(GOLDEN, "closed_forms.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        n = c["n"]
        u = np.array([e[0] for e in c["edges"]], dtype=np.int64)
        v = np.array([e[1] for e in c["edges"]], dtype=np.int64)
        g = gg.csr_from_edges(n, u, v)
        want = np.array(c["bc_ordered"], dtype=np.float64)
        np.testing.assert_allclose(oracle.bc(g, threads=1), want, rtol=1e-13, atol=0, err_msg=c["name"])
        np.testing.assert_allclose(brute.bc_bruteforce(g.n, g.row_ptr, g.col), want, rtol=1e-13,
                                   err_msg=c["name"])


@pytest.mark.parametrize("seed", range(6))
def test_sum_invariant_and_structural_zeros(seed):
    """sum_v bc[v] = sum over ordered connected pairs of (d(s,t)-1); pendants
    score 0; open- and closed-neighbourhood twins score alike."""
    import scipy.sparse as sp
    import scipy.sparse.csgraph as cg

    g = gg.decorated_random(60 + 10 * seed, 0.06, 15, 8, 4, 500 + seed)
    bc = oracle.bc(g)
    a = sp.csr_matrix((np.ones(g.arcs), g.col, g.row_ptr), shape=(g.n, g.n))
    d = cg.shortest_path(a, unweighted=True, directed=False)
    fin = np.isfinite(d) & (d > 0)
    want = float(np.sum(d[fin] - 1))
    assert abs(bc.sum() - want) <= 1e-9 * want
    deg = g.degrees()
    assert np.all(bc[deg == 1] == 0)
    # neighbourhood signature -> equal scores
    sig_open, sig_closed = {}, {}
    for v in range(g.n):
        nb = tuple(sorted(g.col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()))
        sig_open.setdefault(nb, []).append(v)
        sig_closed.setdefault(tuple(sorted(nb + (v,))), []).append(v)
    for groups in (sig_open, sig_closed):
        for members in groups.values():
            if len(members) > 1:
                np.testing.assert_allclose(bc[members], bc[members[0]], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_weighted_reduces_to_plain(seed):
    """Section 3.2.1: Algorithm 2 with reach == 1 (and ident == 1) is Algorithm 1."""
    g = gg.erdos_renyi(80, 0.05, 900 + seed)
    ones = np.ones(g.n, dtype=np.int32)
    np.testing.assert_array_equal(oracle.bc_weighted(g.n, g.row_ptr, g.col, ones, ones), oracle.bc(g))
    np.testing.assert_array_equal(oracle.bc_weighted(g.n, g.row_ptr, g.col, None, None), oracle.bc(g))


@pytest.mark.parametrize("seed", range(30))
def test_weighted_equals_plain_on_expanded_graph(seed):
    """Algorithm 2 + ident rules on an attributed piece, plus the member terms
    the merged traversal cannot see, equals Algorithm 1 on the ordinary graph
    the piece stands for (Theorem 1 with Lemma 1 and Section 3.3.3)."""
    r = gg.rng(seed)
    n = int(r.integers(2, 10))
    g = gg.erdos_renyi(n, float(r.uniform(0.3, 0.9)), 4000 + seed)
    reach, ident = gg.random_attributes(n, 7000 + seed, rmax=3, kmax=3)
    if seed % 3 == 0:
        ident[:] = 1
    if seed % 5 == 1:
        reach[:] = 1
    twin_type = r.integers(1, 3, size=n)
    x, first = expand_attributed(n, g.row_ptr, g.col, reach, ident, twin_type)
    want_all = oracle.bc(x, threads=2)
    comp = gg.components(x)
    got_w = oracle.bc_weighted(n, g.row_ptr, g.col, reach, ident, threads=2)
    corr = twin_corrections(n, g.row_ptr, g.col, reach, ident, twin_type)
    for v in range(n):
        c = first[v]
        N = int(np.sum(comp == comp[c]))                  # size of v's component in the expansion
        pred = got_w[v] + corr[v] + (reach[v] - 1) * (N - 2)
        assert abs(pred - want_all[c]) <= 1e-9 * max(1.0, abs(want_all[c])), (v, pred, want_all[c])
    if x.n <= 12:
        np.testing.assert_allclose(want_all, brute.bc_bruteforce(x.n, x.row_ptr, x.col), rtol=1e-12, atol=1e-12)


def test_single_source_levels_and_counts():
    """Levels equal BFS distances; sigma equals the walk-count shortest-path numbers."""
    for seed in range(5):
        g = gg.erdos_renyi(11, 0.3, 300 + seed)
        dist, sigma = brute.distances_and_counts(brute.adjacency(g.n, g.row_ptr, g.col)[None])
        for s in range(g.n):
            d, sg, dl = oracle.single_source(g.n, g.row_ptr, g.col, s)
            np.testing.assert_array_equal(d, dist[0, s])
            np.testing.assert_array_equal(sg, sigma[0, s].astype(np.float64))
            # delta_s(v) = sum_t sigma_st(v)/sigma_st (Eq. (2)) from the brute-force tables
            for v in range(g.n):
                if v == s or d[v] < 0:
                    continue
                want = 0.0
                for t in range(g.n):
                    if t in (s, v) or dist[0, s, t] < 0:
                        continue
                    if dist[0, s, v] + dist[0, v, t] == dist[0, s, t]:
                        want += sigma[0, s, v] * sigma[0, v, t] / sigma[0, s, t]
                assert abs(dl[v] - want) <= 1e-12 * max(1, want)


def test_source_subset_is_additive():
    g = gg.erdos_renyi(60, 0.08, 77)
    full = oracle.bc(g)
    a = oracle.bc_plain(g.n, g.row_ptr, g.col, sources=np.arange(0, 30))
    b = oracle.bc_plain(g.n, g.row_ptr, g.col, sources=np.arange(30, 60))
    np.testing.assert_allclose(a + b, full, rtol=1e-12, atol=1e-12)


def test_bc_pieces_is_bc_weighted_per_piece():
    """oracle.bc_pieces on a packed set of ragged attributed pieces (one of a
    single vertex, one disconnected) equals oracle.bc_weighted run on each
    piece alone, for one thread and for more threads than pieces."""
    r = gg.rng(71)
    pieces = [gg.erdos_renyi(n, min(0.9, 5.0 / n), 300 + n) for n in (1, 2, 9, 40, 3, 77, 12)]
    pieces.append(gg.csr_from_edges(6, np.array([0, 1, 3]), np.array([1, 2, 4])))
    vtx_off, row, col, reach, ident, want = [0], [0], [], [], [], []
    for g in pieces:
        rc, kc = gg.random_attributes(g.n, int(r.integers(1 << 30)), rmax=4, kmax=3)
        want.append(oracle.bc_weighted(g.n, g.row_ptr, g.col, rc, kc, threads=1))
        base = row[-1]
        row.extend(int(base + x) for x in g.row_ptr[1:])
        col.extend(int(c) for c in g.col)
        reach.extend(rc)
        ident.extend(kc)
        vtx_off.append(vtx_off[-1] + g.n)
    want = np.concatenate(want)
    for threads in (1, 3, 40):
        got = oracle.bc_pieces(np.array(vtx_off), np.array(row), np.array(col), np.array(reach), np.array(ident),
                               threads=threads)
        np.testing.assert_allclose(got, want, rtol=1e-13, atol=0)


def test_device_path_golden_file_is_the_oracle():
    """tests/golden/device_path_bc.txt (read by the C consumer test) holds what
    its script computes with the oracle, and the script's graph has the shape
    the C program describes (63 vertices, 60 + 9 + 3 edges)."""
    import importlib.util

    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("mk", os.path.join(here, "make_device_path_golden.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    n, rp, col = mk.graph()
    assert n == 63 and rp[-1] == 2 * (60 + 9 + 3)
    with open(os.path.join(here, "device_path_bc.txt")) as f:
        lines = [l for l in f.read().split("\n") if l and not l.startswith("#")]
    assert int(lines[0]) == n
    stored = np.array([float(x) for x in lines[1:]])
    np.testing.assert_array_equal(stored, oracle.bc_plain(n, rp, col, threads=1))
    assert stored[60] == stored[61] == stored[62] == 0


def side_vertices(g):
    """Vertices of degree 1..4 whose neighbours are pairwise adjacent (side
    vertices, Section 2), in id order -- detected here independently of the
    library."""
    adj = [set(int(x) for x in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]) for v in range(g.n)]
    return [v for v in range(g.n)
            if 1 <= len(adj[v]) <= 4 and all(b in adj[a] for a in adj[v] for b in adj[v] if a < b)]


@pytest.mark.parametrize("seed", range(24))
def test_bc_side_restores_removed_side_vertices(seed):
    """Section 3.3.2: Algorithm 2 on a graph with reach equals Algorithm 2 on
    the graph with its side vertices removed one by one (in id order), plus
    oracle.bc_side's Algorithm 3 contributions, plus each removed vertex u's
    own term (reach[u]-1) x (reach of its component left after removing u).
    Random graphs with many triangles, pendant paths and cliques, random
    reach; pins bc_side against the pinned bc_weighted."""
    r = gg.rng(500 + seed)
    n = int(r.integers(6, 40))
    g0 = gg.erdos_renyi(n, float(r.uniform(0.05, 0.3)), 600 + seed)
    # the edge list, then triangles and a small clique hung off random vertices
    u0, v0 = g0.edges()
    us, vs = [int(x) for x in u0], [int(x) for x in v0]
    nxt = n
    for _ in range(int(r.integers(1, 6))):
        c = int(r.integers(0, n))
        us += [c, c, nxt]
        vs += [nxt, nxt + 1, nxt + 1]
        nxt += 2
    if seed % 3 == 0:  # a K4 hung on a vertex: every non-attachment vertex is a side vertex
        c = int(r.integers(0, n))
        k = [c, nxt, nxt + 1, nxt + 2]
        for a in range(4):
            for b in range(a + 1, 4):
                us.append(k[a])
                vs.append(k[b])
        nxt += 3
    g = gg.csr_from_edges(nxt, np.array(us, np.int64), np.array(vs, np.int64))
    reach = r.integers(1, 5, size=g.n).astype(np.int32)
    S = side_vertices(g)
    assert S, "no side vertex"
    want = oracle.bc_weighted(g.n, g.row_ptr, g.col, reach, None, threads=1)
    keep = np.ones(g.n, bool)
    keep[S] = False
    sub, idx = gg.induced_subgraph(g, keep)
    got = np.zeros(g.n)
    if sub.n:
        got[idx] = oracle.bc_weighted(sub.n, sub.row_ptr, sub.col, reach[idx], None, threads=1)
    got += oracle.bc_side(g.n, g.row_ptr, g.col, reach, np.array(S, np.int32), threads=2)
    comp = gg.components(g)
    left = {c: int(reach[comp == c].sum()) for c in np.unique(comp)}
    for u in S:
        left[comp[u]] -= int(reach[u])
        got[u] += (reach[u] - 1) * left[comp[u]]
    assert_bc_close(got, want, 1e-12, f"seed {seed}")


def test_bc_side_threads_agree():
    g = gg.decorated_random(30, 0.15, 6, 4, 5, 77)
    S = np.array(side_vertices(g), np.int32)
    reach = gg.rng(3).integers(1, 4, size=g.n).astype(np.int32)
    a = oracle.bc_side(g.n, g.row_ptr, g.col, reach, S, threads=1)
    b = oracle.bc_side(g.n, g.row_ptr, g.col, reach, S, threads=5)
    np.testing.assert_allclose(a, b, rtol=1e-14)


@pytest.mark.parametrize("seed", range(6))
def test_classes_with_equal_reach_are_the_weighted_form(seed):
    """bc_classes with reach sum k*r is bc_weighted with reach r, ident k."""
    g = gg.erdos_renyi(40, 0.12, 300 + seed)
    reach, ident = gg.random_attributes(g.n, 800 + seed, rmax=4, kmax=4)
    np.testing.assert_array_equal(oracle.bc_classes(g.n, g.row_ptr, g.col, reach * ident, ident),
                                  oracle.bc_weighted(g.n, g.row_ptr, g.col, reach, ident))


@pytest.mark.parametrize("seed", range(30))
def test_classes_of_unequal_reach_on_expanded_graph(seed):
    """A piece vertex standing for k identical vertices with reaches
    r_1..r_k: on the ordinary graph it stands for (copies, each with its
    pendant leaves), Algorithm 1 at copy c of class v (reach r_c, class sum R,
    N vertices in the component) is bc_classes[v] plus the pairs the merged
    traversal cannot see or sees at the mean reach R/k:
      (r_c - R/k)(N - R)      sources outside the class, targets below c
      (R - r_c)(r_c - 1)      class-mates' sides to the targets below c
      (r_c - 1)(N - 2)        c's own leaves as sources
      sum over open-twin neighbour classes u of (R_u^2 - sum r^2) / D_u
    (D_u: original neighbours of a member of u)."""
    r = gg.rng(seed + 60)
    n = int(r.integers(2, 9))
    g = gg.erdos_renyi(n, float(r.uniform(0.35, 0.9)), 5000 + seed)
    members = []
    for v in range(n):
        k = int(r.integers(1, 4)) if r.uniform() < 0.6 else 1
        if g.row_ptr[v + 1] == g.row_ptr[v]:
            k = 1  # identical vertices share a neighbour (they lie in one block)
        members.append([int(x) for x in r.integers(1, 5, size=k)])
    twin_type = r.integers(1, 3, size=n)
    x, off = expand_classes(n, g.row_ptr, g.col, members, twin_type)
    want = oracle.bc(x, threads=2)
    comp = gg.components(x)
    ident = np.array([len(m) for m in members], dtype=np.int32)
    rsum = np.array([sum(m) for m in members], dtype=np.int32)
    got = oracle.bc_classes(n, g.row_ptr, g.col, rsum, ident, threads=2)
    share = np.zeros(n)
    for u in range(n):
        if ident[u] >= 2 and twin_type[u] == 1:
            nb = g.col[g.row_ptr[u]:g.row_ptr[u + 1]]
            D = int(ident[nb].sum())
            if D > 0:
                share[nb] += (int(rsum[u]) ** 2 - sum(m * m for m in members[u])) / D
    for v in range(n):
        R, k = int(rsum[v]), int(ident[v])
        for j, c in enumerate(range(off[v], off[v + 1])):
            N = int(np.sum(comp == comp[c]))
            rc = members[v][j]
            pred = got[v] + (rc - R / k) * (N - R) + (R - rc) * (rc - 1) + (rc - 1) * (N - 2) + share[v]
            assert abs(pred - want[c]) <= 1e-9 * max(1.0, abs(want[c])), (v, j, pred, want[c])


@pytest.mark.parametrize("seed", range(8))
def test_brute_distance_sum_against_farness_and_scores(seed):
    """brute.distance_sum_ordered (matrix powers) equals the farness sum (one
    breadth-first search per vertex, in C) minus the ordered connected pairs,
    and the sum of Eq. (1) scores (every interior vertex of a shortest path
    counts once per pair)."""
    r = gg.rng(seed + 40)
    n = int(r.integers(2, 12))
    g = gg.erdos_renyi(n, float(r.uniform(0.1, 0.7)), 600 + seed)
    comp = gg.components(g)
    pairs = int(sum(c * (c - 1) for c in np.bincount(comp)))
    got = brute.distance_sum_ordered(g.n, g.row_ptr, g.col)
    assert got == int(oracle.farness(g.n, g.row_ptr, g.col).sum()) - pairs
    assert abs(got - float(brute.bc_bruteforce(g.n, g.row_ptr, g.col).sum())) <= 1e-9 * max(1, got)
