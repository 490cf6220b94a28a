"""Seeded synthetic graph generators.

This module builds inputs only: undirected, unweighted, loop-free graphs in
symmetric CSR form (both arc directions present, rows sorted, int32), plus
random vertex attributes for attributed-piece tests.  It contains none of the
betweenness arithmetic, so both the oracle tests and the GPU path may use it.

Every generator takes an explicit integer seed and uses numpy's PCG64, so a
(generator, seed) pair always yields the same graph.  The workload shapes stand
in for the paper's test networks (Section 4: social, structural, road-like and
redistricting graphs), which are not available here.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 12096007


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


@dataclass
class Graph:
    """Symmetric CSR graph: row_ptr int32[n+1], col int32[row_ptr[n]]."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    name: str = ""

    @property
    def arcs(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        """Number of undirected edges."""
        return self.arcs // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def edges(self) -> tuple[np.ndarray, np.ndarray]:
        """Each undirected edge once, as (u < v) arrays."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees())
        dst = self.col.astype(np.int64)
        keep = src < dst
        return src[keep], dst[keep]


def csr_from_edges(n: int, u, v, name: str = "") -> Graph:
    """Symmetrise an edge list, drop self loops and duplicate edges, sort rows."""
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    if u.size:
        if u.min() < 0 or v.min() < 0 or max(u.max(), v.max()) >= n:
            raise ValueError("edge endpoint out of range")
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.concatenate([u, v])
    b = np.concatenate([v, u])
    key = np.unique(a * n + b)
    a = key // n
    b = key % n
    counts = np.bincount(a, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("too many arcs for int32 CSR")
    return Graph(n, row_ptr.astype(np.int32), b.astype(np.int32), name)


def relabel(g: Graph, perm: np.ndarray, name: str | None = None) -> Graph:
    """Return the graph with vertex v renamed perm[v]."""
    perm = np.asarray(perm, dtype=np.int64)
    u, v = g.edges()
    return csr_from_edges(g.n, perm[u], perm[v], g.name if name is None else name)


def induced_subgraph(g: Graph, keep_mask: np.ndarray, name: str = "") -> tuple[Graph, np.ndarray]:
    """Subgraph induced by keep_mask, relabelled in increasing original id.

    Returns (graph, old_ids) where old_ids[new] = old id.
    """
    old_ids = np.flatnonzero(keep_mask)
    new_id = np.full(g.n, -1, dtype=np.int64)
    new_id[old_ids] = np.arange(old_ids.size)
    u, v = g.edges()
    ok = keep_mask[u] & keep_mask[v]
    return csr_from_edges(old_ids.size, new_id[u[ok]], new_id[v[ok]], name), old_ids


def components(g: Graph) -> np.ndarray:
    """Connected-component label per vertex (scipy union-find on the CSR)."""
    import scipy.sparse as sp
    import scipy.sparse.csgraph as cg

    a = sp.csr_matrix(
        (np.ones(g.arcs, dtype=np.int8), g.col.astype(np.int64), g.row_ptr.astype(np.int64)),
        shape=(g.n, g.n),
    )
    _, lab = cg.connected_components(a, directed=False)
    return lab


# ---------------------------------------------------------------------------
# Small named graphs (closed-form test cases)
# ---------------------------------------------------------------------------

def path(n: int) -> Graph:
    i = np.arange(n - 1)
    return csr_from_edges(n, i, i + 1, f"path{n}")


def star(n: int) -> Graph:
    """Centre 0 with n-1 leaves."""
    i = np.arange(1, n)
    return csr_from_edges(n, np.zeros_like(i), i, f"star{n}")


def cycle(n: int) -> Graph:
    i = np.arange(n)
    return csr_from_edges(n, i, (i + 1) % n, f"cycle{n}")


def complete(n: int) -> Graph:
    u, v = np.triu_indices(n, 1)
    return csr_from_edges(n, u, v, f"K{n}")


def complete_bipartite(a: int, b: int) -> Graph:
    """Side A = 0..a-1, side B = a..a+b-1."""
    u, v = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return csr_from_edges(a + b, u.ravel(), v.ravel(), f"K{a},{b}")


def grid2d(rows: int, cols: int) -> Graph:
    idx = np.arange(rows * cols).reshape(rows, cols)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return csr_from_edges(rows * cols, u, v, f"grid{rows}x{cols}")


def random_tree(n: int, seed: int) -> Graph:
    """Uniform random recursive tree: vertex i>0 attaches to a uniform j<i."""
    r = rng(seed)
    if n <= 1:
        return csr_from_edges(n, [], [], f"tree{n}")
    i = np.arange(1, n)
    parent = np.floor(r.random(n - 1) * i).astype(np.int64)
    return csr_from_edges(n, i, parent, f"tree{n}")


def binary_tree(n: int) -> Graph:
    """Complete-ish binary tree in heap order: parent of i is (i-1)//2."""
    i = np.arange(1, n)
    return csr_from_edges(n, i, (i - 1) // 2, f"bintree{n}")


def erdos_renyi(n: int, p: float, seed: int) -> Graph:
    r = rng(seed)
    u, v = np.triu_indices(n, 1)
    keep = r.random(u.size) < p
    return csr_from_edges(n, u[keep], v[keep], f"er{n}")


def all_graphs(n: int):
    """Every labelled simple graph on n vertices (2^(n(n-1)/2) of them)."""
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        es = [pairs[i] for i in range(len(pairs)) if (mask >> i) & 1]
        if es:
            u, v = zip(*es)
        else:
            u, v = (), ()
        yield csr_from_edges(n, np.array(u, dtype=np.int64), np.array(v, dtype=np.int64), f"g{n}_{mask}")


def decorated_random(n_core: int, p: float, n_pendants: int, n_twins: int, n_triangles: int, seed: int) -> Graph:
    """Small random graph planted with pendants, twins and hung triangles.

    Used to exercise every preprocessing operation on graphs small enough for
    the oracle to finish in milliseconds.
    """
    r = rng(seed)
    g = erdos_renyi(n_core, p, int(r.integers(1 << 62)))
    us, vs = [list(x) for x in g.edges()]
    adj = [set() for _ in range(n_core)]
    for a, b in zip(us, vs):
        adj[a].add(b)
        adj[b].add(a)
    n = n_core
    for _ in range(n_twins):
        src = int(r.integers(0, n))
        nbrs = sorted(adj[src]) if src < len(adj) else []
        adj.append(set())
        for w in nbrs:
            us.append(n)
            vs.append(w)
            adj[n].add(w)
            adj[w].add(n)
        if r.random() < 0.5 and nbrs:
            # closed-neighbourhood twin: also adjacent to the copied vertex
            us.append(n)
            vs.append(src)
            adj[n].add(src)
            adj[src].add(n)
        n += 1
    for _ in range(n_triangles):
        c = int(r.integers(0, n))
        x, y = n, n + 1
        us += [c, c, x]
        vs += [x, y, y]
        adj.append({c, y})
        adj.append({c, x})
        adj[c].update((x, y))
        n += 2
    for _ in range(n_pendants):
        c = int(r.integers(0, n))
        us.append(c)
        vs.append(n)
        adj.append({c})
        adj[c].add(n)
        n += 1
    return csr_from_edges(n, np.array(us, dtype=np.int64), np.array(vs, dtype=np.int64), f"decorated{n}")


def random_attributes(n: int, seed: int, rmax: int = 4, kmax: int = 3) -> tuple[np.ndarray, np.ndarray]:
    """Random (reach, ident) vertex weights, each >= 1, for attributed-piece tests."""
    r = rng(seed)
    reach = r.integers(1, rmax + 1, size=n).astype(np.int32)
    ident = r.integers(1, kmax + 1, size=n).astype(np.int32)
    return reach, ident


# ---------------------------------------------------------------------------
# Workload generators
# ---------------------------------------------------------------------------

def ba_pendant_triangles(seed: int = SEED_BASE + 1, n_core: int = 1500, m_attach: int = 2,
                         n_pendants: int = 400, n_triangles: int = 100) -> Graph:
    """Barabasi-Albert core with pendants and hung triangles.

    Core: seed triangle on 0,1,2, then vertices 3..n_core-1 each attach m_attach
    edges to distinct earlier vertices chosen with probability proportional to
    degree.  Then n_pendants degree-1 vertices on uniform core vertices, then
    n_triangles triangles {c,x,y} hung on uniform core vertices c.  Ids: core,
    then pendants, then triangle pairs.
    """
    r = rng(seed)
    us = [0, 1, 0]
    vs = [1, 2, 2]
    ends = [0, 1, 1, 2, 0, 2]  # each vertex listed once per incident edge
    for v in range(3, n_core):
        chosen: set[int] = set()
        while len(chosen) < m_attach:
            chosen.add(ends[int(r.integers(0, len(ends)))])
        for t in sorted(chosen):
            us.append(v)
            vs.append(t)
            ends += [v, t]
    n = n_core
    core_pick = r.integers(0, n_core, size=n_pendants)
    for c in core_pick:
        us.append(int(c))
        vs.append(n)
        n += 1
    tri_pick = r.integers(0, n_core, size=n_triangles)
    for c in tri_pick:
        x, y = n, n + 1
        us += [int(c), int(c), x]
        vs += [x, y, y]
        n += 2
    return csr_from_edges(n, np.array(us), np.array(vs), "ba1500+pendants+triangles")


def rmat_edges(scale: int, edge_factor: int, abcd, r: np.random.Generator) -> tuple[np.ndarray, np.ndarray]:
    """R-MAT edge list: each edge descends `scale` quadrant choices."""
    a, b, c, _ = abcd
    ne = (1 << scale) * edge_factor
    src = np.zeros(ne, dtype=np.int64)
    dst = np.zeros(ne, dtype=np.int64)
    for bit in range(scale):
        x = r.random(ne)
        right = (x >= a) & (x < a + b) | (x >= a + b + c)
        down = x >= a + b
        src |= down.astype(np.int64) << bit
        dst |= right.astype(np.int64) << bit
    return src, dst


def rmat_decorated(scale: int = 17, edge_factor: int = 8, abcd=(0.57, 0.19, 0.19, 0.05),
                   twin_frac: float = 0.05, pendant_frac: float = 0.25,
                   seed: int = SEED_BASE + 2) -> Graph:
    """R-MAT graph with planted twins and pendants (social-network stand-in).

    R-MAT edges with a seeded label permutation, symmetrised, loops and
    duplicates removed.  Then twin_frac*2^scale new vertices, each copying the
    neighbour list of a uniform R-MAT vertex of degree >= 2; then
    pendant_frac*2^scale new degree-1 vertices on uniform vertices of degree >= 1.
    """
    r = rng(seed)
    nv = 1 << scale
    s, d = rmat_edges(scale, edge_factor, abcd, r)
    perm = r.permutation(nv)
    base = csr_from_edges(nv, perm[s], perm[d])
    deg = base.degrees()
    n_tw = int(round(twin_frac * nv))
    cand = np.flatnonzero(deg >= 2)
    pick = cand[r.integers(0, cand.size, size=n_tw)]
    us = [base.edges()[0]]
    vs = [base.edges()[1]]
    for i, src_v in enumerate(pick):
        nb = base.col[base.row_ptr[src_v]:base.row_ptr[src_v + 1]].astype(np.int64)
        us.append(np.full(nb.size, nv + i, dtype=np.int64))
        vs.append(nb)
    n = nv + n_tw
    u_all = np.concatenate(us)
    v_all = np.concatenate(vs)
    deg2 = np.bincount(np.concatenate([u_all, v_all]), minlength=n)
    n_pd = int(round(pendant_frac * nv))
    cand = np.flatnonzero(deg2 >= 1)
    att = cand[r.integers(0, cand.size, size=n_pd)]
    u_all = np.concatenate([u_all, att])
    v_all = np.concatenate([v_all, np.arange(n, n + n_pd, dtype=np.int64)])
    n += n_pd
    return csr_from_edges(n, u_all, v_all, f"rmat{scale}+twins+pendants")


def block_tree_sizes(n_pieces: int, r: np.random.Generator, min_size: int = 8, max_size: int = 4096) -> np.ndarray:
    x = r.uniform(math.log(min_size), math.log(max_size), size=n_pieces)
    return np.rint(np.exp(x)).astype(np.int64)


def block_tree(n_pieces: int = 20000, min_size: int = 8, max_size: int = 4096, avg_degree: int = 6,
               seed: int = SEED_BASE + 3, sizes: np.ndarray | None = None) -> Graph:
    """Tree of 2-connected random blocks glued at shared vertices.

    Block i has n_i vertices (log-uniform in [min_size, max_size]): a
    Hamiltonian cycle on a random permutation plus uniform extra edges until it
    has avg_degree*n_i/2 edges.  Block i >= 1 shares one uniform vertex with a
    uniform vertex of a uniform earlier block j < i, so the shared vertices are
    articulation points and the blocks are the biconnected components.
    """
    r = rng(seed)
    if sizes is None:
        sizes = block_tree_sizes(n_pieces, r, min_size, max_size)
    sizes = np.asarray(sizes, dtype=np.int64)
    P = sizes.size
    off = np.zeros(P + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    N = int(off[-1])
    # Hamiltonian cycles.
    piece_of = np.repeat(np.arange(P), sizes)
    perm_local = np.empty(N, dtype=np.int64)
    keys = r.random(N)
    order = np.lexsort((keys, piece_of))          # random order inside each piece
    perm_local[:] = order
    nxt = np.empty(N, dtype=np.int64)
    pos = np.arange(N)
    start = off[piece_of]
    nxt_pos = np.where(pos + 1 < off[piece_of + 1], pos + 1, start)
    nxt[:] = perm_local[nxt_pos]
    cu = perm_local
    cv = nxt
    target = (avg_degree * sizes) // 2
    need = np.maximum(target - sizes, 0)
    maxe = sizes * (sizes - 1) // 2
    need = np.minimum(need, maxe - sizes)
    # Extra edges: rejection sampling, all pieces at once.
    lo = np.minimum(cu, cv)
    hi = np.maximum(cu, cv)
    existing = lo * N + hi
    have = np.zeros(P, dtype=np.int64)
    chosen_keys = []
    existing_set = np.unique(existing)
    while True:
        short = np.flatnonzero(have < need)
        if short.size == 0:
            break
        reps = (need[short] - have[short]) * 2 + 4
        pc = np.repeat(short, reps)
        a = off[pc] + np.floor(r.random(pc.size) * sizes[pc]).astype(np.int64)
        b = off[pc] + np.floor(r.random(pc.size) * sizes[pc]).astype(np.int64)
        ok = a != b
        pc, a, b = pc[ok], a[ok], b[ok]
        k = np.minimum(a, b) * N + np.maximum(a, b)
        k_u, first = np.unique(k, return_index=True)
        sel = np.sort(first)                       # keep draw order
        k, pc = k[sel], pc[sel]
        fresh = ~np.isin(k, existing_set)
        k, pc = k[fresh], pc[fresh]
        # take at most need-have per piece, in draw order
        order = np.argsort(pc, kind="stable")
        k, pc = k[order], pc[order]
        rank = np.arange(pc.size) - np.searchsorted(pc, pc, side="left")
        take = rank < (need[pc] - have[pc])
        k, pc = k[take], pc[take]
        have += np.bincount(pc, minlength=P)
        chosen_keys.append(k)
        existing_set = np.union1d(existing_set, k)
    if chosen_keys:
        ek = np.concatenate(chosen_keys)
        eu = np.concatenate([cu, ek // N])
        ev = np.concatenate([cv, ek % N])
    else:
        eu, ev = cu, cv
    # Glue piece i>=1 to an earlier piece: identify vertex x_i of piece i with y_i of piece j<i.
    rep = np.arange(N, dtype=np.int64)
    if P > 1:
        i = np.arange(1, P)
        j = np.floor(r.random(P - 1) * i).astype(np.int64)
        xi = off[i] + np.floor(r.random(P - 1) * sizes[i]).astype(np.int64)
        yj = off[j] + np.floor(r.random(P - 1) * sizes[j]).astype(np.int64)
        # resolve in order so chains of identifications collapse to the earliest piece
        rep[xi] = yj
        for _ in range(64):
            nr = rep[rep]
            if np.array_equal(nr, rep):
                break
            rep = nr
        else:  # pragma: no cover - chains are short in practice
            while True:
                nr = rep[rep]
                if np.array_equal(nr, rep):
                    break
                rep = nr
    eu = rep[eu]
    ev = rep[ev]
    alive = np.zeros(N, dtype=bool)
    alive[rep] = True
    new_id = np.cumsum(alive) - 1
    n = int(alive.sum())
    return csr_from_edges(n, new_id[eu], new_id[ev], f"blocktree{P}")


def grid_deleted(side: int = 512, delete_frac: float = 0.12, seed: int = SEED_BASE + 4) -> Graph:
    """Road-like stand-in: side x side grid, a seeded fraction of edges deleted,
    largest connected component kept and relabelled in row-major order."""
    r = rng(seed)
    g = grid2d(side, side)
    u, v = g.edges()
    ne = u.size
    n_del = int(round(delete_frac * ne))
    order = r.permutation(ne)
    keep = np.ones(ne, dtype=bool)
    keep[order[:n_del]] = False
    h = csr_from_edges(g.n, u[keep], v[keep])
    lab = components(h)
    big = np.argmax(np.bincount(lab))
    sub, _ = induced_subgraph(h, lab == big, f"grid{side}-del{delete_frac}")
    return sub


@dataclass
class Request:
    idx: int
    arrival_s: float
    kind: str
    size: int
    seed: int


def serving_stream(n_requests: int = 600, rate_per_s: float = 20.0, seed: int = SEED_BASE + 5,
                   rmat_scales=(10, 15), grid_sides=(32, 256)) -> list[Request]:
    """Poisson arrivals of BC jobs: each is an R-MAT (scale uniform in range,
    same decorations as the scale-17 workload) or a deleted-edge grid (side
    uniform in range), by a fair coin."""
    r = rng(seed)
    gaps = r.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n_requests):
        if r.random() < 0.5:
            out.append(Request(i, float(t[i]), "rmat", int(r.integers(rmat_scales[0], rmat_scales[1] + 1)),
                               SEED_BASE * 1000 + i))
        else:
            out.append(Request(i, float(t[i]), "grid", int(r.integers(grid_sides[0], grid_sides[1] + 1)),
                               SEED_BASE * 1000 + i))
    return out


def request_graph(req: Request) -> Graph:
    if req.kind == "rmat":
        return rmat_decorated(scale=req.size, seed=req.seed)
    return grid_deleted(side=req.size, seed=req.seed)


WORKLOADS = {
    "ba1500": lambda: ba_pendant_triangles(),
    "rmat17": lambda: rmat_decorated(),
    "blocktree20000": lambda: block_tree(),
    # the block tree's recipe with pieces of 8..256 vertices only: the
    # small-piece kernel's workload
    "blocktree20000s": lambda: block_tree(max_size=256),
    "grid512": lambda: grid_deleted(),
}
