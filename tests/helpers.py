"""Test-side helpers: graph expansions and closed forms (no library code)."""
from __future__ import annotations

import numpy as np

import graphgen as gg


def expand_attributed(n, row_ptr, col, reach, ident, twin_type):
    """Build the ordinary graph an attributed piece stands for.

    Vertex v of the piece becomes ident[v] copies; copies of adjacent vertices
    are all adjacent; copies of v are pairwise adjacent when twin_type[v] == 2
    (closed-neighbourhood twins) and pairwise non-adjacent when it is 1
    (open-neighbourhood twins).  Each copy then gets reach[v]-1 pendant leaves,
    the vertices it represents that hang off it through it alone.

    Returns (Graph, first_copy) with first_copy[v] = id of v's first copy.
    """
    reach = np.asarray(reach, dtype=np.int64)
    ident = np.asarray(ident, dtype=np.int64)
    copy_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(ident, out=copy_off[1:])
    nc = int(copy_off[-1])
    us, vs = [], []
    rp = np.asarray(row_ptr)
    for v in range(n):
        cv = range(copy_off[v], copy_off[v + 1])
        for e in range(rp[v], rp[v + 1]):
            u = int(col[e])
            if u < v:
                continue
            for a in cv:
                for b in range(copy_off[u], copy_off[u + 1]):
                    us.append(a)
                    vs.append(b)
        if twin_type[v] == 2:
            cl = list(cv)
            for i in range(len(cl)):
                for j in range(i + 1, len(cl)):
                    us.append(cl[i])
                    vs.append(cl[j])
    nxt = nc
    for v in range(n):
        for a in range(copy_off[v], copy_off[v + 1]):
            for _ in range(int(reach[v]) - 1):
                us.append(a)
                vs.append(nxt)
                nxt += 1
    g = gg.csr_from_edges(nxt, np.array(us, dtype=np.int64), np.array(vs, dtype=np.int64), "expanded")
    return g, copy_off[:-1]


def expand_classes(n, row_ptr, col, members, twin_type):
    """Like expand_attributed, with members[v] the list of the reaches of v's
    copies (which may differ): copy j of v gets members[v][j] - 1 pendant
    leaves.  Returns (Graph, copy_off) with v's copies copy_off[v] ..
    copy_off[v+1]-1."""
    ident = np.array([len(m) for m in members], dtype=np.int64)
    copy_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(ident, out=copy_off[1:])
    us, vs = [], []
    rp = np.asarray(row_ptr)
    for v in range(n):
        cv = range(copy_off[v], copy_off[v + 1])
        for e in range(rp[v], rp[v + 1]):
            u = int(col[e])
            if u < v:
                continue
            for a in cv:
                for b in range(copy_off[u], copy_off[u + 1]):
                    us.append(a)
                    vs.append(b)
        if twin_type[v] == 2:
            cl = list(cv)
            for i in range(len(cl)):
                for j in range(i + 1, len(cl)):
                    us.append(cl[i])
                    vs.append(cl[j])
    nxt = int(copy_off[-1])
    for v in range(n):
        for j, a in enumerate(range(copy_off[v], copy_off[v + 1])):
            for _ in range(int(members[v][j]) - 1):
                us.append(a)
                vs.append(nxt)
                nxt += 1
    g = gg.csr_from_edges(nxt, np.array(us, dtype=np.int64), np.array(vs, dtype=np.int64), "expanded")
    return g, copy_off


def twin_corrections(n, row_ptr, col, reach, ident, twin_type):
    """Per-member score the merged traversal cannot see (derived from Sec. 3.3.3).

    (i)  every member of a class of k >= 2 members with reach r gets
         (k-1)*r*(r-1): pairs from a class-mate's group to targets hanging
         below this member;
    (ii) an open-neighbourhood class spreads its k(k-1)*r^2 member-to-member
         paths evenly over the D = sum of ident over its neighbours, so each
         member of a neighbour class gets k(k-1)r^2/D.
    """
    rp = np.asarray(row_ptr)
    corr = np.zeros(n, dtype=np.float64)
    for v in range(n):
        k, r = int(ident[v]), int(reach[v])
        if k < 2:
            continue
        corr[v] += (k - 1) * r * (r - 1)
        if twin_type[v] == 1:
            nb = col[rp[v]:rp[v + 1]]
            D = int(np.sum(np.asarray(ident)[nb]))
            if D > 0:
                for x in nb:
                    corr[int(x)] += k * (k - 1) * r * r / D
    return corr


def tree_closed_form(g: gg.Graph) -> np.ndarray:
    """Ordered-pair BC of a tree: (n-1)^2 - sum of squared branch sizes at v."""
    n = g.n
    rp, col = g.row_ptr, g.col
    parent = np.full(n, -1)
    order = []
    seen = np.zeros(n, dtype=bool)
    out = np.zeros(n)
    for root in range(n):
        if seen[root]:
            continue
        comp = []
        stack = [root]
        seen[root] = True
        while stack:
            v = stack.pop()
            comp.append(v)
            for w in col[rp[v]:rp[v + 1]]:
                if not seen[w]:
                    seen[w] = True
                    parent[w] = v
                    stack.append(w)
        size = {v: 1 for v in comp}
        for v in reversed(comp):
            if parent[v] >= 0:
                size[parent[v]] += size[v]
        N = len(comp)
        for v in comp:
            br = [size[w] for w in col[rp[v]:rp[v + 1]] if parent[w] == v]
            if parent[v] >= 0:
                br.append(N - size[v])
            out[v] = (N - 1) ** 2 - sum(b * b for b in br)
        order += comp
    return out


def unequal_atol(n: int) -> float:
    """Absolute slack for results with identical vertices of unequal reach
    merged ('u'): a member's score is its class's traversal value (dependency
    started at the members' mean reach) plus a signed per-member term, both of
    magnitude up to n^2, so an exact 0 comes out within rounding of 0.  About
    4 ulps of n^2; a wrong term is off by at least a fraction of one pair."""
    return 1e-15 * float(n) * float(n)


def assert_bc_close(got, want, rtol=1e-9, what="", atol=0.0):
    """Per-vertex |g - o| <= rtol*|o| + atol; with atol = 0 (every term of a
    score non-negative), g == 0 exactly where o == 0."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape, (got.shape, want.shape)
    zero = want == 0
    bad_zero = np.flatnonzero(zero & (np.abs(got) > atol))
    assert bad_zero.size == 0, f"{what}: nonzero where exact value is 0 at {bad_zero[:10]} -> {got[bad_zero[:10]]}"
    err = np.abs(got - want)
    tol = rtol * np.abs(want) + atol
    bad = np.flatnonzero(err > tol)
    assert bad.size == 0, (f"{what}: {bad.size} vertices off; worst rel "
                           f"{np.max(err[~zero] / np.abs(want[~zero])) if (~zero).any() else 0:.3e} at "
                           f"{bad[:5]} got {got[bad[:5]]} want {want[bad[:5]]}")


def member_reach(ex):
    """Per-member reach of exported piece vertices whose members all have the
    same reach (the export carries each piece vertex's members' reach sum)."""
    r, k = ex["reach"].astype(np.int64), ex["ident"].astype(np.int64)
    assert np.all(r % k == 0), "a piece vertex merges members of unequal reach"
    return (r // k).astype(np.int32)


def oracle_pieces(ex, threads=None):
    """bc' of every exported piece by the oracle: Algorithm 2 with ident
    weights (oracle.bc_pieces) where every class has members of one reach,
    oracle.bc_classes for the pieces holding a class of unequal reaches."""
    import oracle

    r, k = ex["reach"].astype(np.int64), ex["ident"].astype(np.int64)
    even = r % k == 0
    bcp = oracle.bc_pieces(ex["vtx_off"], ex["row"], ex["col"], np.where(even, r // k, 1).astype(np.int32),
                           ex["ident"], threads=threads)
    for p in np.unique(np.searchsorted(ex["vtx_off"], np.flatnonzero(~even), side="right") - 1):
        vb, ve = int(ex["vtx_off"][p]), int(ex["vtx_off"][p + 1])
        rp = (ex["row"][vb:ve + 1] - ex["row"][vb]).astype(np.int32)
        cl = ex["col"][ex["row"][vb]:ex["row"][ve]].astype(np.int32)
        bcp[vb:ve] = oracle.bc_classes(ve - vb, rp, cl, ex["reach"][vb:ve], ex["ident"][vb:ve], threads=threads)
    return bcp


def piece_csr(ex, p):
    """Local CSR (row_ptr, col), per-member reach and ident of exported piece p."""
    vb, ve = int(ex["vtx_off"][p]), int(ex["vtx_off"][p + 1])
    rp = (ex["row"][vb:ve + 1] - ex["row"][vb]).astype(np.int32)
    cl = ex["col"][ex["row"][vb]:ex["row"][ve]].astype(np.int32)
    return rp, cl, member_reach(ex)[vb:ve], ex["ident"][vb:ve]


def map_back(ex, bcp):
    """Eq. (5): bc[v] = bcx[v] + sum over the piece vertices x standing for v
    of (bc'[x] + corr[x]), for an exported preprocessing and per-piece bc'."""
    n = len(ex["map_off"]) - 1
    out = np.array(ex["bcx"][:n], dtype=np.float64, copy=True)
    owner = np.repeat(np.arange(n), np.diff(ex["map_off"]))
    idx = ex["map_idx"][:len(owner)]
    np.add.at(out, owner, np.asarray(bcp)[idx] + ex["corr"][idx])
    return out
