// Farness and closeness on the shattered graph: host preparation and the
// block-cut tree pass that puts the per-piece sums together (the formulas are
// stated in far.hpp).
#include "far.hpp"

#include <algorithm>
#include <chrono>
#include <numeric>

#include "shatterbc.h"

namespace sbc {

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Appends one piece from an edge list over original ids; reach_of(x) gives
// each vertex's copy reach.  With `bfs_order`, local ids follow a
// breadth-first search from the highest-degree vertex.  Returns the piece
// index; `loc` must be all -1 on entry and is restored.
template <typename ReachOf>
int32_t add_piece(FarPrepared* F, const std::vector<int32_t>& eu, const std::vector<int32_t>& ev, bool bfs_order,
                  std::vector<int32_t>& loc, ReachOf reach_of) {
  std::vector<int32_t> verts;
  for (size_t i = 0; i < eu.size(); ++i)
    for (int32_t x : {eu[i], ev[i]})
      if (loc[x] < 0) {
        loc[x] = (int32_t)verts.size();
        verts.push_back(x);
      }
  const int32_t np = (int32_t)verts.size();
  std::vector<int32_t> deg(np, 0);
  for (size_t i = 0; i < eu.size(); ++i) {
    deg[loc[eu[i]]]++;
    deg[loc[ev[i]]]++;
  }
  std::vector<int32_t> rp(np + 1, 0), cl(2 * eu.size());
  for (int32_t v = 0; v < np; ++v) rp[v + 1] = rp[v] + deg[v];
  std::vector<int32_t> fill(rp.begin(), rp.end() - 1);
  for (size_t i = 0; i < eu.size(); ++i) {
    const int32_t a = loc[eu[i]], b = loc[ev[i]];
    cl[fill[a]++] = b;
    cl[fill[b]++] = a;
  }
  // new local id of each first-seen local id
  std::vector<int32_t> perm(np);
  if (bfs_order && np > 0) {
    int32_t start = 0;
    for (int32_t v = 1; v < np; ++v)
      if (deg[v] > deg[start]) start = v;
    std::vector<int32_t> q;
    q.reserve(np);
    std::vector<uint8_t> seen(np, 0);
    for (int32_t s0 = 0; s0 < np; ++s0) {  // a block is connected; the loop only guards
      const int32_t s = (s0 == 0) ? start : s0;
      if (seen[s]) continue;
      seen[s] = 1;
      q.push_back(s);
      for (size_t h = q.size() - 1; h < q.size(); ++h) {
        const int32_t v = q[h];
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e)
          if (!seen[cl[e]]) {
            seen[cl[e]] = 1;
            q.push_back(cl[e]);
          }
      }
    }
    for (int32_t i = 0; i < np; ++i) perm[q[i]] = i;
  } else {
    std::iota(perm.begin(), perm.end(), 0);
  }
  std::vector<int32_t> inv(np);
  for (int32_t v = 0; v < np; ++v) inv[perm[v]] = v;
  const int32_t base = F->vtx_off.back();
  const int32_t piece = F->pieces();
  for (int32_t nv = 0; nv < np; ++nv) {
    const int32_t v = inv[nv];
    std::vector<int32_t> nb;
    nb.reserve(rp[v + 1] - rp[v]);
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e) nb.push_back(perm[cl[e]]);
    std::sort(nb.begin(), nb.end());
    F->col.insert(F->col.end(), nb.begin(), nb.end());
    F->row.push_back((int32_t)F->col.size());
    const int64_t r = reach_of(verts[v]);
    F->reach.push_back((int32_t)r);
    if (r > 1) F->weighted = true;
    F->orig.push_back(verts[v]);
  }
  F->vtx_off.push_back(base + np);
  for (int32_t x : verts) loc[x] = -1;
  return piece;
}

int32_t local_of(const FarPrepared& F, int32_t piece, int32_t x) {
  for (int32_t g = F.vtx_off[piece]; g < F.vtx_off[piece + 1]; ++g)
    if (F.orig[g] == x) return g - F.vtx_off[piece];
  return -1;
}

}  // namespace

int far_prepare(const HostGraph& g, const std::string& ops, FarPrepared* F, std::string* why) {
  bool opd = false, opa = false, opo = false;
  for (char c : ops) {
    if (c == 'o') opo = true;
    else if (c == 'd') opd = true;
    else if (c == 'a') opa = true;
    else {
      *why = std::string("preprocessing letter '") + c + "' is not available for farness (known: o, d, a)";
      return SBC_E_INVALID_ARG;
    }
  }
  const double t0 = now_ms();
  *F = FarPrepared();
  const int32_t n = g.n;
  F->n = n;
  F->vtx_off.push_back(0);
  F->row.push_back(0);
  F->comp.assign(n, -1);
  {
    std::vector<int32_t> q;
    q.reserve(n);
    for (int32_t s = 0; s < n; ++s) {
      if (F->comp[s] >= 0) continue;
      const int32_t c = (int32_t)F->comp_size.size();
      F->comp[s] = c;
      q.clear();
      q.push_back(s);
      for (size_t h = 0; h < q.size(); ++h)
        for (int32_t e = g.row_ptr[q[h]]; e < g.row_ptr[q[h] + 1]; ++e)
          if (F->comp[g.col[e]] < 0) {
            F->comp[g.col[e]] = c;
            q.push_back(g.col[e]);
          }
      F->comp_size.push_back((int64_t)q.size());
    }
  }
  std::vector<int64_t> r(n, 1);
  F->h.assign(n, 0);
  std::vector<uint8_t> alive(n, 1);
  std::vector<int32_t> deg(n);
  for (int32_t v = 0; v < n; ++v) deg[v] = g.row_ptr[v + 1] - g.row_ptr[v];

  if (opd) {
    std::vector<int32_t> q;
    for (int32_t v = 0; v < n; ++v)
      if (deg[v] == 1) q.push_back(v);
    for (size_t k = 0; k < q.size(); ++k) {
      const int32_t u = q[k];
      if (!alive[u] || deg[u] != 1) continue;
      int32_t v = -1;
      for (int32_t e = g.row_ptr[u]; e < g.row_ptr[u + 1]; ++e)
        if (alive[g.col[e]]) {
          v = g.col[e];
          break;
        }
      F->strip_u.push_back(u);
      F->strip_v.push_back(v);
      F->strip_size.push_back(r[u]);
      F->h[v] += F->h[u] + r[u];
      r[v] += r[u];
      alive[u] = 0;
      deg[u] = 0;
      F->stripped++;
      if (--deg[v] == 1) q.push_back(v);
    }
  }

  std::vector<int32_t> loc(n, -1), eu, ev;
  if (opa) {
    // Blocks of the stripped graph by an iterative Hopcroft-Tarjan search;
    // copy reach as in the betweenness preprocessing: R - W(child) for the
    // block's top vertex, the vertex's own reach plus the subtrees already
    // hung from it as separate blocks for every other vertex.
    std::vector<int32_t> disc(n, -1), low(n, 0), parent(n, -1), it(n, 0);
    std::vector<int64_t> Wsub(n, 0), hang(n, 0);
    std::vector<int32_t> stk, est_u, est_v;
    int32_t timer = 0;
    for (int32_t root = 0; root < n; ++root) {
      if (!alive[root] || disc[root] >= 0) continue;
      F->roots.push_back(root);
      const int64_t R = F->comp_size[F->comp[root]];
      disc[root] = low[root] = timer++;
      Wsub[root] = hang[root] = r[root];
      it[root] = g.row_ptr[root];
      stk.push_back(root);
      while (!stk.empty()) {
        const int32_t v = stk.back();
        if (it[v] < g.row_ptr[v + 1]) {
          const int32_t w = g.col[it[v]++];
          if (!alive[w]) continue;
          if (disc[w] < 0) {
            parent[w] = v;
            disc[w] = low[w] = timer++;
            Wsub[w] = hang[w] = r[w];
            it[w] = g.row_ptr[w];
            est_u.push_back(v);
            est_v.push_back(w);
            stk.push_back(w);
          } else if (w != parent[v] && disc[w] < disc[v]) {
            low[v] = std::min(low[v], disc[w]);
            est_u.push_back(v);
            est_v.push_back(w);
          }
          continue;
        }
        stk.pop_back();
        if (v == root) break;
        const int32_t p = parent[v];
        low[p] = std::min(low[p], low[v]);
        Wsub[p] += Wsub[v];
        if (low[v] < disc[p]) continue;
        // p is the top of a block whose edges sit on the edge stack down to (p, v)
        F->nblocks++;
        hang[p] += Wsub[v];
        eu.clear();
        ev.clear();
        while (true) {
          const int32_t a = est_u.back(), b = est_v.back();
          est_u.pop_back();
          est_v.pop_back();
          eu.push_back(a);
          ev.push_back(b);
          if (a == p && b == v) break;
        }
        FarBlock B;
        B.top = p;
        const int64_t rtop = R - Wsub[v];
        if (eu.size() == 1) {
          B.a = p;
          B.b = v;
          B.ra = rtop;
          B.rb = hang[v];
          F->bridges++;
        } else {
          B.piece = add_piece(F, eu, ev, opo, loc, [&](int32_t x) { return x == p ? rtop : hang[x]; });
          B.top_local = local_of(*F, B.piece, p);
        }
        F->blocks.push_back(B);
      }
    }
  } else {
    // No shattering: every component of the stripped graph with an edge is one piece.
    std::vector<uint8_t> seen(n, 0);
    std::vector<int32_t> q;
    for (int32_t s = 0; s < n; ++s) {
      if (!alive[s] || seen[s]) continue;
      F->roots.push_back(s);
      q.clear();
      q.push_back(s);
      seen[s] = 1;
      eu.clear();
      ev.clear();
      for (size_t k = 0; k < q.size(); ++k) {
        const int32_t v = q[k];
        for (int32_t e = g.row_ptr[v]; e < g.row_ptr[v + 1]; ++e) {
          const int32_t w = g.col[e];
          if (!alive[w]) continue;
          if (v < w) {
            eu.push_back(v);
            ev.push_back(w);
          }
          if (!seen[w]) {
            seen[w] = 1;
            q.push_back(w);
          }
        }
      }
      if (eu.empty()) continue;
      FarBlock B;
      B.piece = add_piece(F, eu, ev, opo, loc, [&](int32_t x) { return r[x]; });
      F->blocks.push_back(B);
    }
  }
  {
    // source order (the clustering of the betweenness batches, mode 2)
    Prepared tmp;
    tmp.n = n;
    std::swap(tmp.vtx_off, F->vtx_off);
    std::swap(tmp.row, F->row);
    std::swap(tmp.col, F->col);
    tmp.src_order.assign((size_t)tmp.V(), 0);
    cluster_sources(&tmp, 64, 2);
    std::swap(tmp.vtx_off, F->vtx_off);
    std::swap(tmp.row, F->row);
    std::swap(tmp.col, F->col);
    std::swap(tmp.src_order, F->src_order);
  }
  F->ms_prep = now_ms() - t0;
  return SBC_OK;
}

int far_finish(const FarPrepared& F, const int64_t* W, int64_t* farness, double* closeness, std::string* why) {
  const int32_t n = F.n;
  if (F.V() > 0 && !W) {
    *why = "piece sums missing";
    return SBC_E_INVALID_ARG;
  }
  std::vector<int64_t> acc(F.h.begin(), F.h.end());
  std::vector<int64_t> f(n, -1);
  auto w_of = [&](const FarBlock& B, int32_t x_local_or_orig, bool top) -> int64_t {
    if (B.piece >= 0) return W[F.vtx_off[B.piece] + (top ? B.top_local : x_local_or_orig)];
    return (top || x_local_or_orig == B.a) ? B.rb : B.ra;  // the other end's reach at distance 1
  };
  // Upward: the blocks closed first hang lowest.
  for (const FarBlock& B : F.blocks) {
    if (B.top < 0) {  // a whole component
      int64_t down = 0;
      for (int32_t gx = F.vtx_off[B.piece]; gx < F.vtx_off[B.piece + 1]; ++gx) down += acc[F.orig[gx]];
      for (int32_t gx = F.vtx_off[B.piece]; gx < F.vtx_off[B.piece + 1]; ++gx) f[F.orig[gx]] = W[gx] + down;
      continue;
    }
    int64_t down = 0;
    if (B.piece >= 0) {
      for (int32_t gx = F.vtx_off[B.piece]; gx < F.vtx_off[B.piece + 1]; ++gx)
        if (F.orig[gx] != B.top) down += acc[F.orig[gx]];
    } else {
      down = acc[B.b];
    }
    acc[B.top] += w_of(B, 0, true) + down;
  }
  // Search roots (also a stripped graph's lone vertices): everything hangs from them.
  for (int32_t rt : F.roots)
    if (f[rt] < 0) f[rt] = acc[rt];
  // Downward: parents before children.
  for (size_t k = F.blocks.size(); k-- > 0;) {
    const FarBlock& B = F.blocks[k];
    if (B.top < 0) continue;
    const int64_t ft = f[B.top];
    if (ft < 0) {
      *why = "block-cut tree order broken";
      return SBC_E_INVALID_ARG;
    }
    const int64_t wt = w_of(B, 0, true);
    if (B.piece >= 0) {
      for (int32_t gx = F.vtx_off[B.piece]; gx < F.vtx_off[B.piece + 1]; ++gx)
        if (F.orig[gx] != B.top) f[F.orig[gx]] = W[gx] + ft - wt;
    } else {
      f[B.b] = w_of(B, B.b, false) + ft - wt;
    }
  }
  // Stripped vertices, last removed first.
  for (size_t k = F.strip_u.size(); k-- > 0;) {
    const int32_t u = F.strip_u[k], v = F.strip_v[k];
    const int64_t R = F.comp_size[F.comp[u]];
    f[u] = f[v] + R - 2 * F.strip_size[k];
  }
  for (int32_t v = 0; v < n; ++v) {
    if (f[v] < 0) {  // only a vertex no step reached: an isolated vertex has farness 0
      if (F.comp_size[F.comp[v]] != 1) {
        *why = "vertex without farness";
        return SBC_E_INVALID_ARG;
      }
      f[v] = 0;
    }
    farness[v] = f[v];
    if (closeness) closeness[v] = f[v] > 0 ? (double)(F.comp_size[F.comp[v]] - 1) / (double)f[v] : 0.0;
  }
  return SBC_OK;
}

}  // namespace sbc
