// Host-side validation and preprocessing.  See prep.hpp for the overview.
#include "prep.hpp"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>

#include "status.hpp"

namespace sbc {

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

inline uint64_t mix64(uint64_t x) {  // splitmix64 finaliser
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

}  // namespace

int validate_csr(int32_t n, const int32_t* row_ptr, const int32_t* col, bool sanitize, HostGraph* out,
                 std::string* why) {
  if (n < 0 || (!row_ptr)) {
    *why = "n < 0 or row_ptr is NULL";
    return SBC_E_INVALID_ARG;
  }
  if (row_ptr[0] != 0) {
    *why = "row_ptr[0] != 0";
    return SBC_E_INVALID_ARG;
  }
  for (int32_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) {
      *why = "row_ptr is not non-decreasing at vertex " + std::to_string(v);
      return SBC_E_INVALID_ARG;
    }
  const int64_t arcs = row_ptr[n];
  if (arcs > 0 && !col) {
    *why = "col is NULL";
    return SBC_E_INVALID_ARG;
  }
  for (int64_t e = 0; e < arcs; ++e)
    if (col[e] < 0 || col[e] >= n) {
      *why = "column index out of range at arc " + std::to_string(e);
      return SBC_E_INDEX_RANGE;
    }
  HostGraph g;
  g.n = n;
  if (!sanitize) {
    g.row_ptr.assign(row_ptr, row_ptr + n + 1);
    g.col.assign(col, col + arcs);
    for (int32_t v = 0; v < n; ++v) {
      auto b = g.col.begin() + g.row_ptr[v], e = g.col.begin() + g.row_ptr[v + 1];
      std::sort(b, e);
      for (auto it = b; it != e; ++it) {
        if (*it == v) {
          *why = "self loop at vertex " + std::to_string(v);
          return SBC_E_SELF_LOOP;
        }
        if (it != b && *it == *(it - 1)) {
          *why = "duplicate arc " + std::to_string(v) + "->" + std::to_string(*it);
          return SBC_E_DUP_EDGE;
        }
      }
    }
    for (int32_t v = 0; v < n; ++v)
      for (int32_t e = g.row_ptr[v]; e < g.row_ptr[v + 1]; ++e) {
        int32_t u = g.col[e];
        auto b = g.col.begin() + g.row_ptr[u], en = g.col.begin() + g.row_ptr[u + 1];
        if (!std::binary_search(b, en, v)) {
          *why = "arc " + std::to_string(v) + "->" + std::to_string(u) + " has no reverse arc";
          return SBC_E_NOT_SYMMETRIC;
        }
      }
  } else {
    std::vector<uint64_t> keys;
    keys.reserve(2 * arcs);
    for (int32_t v = 0; v < n; ++v)
      for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        int32_t u = col[e];
        if (u == v) continue;
        keys.push_back((uint64_t)v * (uint64_t)n + (uint64_t)u);
        keys.push_back((uint64_t)u * (uint64_t)n + (uint64_t)v);
      }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    if (keys.size() > (size_t)INT32_MAX) {
      *why = "symmetrised graph has 2^31 or more arcs";
      return SBC_E_TOO_LARGE;
    }
    g.row_ptr.assign(n + 1, 0);
    g.col.resize(keys.size());
    for (size_t i = 0; i < keys.size(); ++i) {
      g.row_ptr[keys[i] / n + 1]++;
      g.col[i] = (int32_t)(keys[i] % n);
    }
    for (int32_t v = 0; v < n; ++v) g.row_ptr[v + 1] += g.row_ptr[v];
  }
  *out = std::move(g);
  return SBC_OK;
}

void plain_problem(const HostGraph& g, Prepared* P) {
  *P = Prepared();
  P->n = g.n;
  P->vtx_off = {0, g.n};
  P->row = g.row_ptr;
  P->col = g.col;
  P->reach.assign(g.n, 1);
  P->ident.assign(g.n, 1);
  P->corr.assign(g.n, 0.0);
  P->bcx.assign(g.n, 0.0);
  P->map_off.resize(g.n + 1);
  std::iota(P->map_off.begin(), P->map_off.end(), 0);
  P->map_idx.resize(g.n);
  std::iota(P->map_idx.begin(), P->map_idx.end(), 0);
  P->src_order.resize(g.n);
  std::iota(P->src_order.begin(), P->src_order.end(), 0);
  P->nside.assign(1, 0);
}

namespace {

// A piece before twin merging: original vertex ids, their reach in the piece,
// and a local CSR.
struct RawPiece {
  std::vector<int32_t> verts;
  std::vector<int64_t> reach;
  std::vector<int32_t> rp, cl;
};

// Final piece contents collected before packing.
struct OutPiece {
  std::vector<int32_t> rp, cl;    // quotient CSR (local ids)
  std::vector<int32_t> reach, ident;
  std::vector<double> corr;
  std::vector<int32_t> member_orig;  // original id of each member
  std::vector<int32_t> member_cls;   // quotient vertex of each member
  int32_t nside = 0;                 // side piece: its side vertices are local 0..nside-1
};

struct Builder {
  const HostGraph& g;
  bool opi, op_side;
  bool any_reach = false;  // identical vertices merge whatever their reach ('u')
  std::vector<double>& bcx;
  PrepStats* st;
  std::vector<OutPiece> out;
  std::vector<int32_t> loc;  // scratch: original id -> local id, -1 otherwise
  double ms_twins = 0;

  Builder(const HostGraph& g_, bool opi_, bool side_, std::vector<double>& bcx_, PrepStats* st_)
      : g(g_), opi(opi_), op_side(side_), bcx(bcx_), st(st_), loc(g_.n, -1) {}

  // Side vertices (Section 3.3.2): vertices of degree 1..4 whose neighbours
  // are pairwise adjacent, so that no shortest path between two other
  // vertices passes through them.  They are removed one after another in
  // local id order (each stays a side vertex when earlier ones go, since a
  // clique minus a vertex is a clique), and at least one vertex stays.  The
  // block as it was goes out as a side piece with the side vertices first,
  // in removal order; each removed vertex u gets its own dependency term
  // (reach[u]-1) x (the reach left in the component after removing it) on
  // the host; the piece continues without them.
  void strip_side_vertices(RawPiece& p) {
    const int32_t np = (int32_t)p.verts.size();
    if (np < 3) return;
    auto adjacent = [&](int32_t a, int32_t b) {
      return std::binary_search(p.cl.begin() + p.rp[a], p.cl.begin() + p.rp[a + 1], b);
    };
    std::vector<int32_t> side;
    for (int32_t v = 0; v < np; ++v) {
      const int32_t k = p.rp[v + 1] - p.rp[v];
      if (k < 1 || k > 4) continue;
      bool clique = true;
      for (int32_t i = p.rp[v]; i < p.rp[v + 1] && clique; ++i)
        for (int32_t j = i + 1; j < p.rp[v + 1] && clique; ++j) clique = adjacent(p.cl[i], p.cl[j]);
      if (clique) side.push_back(v);
    }
    if ((int32_t)side.size() == np) side.pop_back();
    if (side.empty()) return;
    const int32_t ns = (int32_t)side.size();
    // the side piece: side vertices first, then the rest in local order
    std::vector<int32_t> nid(np, -1), old_of(np);
    for (int32_t i = 0; i < ns; ++i) nid[side[i]] = i;
    int32_t nxt = ns;
    for (int32_t v = 0; v < np; ++v)
      if (nid[v] < 0) nid[v] = nxt++;
    for (int32_t v = 0; v < np; ++v) old_of[nid[v]] = v;
    OutPiece q;
    q.rp.assign(np + 1, 0);
    for (int32_t i = 0; i < np; ++i) {
      const int32_t v = old_of[i];
      for (int32_t e = p.rp[v]; e < p.rp[v + 1]; ++e) q.cl.push_back(nid[p.cl[e]]);
      std::sort(q.cl.begin() + q.rp[i], q.cl.end());
      q.rp[i + 1] = (int32_t)q.cl.size();
      q.reach.push_back((int32_t)p.reach[v]);
      q.member_orig.push_back(p.verts[v]);
    }
    q.ident.assign(np, 1);
    q.corr.assign(np, 0.0);
    q.member_cls.resize(np);
    std::iota(q.member_cls.begin(), q.member_cls.end(), 0);
    q.nside = ns;
    // each removed vertex's own term, with the reach left after removing it
    int64_t left = 0;
    for (int32_t v = 0; v < np; ++v) left += p.reach[v];
    for (int32_t u : side) {
      left -= p.reach[u];
      bcx[p.verts[u]] += (double)(p.reach[u] - 1) * (double)left;
    }
    out.push_back(std::move(q));
    st->side_vertices += ns;
    st->side_pieces++;
    // the block without its side vertices
    std::vector<uint8_t> gone(np, 0);
    for (int32_t u : side) gone[u] = 1;
    RawPiece r;
    std::vector<int32_t> rid(np, -1);
    for (int32_t v = 0; v < np; ++v)
      if (!gone[v]) {
        rid[v] = (int32_t)r.verts.size();
        r.verts.push_back(p.verts[v]);
        r.reach.push_back(p.reach[v]);
      }
    r.rp.assign(r.verts.size() + 1, 0);
    for (int32_t v = 0; v < np; ++v) {
      if (gone[v]) continue;
      for (int32_t e = p.rp[v]; e < p.rp[v + 1]; ++e)
        if (!gone[p.cl[e]]) r.cl.push_back(rid[p.cl[e]]);  // rows stay sorted: rid keeps the order
      r.rp[rid[v] + 1] = (int32_t)r.cl.size();
    }
    p = std::move(r);
  }

  // Local CSR of the piece from an edge list of original ids.
  void build_local(RawPiece& p, const std::vector<int32_t>& eu, const std::vector<int32_t>& ev) {
    const int32_t np = (int32_t)p.verts.size();
    for (int32_t i = 0; i < np; ++i) loc[p.verts[i]] = i;
    p.rp.assign(np + 1, 0);
    for (size_t i = 0; i < eu.size(); ++i) {
      p.rp[loc[eu[i]] + 1]++;
      p.rp[loc[ev[i]] + 1]++;
    }
    for (int32_t i = 0; i < np; ++i) p.rp[i + 1] += p.rp[i];
    p.cl.resize(p.rp[np]);
    std::vector<int32_t> fill(p.rp.begin(), p.rp.end() - 1);
    for (size_t i = 0; i < eu.size(); ++i) {
      int32_t a = loc[eu[i]], b = loc[ev[i]];
      p.cl[fill[a]++] = b;
      p.cl[fill[b]++] = a;
    }
    for (int32_t i = 0; i < np; ++i) std::sort(p.cl.begin() + p.rp[i], p.cl.begin() + p.rp[i + 1]);
    for (int32_t i = 0; i < np; ++i) loc[p.verts[i]] = -1;
  }

  // Identical-vertex classes (Section 3.3.3) inside one piece, then the
  // quotient graph with ident = class size and the per-member terms the merged
  // traversal cannot see:
  //  (i)  each member of a class of k members with reach r: (k-1) r (r-1), the
  //       pairs (class-mate group -> vertices hanging below this member);
  //  (ii) an open-neighbourhood class spreads its k(k-1) r^2 member-to-member
  //       paths evenly over the D members of its neighbour classes.
  // Only members with equal reach are merged.
  void finish_piece(RawPiece& p) {
    if (op_side) strip_side_vertices(p);
    const int32_t np = (int32_t)p.verts.size();
    std::vector<int32_t> cls(np);
    std::vector<int8_t> ctype;  // per class: 0 singleton, 1 open, 2 closed neighbourhood
    int32_t C = 0;
    if (opi && np >= 2) {
      double t0 = now_ms();
      std::vector<uint64_t> hsum(np, 0);
      for (int32_t v = 0; v < np; ++v) {
        uint64_t h = 0;
        for (int32_t e = p.rp[v]; e < p.rp[v + 1]; ++e) h += mix64((uint64_t)p.cl[e]);
        hsum[v] = h;
      }
      std::vector<int32_t> head(np, -1);  // class representative of each vertex (-1: none yet)
      auto deg = [&](int32_t v) { return p.rp[v + 1] - p.rp[v]; };
      auto same_open = [&](int32_t a, int32_t b) {
        return deg(a) == deg(b) &&
               std::equal(p.cl.begin() + p.rp[a], p.cl.begin() + p.rp[a + 1], p.cl.begin() + p.rp[b]);
      };
      auto same_closed = [&](int32_t a, int32_t b) {
        if (deg(a) != deg(b)) return false;
        if (!std::binary_search(p.cl.begin() + p.rp[a], p.cl.begin() + p.rp[a + 1], b)) return false;
        // Gamma(a) \ {b} must equal Gamma(b) \ {a}
        int32_t i = p.rp[a], ie = p.rp[a + 1], j = p.rp[b], je = p.rp[b + 1];
        while (true) {
          while (i < ie && p.cl[i] == b) ++i;
          while (j < je && p.cl[j] == a) ++j;
          if (i == ie || j == je) return i == ie && j == je;
          if (p.cl[i] != p.cl[j]) return false;
          ++i;
          ++j;
        }
      };
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<int32_t> order;
        order.reserve(np);
        for (int32_t v = 0; v < np; ++v)
          if (head[v] == -1 && deg(v) > 0) order.push_back(v);
        auto key = [&](int32_t v) {
          return pass == 0 ? hsum[v] : hsum[v] + mix64((uint64_t)v);
        };
        std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
          uint64_t ka = key(a), kb = key(b);
          if (ka != kb) return ka < kb;
          if (deg(a) != deg(b)) return deg(a) < deg(b);
          if (!any_reach && p.reach[a] != p.reach[b]) return p.reach[a] < p.reach[b];
          return a < b;
        });
        size_t i = 0;
        while (i < order.size()) {
          size_t j = i + 1;
          while (j < order.size() && key(order[j]) == key(order[i]) && deg(order[j]) == deg(order[i]) &&
                 (any_reach || p.reach[order[j]] == p.reach[order[i]]))
            ++j;
          if (j - i >= 2) {
            std::vector<int32_t> reps;
            for (size_t t = i; t < j; ++t) {
              int32_t v = order[t];
              bool joined = false;
              for (int32_t rep : reps)
                if (pass == 0 ? same_open(rep, v) : same_closed(rep, v)) {
                  head[v] = rep;
                  joined = true;
                  break;
                }
              if (!joined) reps.push_back(v);
            }
            for (int32_t rep : reps) {
              bool has_member = false;
              for (size_t t = i; t < j; ++t)
                if (head[order[t]] == rep) has_member = true;
              if (has_member) head[rep] = rep;
            }
          }
          i = j;
        }
        if (pass == 0) {
          // members found in pass 0 are open-neighbourhood twins; mark them so
          // pass 1 skips them (a vertex cannot have twins of both kinds)
          for (int32_t v = 0; v < np; ++v)
            if (head[v] >= 0) head[v] = -2 - head[v];
        }
      }
      // classes numbered by representative (smallest local id) order
      std::vector<int32_t> rep_of(np);
      std::vector<int8_t> kind(np, 0);
      for (int32_t v = 0; v < np; ++v) {
        if (head[v] <= -2) {
          rep_of[v] = -2 - head[v];
          kind[v] = 1;
        } else if (head[v] >= 0) {
          rep_of[v] = head[v];
          kind[v] = 2;
        } else {
          rep_of[v] = v;
        }
      }
      std::vector<int32_t> cid(np, -1);
      for (int32_t v = 0; v < np; ++v)
        if (rep_of[v] == v) {
          cid[v] = C++;
          ctype.push_back(kind[v]);
        }
      for (int32_t v = 0; v < np; ++v) cls[v] = cid[rep_of[v]];
      ms_twins += now_ms() - t0;
    } else {
      for (int32_t v = 0; v < np; ++v) cls[v] = v;
      C = np;
      ctype.assign(np, 0);
    }
    // A class stands for its members: ident = their number, reach = the sum
    // of their reaches (k x r when all have reach r).
    OutPiece q;
    q.ident.assign(C, 0);
    q.reach.assign(C, 0);
    q.corr.assign(C, 0.0);
    std::vector<int32_t> rep(C, -1);
    std::vector<int64_t> rsum(C, 0), rsq(C, 0), rlo(C, INT64_MAX), rhi(C, 0);
    int64_t rtot = 0;  // the piece's sources weigh this much together
    for (int32_t v = 0; v < np; ++v) {
      const int32_t c = cls[v];
      const int64_t r = p.reach[v];
      q.ident[c]++;
      rsum[c] += r;
      rsq[c] += r * r;
      rlo[c] = std::min(rlo[c], r);
      rhi[c] = std::max(rhi[c], r);
      rtot += r;
      if (rep[c] < 0) rep[c] = v;
    }
    for (int32_t c = 0; c < C; ++c) q.reach[c] = (int32_t)rsum[c];
    // quotient CSR from the representatives' rows
    q.rp.assign(C + 1, 0);
    for (int32_t c = 0; c < C; ++c) {
      int32_t v = rep[c];
      size_t base = q.cl.size();
      for (int32_t e = p.rp[v]; e < p.rp[v + 1]; ++e) {
        int32_t cu = cls[p.cl[e]];
        if (cu != c) q.cl.push_back(cu);
      }
      std::sort(q.cl.begin() + base, q.cl.end());
      q.cl.erase(std::unique(q.cl.begin() + base, q.cl.end()), q.cl.end());
      q.rp[c + 1] = (int32_t)q.cl.size();
    }
    // Pairs the merged traversal no longer sees, per class of k >= 2 members
    // a, b with reaches r_a, r_b (R = their sum):
    //  (i) sources on member a's side (r_a of them) to targets hung strictly
    //      below another member b pass b: b gets (R - r_b)(r_b - 1), which is
    //      (k - 1) r (r - 1) when all reaches are r;
    //  (ii) open-neighbourhood twins: the sum over a != b of r_a r_b pairs run
    //      through the class's common neighbours, split evenly over the D
    //      original neighbours of a member: each gets (R^2 - sum r^2) / D.
    // With unequal reaches the traversal starts every member's dependency at
    // the class's mean reach R/k minus one, so member b also gets
    // (r_b - R/k) times the weight of every other source of the piece,
    // (rtot - R), when the piece is traversed at all.
    const bool traversed = C > 2;
    std::vector<double> member_extra(np, 0.0);  // per-member terms of unequal classes
    for (int32_t c = 0; c < C; ++c) {
      const int32_t k = q.ident[c];
      if (k < 2) continue;
      st->twin_classes++;
      st->twins_merged += (int64_t)k - 1;
      if (rlo[c] == rhi[c]) {
        const double kk = k, r = (double)rlo[c];
        q.corr[c] += (kk - 1) * r * (r - 1);
      }
      if (ctype[c] == 1) {
        double D = 0;
        for (int32_t e = q.rp[c]; e < q.rp[c + 1]; ++e) D += q.ident[q.cl[e]];
        if (D > 0) {
          double share;
          if (rlo[c] == rhi[c]) {
            const double kk = k, r = (double)rlo[c];
            share = kk * (kk - 1) * r * r / D;
          } else {
            share = (double)(rsum[c] * rsum[c] - rsq[c]) / D;
          }
          for (int32_t e = q.rp[c]; e < q.rp[c + 1]; ++e) q.corr[q.cl[e]] += share;
        }
      }
    }
    for (int32_t v = 0; v < np; ++v) {
      const int32_t c = cls[v];
      if (q.ident[c] < 2 || rlo[c] == rhi[c]) continue;
      const int64_t rb = p.reach[v], R = rsum[c];
      member_extra[v] += (double)((R - rb) * (rb - 1));
      if (traversed) member_extra[v] += ((double)rb - (double)R / (double)q.ident[c]) * (double)(rtot - R);
    }
    q.member_orig = p.verts;
    q.member_cls = cls;
    if (C <= 2) {
      // closed form of Algorithm 2 with ident weights on one or two vertices:
      // the other class's sources (its reach sum) to the targets hung
      // strictly below each member
      if (C == 2) {
        for (int32_t v = 0; v < np; ++v) {
          const int32_t c = cls[v], o = 1 - c;
          if (rlo[c] == rhi[c]) continue;
          member_extra[v] += (double)rsum[o] * (double)(p.reach[v] - 1);
        }
        for (int32_t c = 0; c < 2; ++c) {
          if (rlo[c] != rhi[c]) continue;
          const int32_t o = 1 - c;
          if (rlo[o] == rhi[o]) {
            const double ko = q.ident[o], ro = (double)rlo[o];
            q.corr[c] += ko * ro * ((double)rlo[c] - 1);
          } else {
            q.corr[c] += (double)rsum[o] * ((double)rlo[c] - 1);
          }
        }
      }
      for (int32_t v = 0; v < np; ++v) bcx[p.verts[v]] += q.corr[cls[v]] + member_extra[v];
      st->tiny_pieces++;
      return;
    }
    for (int32_t v = 0; v < np; ++v)
      if (member_extra[v] != 0.0) bcx[p.verts[v]] += member_extra[v];
    out.push_back(std::move(q));
  }
};

}  // namespace

int preprocess(const HostGraph& g, const std::string& ops, Prepared* P, PrepStats* st, std::string* why) {
  bool opd = false, opa = false, opi = false, opo = false, op_side = false, opu = false;
  for (char c : ops) {
    if (c == 'o') opo = true;
    else if (c == 'd') opd = true;
    else if (c == 'a' || c == 'b') opa = true;
    else if (c == 'i') opi = true;
    else if (c == 'u') opi = opu = true;
    else if (c == 's') op_side = true;
    else {
      *why = std::string("unknown preprocessing letter '") + c + "' (known: o, d, a, b, s, i, u)";
      return SBC_E_INVALID_ARG;
    }
  }
  *st = PrepStats();
  const int32_t n = g.n;
  st->n = n;
  st->m = g.arcs() / 2;
  double t0 = now_ms();

  // Connected components; R (the component size) is conserved by every
  // operation, since each original vertex stays represented exactly once.
  std::vector<int32_t> comp(n, -1);
  std::vector<int64_t> comp_size;
  {
    std::vector<int32_t> q;
    q.reserve(n);
    for (int32_t s = 0; s < n; ++s) {
      if (comp[s] >= 0) continue;
      int32_t c = (int32_t)comp_size.size();
      comp[s] = c;
      q.clear();
      q.push_back(s);
      for (size_t h = 0; h < q.size(); ++h) {
        int32_t v = q[h];
        for (int32_t e = g.row_ptr[v]; e < g.row_ptr[v + 1]; ++e) {
          int32_t w = g.col[e];
          if (comp[w] < 0) {
            comp[w] = c;
            q.push_back(w);
          }
        }
      }
      comp_size.push_back((int64_t)q.size());
    }
  }
  st->components = (int64_t)comp_size.size();

  std::vector<int64_t> r(n, 1);
  std::vector<uint8_t> alive(n, 1);
  std::vector<int32_t> deg(n);
  std::vector<double> bcx(n, 0.0);
  for (int32_t v = 0; v < n; ++v) deg[v] = g.row_ptr[v + 1] - g.row_ptr[v];

  // Degree-1 compression (Section 3.3.1).  Removing u (only neighbour v) is a
  // bridge removal: with S the reach of the rest of the component,
  //   bc[u] += (reach[u]-1) * S          (sources beyond v, targets below u)
  //   bc[v] += (S-1) * reach[u]          (sources below u, targets beyond v)
  //   reach[v] += reach[u].
  if (opd) {
    std::vector<int32_t> q;
    for (int32_t v = 0; v < n; ++v)
      if (deg[v] == 1) q.push_back(v);
    for (size_t h = 0; h < q.size(); ++h) {
      int32_t u = q[h];
      if (!alive[u] || deg[u] != 1) continue;
      int32_t v = -1;
      for (int32_t e = g.row_ptr[u]; e < g.row_ptr[u + 1]; ++e)
        if (alive[g.col[e]]) {
          v = g.col[e];
          break;
        }
      const int64_t R = comp_size[comp[u]];
      const int64_t S = R - r[u];
      bcx[u] += (double)((r[u] - 1) * S);
      bcx[v] += (double)((S - 1) * r[u]);
      r[v] += r[u];
      alive[u] = 0;
      deg[u] = 0;
      st->stripped++;
      if (--deg[v] == 1) q.push_back(v);
    }
  }
  double t1 = now_ms();
  st->ms_degree1 = t1 - t0;

  Builder B(g, opi, op_side, bcx, st);
  B.any_reach = opu;
  std::vector<int32_t> eu, ev;

  if (opa) {
    // Biconnected components of the remaining graph by an iterative
    // Hopcroft-Tarjan depth-first search (Section 3.4).  For a block B and a
    // vertex v of B, the copy of v in B represents every vertex of the
    // component of (G - E(B)) that contains v (Eq. (4)):
    //   - v below the block's top vertex: reach[v] plus the DFS subtrees that
    //     hang off v as separate blocks;
    //   - the top vertex t (entered from the DFS child w): R - W(w), with W the
    //     reach total of a DFS subtree.
    std::vector<int32_t> disc(n, -1), low(n, 0), parent(n, -1), it(n, 0);
    std::vector<int64_t> W(n, 0), hang(n, 0);
    std::vector<int32_t> stk, est_u, est_v;
    int32_t timer = 0;
    for (int32_t root = 0; root < n; ++root) {
      if (!alive[root] || disc[root] >= 0) continue;
      const int64_t R = comp_size[comp[root]];
      disc[root] = low[root] = timer++;
      W[root] = hang[root] = r[root];
      it[root] = g.row_ptr[root];
      stk.push_back(root);
      while (!stk.empty()) {
        int32_t v = stk.back();
        if (it[v] < g.row_ptr[v + 1]) {
          int32_t w = g.col[it[v]++];
          if (!alive[w]) continue;
          if (disc[w] < 0) {
            parent[w] = v;
            disc[w] = low[w] = timer++;
            W[w] = hang[w] = r[w];
            it[w] = g.row_ptr[w];
            est_u.push_back(v);
            est_v.push_back(w);
            stk.push_back(w);
          } else if (w != parent[v] && disc[w] < disc[v]) {
            low[v] = std::min(low[v], disc[w]);
            est_u.push_back(v);
            est_v.push_back(w);
          }
        } else {
          stk.pop_back();
          if (v == root) break;
          int32_t p = parent[v];
          low[p] = std::min(low[p], low[v]);
          W[p] += W[v];
          if (low[v] >= disc[p]) {
            // p is the top of a block whose edges sit on the edge stack down to (p, v)
            st->blocks++;
            hang[p] += W[v];
            eu.clear();
            ev.clear();
            while (true) {
              int32_t a = est_u.back(), b = est_v.back();
              est_u.pop_back();
              est_v.pop_back();
              eu.push_back(a);
              ev.push_back(b);
              if (a == p && b == v) break;
            }
            if (eu.size() == 1) {
              // two-vertex block (a bridge): Algorithm 2 on it in closed form
              const double rp = (double)(R - W[v]), rv = (double)hang[v];
              bcx[p] += rv * (rp - 1);
              bcx[v] += rp * (rv - 1);
              st->bridges++;
              continue;
            }
            RawPiece piece;
            // vertex set of the block: endpoints of its edges
            for (size_t i = 0; i < eu.size(); ++i)
              for (int32_t x : {eu[i], ev[i]})
                if (B.loc[x] < 0) {
                  B.loc[x] = (int32_t)piece.verts.size();
                  piece.verts.push_back(x);
                }
            for (int32_t x : piece.verts) B.loc[x] = -1;
            std::sort(piece.verts.begin(), piece.verts.end());
            piece.reach.resize(piece.verts.size());
            for (size_t i = 0; i < piece.verts.size(); ++i) {
              int32_t x = piece.verts[i];
              piece.reach[i] = (x == p) ? (R - W[v]) : hang[x];
            }
            B.build_local(piece, eu, ev);
            B.finish_piece(piece);
          }
        }
      }
    }
  } else {
    // No shattering: each connected component of what is left is one piece.
    std::vector<int32_t> seen(n, 0), q;
    for (int32_t s = 0; s < n; ++s) {
      if (!alive[s] || seen[s]) continue;
      q.clear();
      q.push_back(s);
      seen[s] = 1;
      eu.clear();
      ev.clear();
      for (size_t h = 0; h < q.size(); ++h) {
        int32_t v = q[h];
        for (int32_t e = g.row_ptr[v]; e < g.row_ptr[v + 1]; ++e) {
          int32_t w = g.col[e];
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
      if (q.size() < 2) continue;  // isolated vertex: bc is whatever stripping gave it
      RawPiece piece;
      piece.verts = q;
      std::sort(piece.verts.begin(), piece.verts.end());
      piece.reach.resize(q.size());
      for (size_t i = 0; i < q.size(); ++i) piece.reach[i] = r[piece.verts[i]];
      B.build_local(piece, eu, ev);
      B.finish_piece(piece);
    }
  }
  double t2 = now_ms();
  st->ms_twins = B.ms_twins;
  st->ms_shatter = t2 - t1 - B.ms_twins;

  // Pack device pieces, largest first.
  std::vector<int32_t> order(B.out.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return B.out[a].ident.size() > B.out[b].ident.size(); });
  Prepared Q;
  Q.n = n;
  Q.vtx_off.push_back(0);
  Q.row.push_back(0);
  int64_t V = 0, A = 0;
  for (int32_t idx : order) {
    V += (int64_t)B.out[idx].ident.size();
    A += (int64_t)B.out[idx].cl.size();
  }
  if (V >= INT32_MAX || A >= INT32_MAX) {
    *why = "packed pieces exceed 2^31 vertices or arcs";
    return SBC_E_TOO_LARGE;
  }
  Q.row.reserve(V + 1);
  Q.col.reserve(A);
  Q.reach.reserve(V);
  Q.ident.reserve(V);
  Q.corr.reserve(V);
  std::vector<int32_t> cnt(n, 0);
  for (int32_t idx : order)
    for (int32_t x : B.out[idx].member_orig) cnt[x]++;
  Q.map_off.assign(n + 1, 0);
  for (int32_t v = 0; v < n; ++v) Q.map_off[v + 1] = Q.map_off[v] + cnt[v];
  Q.map_idx.assign(Q.map_off[n], 0);
  std::vector<int32_t> fill(Q.map_off.begin(), Q.map_off.end() - 1);
  for (int32_t idx : order) {
    const OutPiece& q = B.out[idx];
    const int32_t base = (int32_t)Q.reach.size();
    const int32_t C = (int32_t)q.ident.size();
    const int32_t abase = (int32_t)Q.col.size();
    for (int32_t c = 0; c < C; ++c) Q.row.push_back(abase + q.rp[c + 1]);
    Q.col.insert(Q.col.end(), q.cl.begin(), q.cl.end());
    Q.reach.insert(Q.reach.end(), q.reach.begin(), q.reach.end());
    Q.ident.insert(Q.ident.end(), q.ident.begin(), q.ident.end());
    Q.corr.insert(Q.corr.end(), q.corr.begin(), q.corr.end());
    for (size_t i = 0; i < q.member_orig.size(); ++i)
      Q.map_idx[fill[q.member_orig[i]]++] = base + q.member_cls[i];
    Q.vtx_off.push_back(base + C);
    Q.nside.push_back(q.nside);
    st->pieces++;
    st->piece_vertices += C;
    st->piece_arcs += (int64_t)q.cl.size();
    st->work_teps += (double)(q.nside > 0 ? q.nside : C) * (double)q.cl.size() * 0.5;
    for (int32_t c = 0; c < C; ++c) {
      if (q.reach[c] > q.ident[c]) Q.weighted = true;  // some member hangs more than itself
      if (q.ident[c] > 1) Q.has_ident = true;
    }
  }
  Q.bcx = std::move(bcx);
  Q.src_order.resize(V);
  for (int32_t p = 0; p < Q.pieces(); ++p)
    for (int32_t i = Q.vtx_off[p]; i < Q.vtx_off[p + 1]; ++i) Q.src_order[i] = i - Q.vtx_off[p];
  if (opo) order_pieces(&Q);
  st->ms_pack = now_ms() - t2;
  *P = std::move(Q);
  return SBC_OK;
}

void order_pieces(Prepared* P) {
  const int32_t np_total = P->pieces();
  const int64_t V = P->V();
  std::vector<int32_t> newid(V);  // global old piece vertex -> global new piece vertex
  std::vector<int32_t> order, seen;
  std::vector<int32_t> row2(V + 1), col2(P->col.size()), reach2(V), ident2(V), src2(V);
  std::vector<double> corr2(V);
  row2[0] = 0;
  for (int32_t p = 0; p < np_total; ++p) {
    const int32_t vb = P->vtx_off[p], np = P->vtx_off[p + 1] - vb;
    order.clear();
    seen.assign(np, 0);
    if (!P->nside.empty() && P->nside[p] > 0) {
      // a side piece keeps its ids: its side vertices are 0..nside-1 in removal order
      for (int32_t v = 0; v < np; ++v) order.push_back(v);
      std::fill(seen.begin(), seen.end(), 1);
    }
    int32_t start = 0;
    for (int32_t v = 1; v < np; ++v)
      if (P->row[vb + v + 1] - P->row[vb + v] > P->row[vb + start + 1] - P->row[vb + start]) start = v;
    for (int32_t root = start, scan = 0; (int32_t)order.size() < np;) {
      if (seen[root]) {
        while (scan < np && seen[scan]) ++scan;
        root = scan;
        continue;
      }
      seen[root] = 1;
      size_t h = order.size();
      order.push_back(root);
      for (; h < order.size(); ++h) {
        const int32_t v = order[h];
        for (int32_t e = P->row[vb + v]; e < P->row[vb + v + 1]; ++e) {
          const int32_t w = P->col[e];
          if (!seen[w]) {
            seen[w] = 1;
            order.push_back(w);
          }
        }
      }
    }
    for (int32_t i = 0; i < np; ++i) newid[vb + order[i]] = vb + i;
    for (int32_t i = 0; i < np; ++i) {
      const int32_t old = vb + order[i];
      const int32_t deg = P->row[old + 1] - P->row[old];
      const int32_t out = row2[vb + i];
      for (int32_t k = 0; k < deg; ++k) col2[out + k] = newid[vb + P->col[P->row[old] + k]] - vb;
      std::sort(col2.begin() + out, col2.begin() + out + deg);
      row2[vb + i + 1] = out + deg;
      reach2[vb + i] = P->reach[old];
      ident2[vb + i] = P->ident[old];
      corr2[vb + i] = P->corr[old];
      src2[vb + i] = i;
    }
  }
  for (auto& x : P->map_idx) x = newid[x];
  P->row.swap(row2);
  P->col.swap(col2);
  P->reach.swap(reach2);
  P->ident.swap(ident2);
  P->corr.swap(corr2);
  P->src_order.swap(src2);
}

void cluster_sources(Prepared* P, int group, int mode) {
  // Mode 1: greedy balls: from the lowest unassigned vertex, breadth-first
  // search over unassigned vertices until `group` are collected; then start a
  // new ball.  Mode 2 first groups every vertex whose highest-degree
  // neighbour (itself included) has degree >= kHubDegree by that hub, hubs in
  // id order, so that a batch's sources are all within one hop of a common
  // vertex; the remaining vertices form balls as in mode 1.
  constexpr int32_t kHubDegree = 32;
  const int32_t np_total = P->pieces();
  std::vector<int32_t> q, hub, idx;
  std::vector<uint8_t> used;
  std::vector<int32_t> mark;
  for (int32_t p = 0; p < np_total; ++p) {
    const int32_t vb = P->vtx_off[p], np = P->vtx_off[p + 1] - vb;
    if (!P->nside.empty() && P->nside[p] > 0) {  // side piece: its sources are 0..nside-1
      for (int32_t v = 0; v < np; ++v) P->src_order[vb + v] = v;
      continue;
    }
    used.assign(np, 0);
    mark.assign(np, -1);
    int32_t out = 0;
    if (mode == 2) {
      auto deg = [&](int32_t v) { return P->row[vb + v + 1] - P->row[vb + v]; };
      hub.assign(np, -1);
      idx.clear();
      for (int32_t v = 0; v < np; ++v) {
        int32_t best = v;
        for (int32_t e = P->row[vb + v]; e < P->row[vb + v + 1]; ++e) {
          const int32_t w = P->col[e];
          if (deg(w) > deg(best) || (deg(w) == deg(best) && w < best)) best = w;
        }
        if (deg(best) >= kHubDegree) {
          hub[v] = best;
          idx.push_back(v);
        }
      }
      std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return hub[a] < hub[b]; });
      for (int32_t v : idx) {
        used[v] = 1;
        P->src_order[vb + out++] = v;
      }
    }
    int32_t next_seed = 0, ball = 0;
    while (out < np) {
      while (used[next_seed]) ++next_seed;
      q.clear();
      q.push_back(next_seed);
      mark[next_seed] = ball;
      int32_t taken = 0;
      for (size_t h = 0; h < q.size() && taken < group; ++h) {
        int32_t v = q[h];
        used[v] = 1;
        P->src_order[vb + out++] = v;
        ++taken;
        for (int32_t e = P->row[vb + v]; e < P->row[vb + v + 1]; ++e) {
          int32_t w = P->col[e];
          if (!used[w] && mark[w] != ball) {
            mark[w] = ball;
            q.push_back(w);
          }
        }
      }
      ++ball;
    }
  }
}

}  // namespace sbc
