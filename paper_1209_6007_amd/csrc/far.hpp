// Farness and closeness on the shattered graph.
//
// The paper builds its shattering and compression for betweenness and names
// closeness as the next measure to carry them to (Sections 1 and 5) without
// formulas.  The host side here prepares the pieces and puts the per-piece
// sums back together:
//
//  * degree-1 stripping (Section 3.3.1): each removed vertex u hands its
//    subtree to its neighbour v, whose reach grows by reach[u] and whose
//    hung-tree distance sum h grows by h[u] + reach[u];
//  * shattering at articulation vertices (Section 3.2.1, bridges as
//    two-vertex blocks, Section 3.2.2): the copy of v in block B stands for
//    the component of G - E(B) that contains v, reach as for betweenness.
//
// For a block B with copies of reach R_B(w), and any v in B:
//   farness(v) = W_B(v) + sum over w in B of H_B(w),
//   W_B(v) = sum over w in B of R_B(w) * d_B(v, w)   (the device's part),
// where H_B(w) is the distance sum from w over what its copy stands for.
// Going down the block-cut tree (blocks closed by the depth-first search
// before their parents), with top(B) the vertex through which B hangs:
//   down(B) = sum over x in B, x != top(B) of acc(x),
//   acc(x)  = h(x) + sum over blocks B' with top(B') = x of W_B'(x) + down(B'),
// the search root r has farness acc(r), and for v in B below top t
//   farness(v) = W_B(v) + farness(t) - W_B(t).
// A stripped vertex u with neighbour v and subtree size s in a component of
// R vertices has farness(u) = farness(v) + R - 2 s.  All of it is exact in
// int64 (a component of R < 2^31 vertices keeps every sum below R^2 < 2^62).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "prep.hpp"

namespace sbc {

// A block of the stripped graph, in the order the search closed it.
struct FarBlock {
  int32_t top = -1;        // vertex the block hangs from (-1: a whole component, not shattered)
  int32_t piece = -1;      // device piece, or -1 for a two-vertex block
  int32_t top_local = -1;  // local id of `top` in the piece
  int32_t a = -1, b = -1;  // two-vertex block: its vertices (a == top)
  int64_t ra = 0, rb = 0;  // and the reach of their copies
};

struct FarPrepared {
  int32_t n = 0;
  bool weighted = false;          // some piece vertex has reach > 1
  // device pieces: packed CSR, local ids, reach and original id per piece vertex
  std::vector<int32_t> vtx_off, row, col, reach, orig;
  // per piece, the order its vertices run as sources: vertices around a
  // common hub first, then breadth-first balls, so that a 64-source item's
  // sources are close together and reach each vertex at few distinct levels
  std::vector<int32_t> src_order;
  std::vector<FarBlock> blocks;
  std::vector<int32_t> comp;      // n: connected component
  std::vector<int64_t> comp_size;
  std::vector<int64_t> h;         // n: distance sum over each vertex's stripped subtree
  std::vector<int32_t> strip_u, strip_v;  // in removal order: vertex and its neighbour
  std::vector<int64_t> strip_size;        // and its subtree size then
  std::vector<int32_t> roots;     // one vertex per component of the stripped graph
  int64_t stripped = 0, nblocks = 0, bridges = 0;
  double ms_prep = 0;
  int32_t pieces() const { return vtx_off.empty() ? 0 : (int32_t)vtx_off.size() - 1; }
  int64_t V() const { return vtx_off.empty() ? 0 : vtx_off.back(); }
  int64_t A() const { return (int64_t)col.size(); }
};

// ops: any of 'o' (breadth-first vertex order per piece, Section 4.1), 'd'
// (degree-1 stripping), 'a' (articulation shattering); "" keeps every
// component whole.  Returns a status code.
int far_prepare(const HostGraph& g, const std::string& ops, FarPrepared* out, std::string* why);

// Puts the per-piece sums W (one per packed piece vertex) together into the
// farness of every original vertex and, when `closeness` is not null,
// (component size - 1) / farness (0 where the farness is 0).
int far_finish(const FarPrepared& F, const int64_t* W, int64_t* farness, double* closeness, std::string* why);

}  // namespace sbc
