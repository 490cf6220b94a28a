// Host-side graph container and preprocessing (shattering and compression).
//
// The preprocessing follows Section 3 of the paper: degree-1 stripping
// (Section 3.3.1), shattering at articulation vertices with bridges treated as
// two-vertex blocks (Sections 3.2.1, 3.2.2, 3.4), and identical-vertex merging
// (Section 3.3.3), each keeping the reach / ident bookkeeping that lets the
// per-piece traversal (Algorithm 2 with ident weights) reproduce Eq. (1).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace sbc {

struct HostGraph {
  int32_t n = 0;
  std::vector<int32_t> row_ptr;  // n+1
  std::vector<int32_t> col;      // row_ptr[n], rows sorted ascending
  int64_t arcs() const { return row_ptr.empty() ? 0 : row_ptr[n]; }
};

// Validation result codes match the public status codes.
int validate_csr(int32_t n, const int32_t* row_ptr, const int32_t* col, bool sanitize, HostGraph* out,
                 std::string* why);

struct PrepStats {
  int64_t n = 0, m = 0;
  int64_t components = 0;
  int64_t stripped = 0;        // degree-1 vertices removed
  int64_t blocks = 0;          // biconnected components found
  int64_t bridges = 0;         // two-vertex blocks closed in form on the host
  int64_t twin_classes = 0;    // classes with >= 2 members
  int64_t twins_merged = 0;    // vertices removed by merging (sum of k-1)
  int64_t tiny_pieces = 0;     // pieces of <= 2 vertices after merging, closed in form
  int64_t side_vertices = 0;   // side vertices removed (Section 3.3.2)
  int64_t side_pieces = 0;     // pieces that carry Algorithm 3 searches
  int64_t pieces = 0;          // pieces left for the device
  int64_t piece_vertices = 0;  // sum of n_p over device pieces
  int64_t piece_arcs = 0;      // sum of arcs over device pieces
  double work_teps = 0;        // sum over device pieces of n_p * m_p (sources x edges)
  double ms_degree1 = 0, ms_shatter = 0, ms_twins = 0, ms_pack = 0;
};

// The prepared problem: pieces in a packed CSR (local vertex ids per piece),
// per-piece-vertex attributes, and the data that maps piece scores back to
// the original vertices (Eq. (5)).
struct Prepared {
  int32_t n = 0;                 // original vertex count
  bool weighted = false;         // reach used (any piece vertex with reach > 1)
  bool has_ident = false;        // ident used (any piece vertex with ident > 1)
  std::vector<int32_t> vtx_off;  // P+1: piece p owns global piece vertices [vtx_off[p], vtx_off[p+1])
  std::vector<int32_t> row;      // V+1: absolute arc offsets into col
  std::vector<int32_t> col;      // A: local (piece-relative) neighbour ids
  std::vector<int32_t> reach;    // V: reach of the piece vertex's members together (their sum)
  std::vector<int32_t> ident;    // V: members (identical vertices merged into the piece vertex)
  std::vector<double> corr;      // V: per-member terms added to bc' of each piece vertex
  std::vector<double> bcx;       // n: per-original-vertex terms closed in form on the host
  std::vector<int32_t> map_off;  // n+1: original v maps to piece vertices map_idx[map_off[v]..]
  std::vector<int32_t> map_idx;  // global piece vertex ids
  std::vector<int32_t> src_order;  // V: per piece, local source order (clustered for batching)
  // Per piece: 0 for a piece of Algorithm 2, or k > 0 for a side piece -- a
  // block as it was before its k side vertices were removed, those vertices
  // being local ids 0..k-1 in removal order; its only sources are those k
  // vertices, each running Algorithm 3 with the vertices removed before it
  // left out (Section 3.3.2).
  std::vector<int32_t> nside;
  int32_t pieces() const { return vtx_off.empty() ? 0 : (int32_t)vtx_off.size() - 1; }
  int64_t V() const { return vtx_off.empty() ? 0 : vtx_off.back(); }
  int64_t A() const { return col.size(); }
};

// ops: any of 'd' (degree-1), 'a' (articulation / biconnected shattering),
// 's' (side vertices), 'i' (identical vertices of equal reach), 'u'
// (identical vertices whatever their reach), applied in that order.  ""
// keeps each connected component whole.
int preprocess(const HostGraph& g, const std::string& ops, Prepared* out, PrepStats* st, std::string* why);

// The plain problem: the whole graph as one piece, no attributes.
void plain_problem(const HostGraph& g, Prepared* out);

// Source order inside each piece, so that the sources of one multi-source
// batch lie close together: mode 1, greedy breadth-first balls of `group`
// vertices; mode 2, vertices grouped by a common high-degree neighbour first
// (few distinct distances to any vertex), then balls for the rest.
void cluster_sources(Prepared* p, int group, int mode);

// Vertex ordering of Section 4.1 ("o"), per piece: local ids are renumbered
// in breadth-first order from the piece's highest-degree vertex, so that a
// traversal touches nearby rows and the most-used (hub) rows sit together.
// Rows, attributes, per-member terms and the map back to the original graph
// are permuted consistently.
void order_pieces(Prepared* p);

}  // namespace sbc
