// Traversal kernels for gfx950 (CDNA4, wave64).
//
// Every kernel computes, for the sources of one piece, Algorithm 2 of the
// paper (Bc-Reach, Section 3.2.1) with the identical-vertex weights of
// Section 3.3.3:
//   forward   d[s]=0, sigma[s]=1; for a vertex w first reached at level l,
//             sigma[w] = sum over neighbours v at level l-1 of
//             sigma[v] * (v == s ? 1 : ident[v])
//   backward  delta[v] = (reach[v]-1)
//                        + sigma[v] * sum over neighbours w at level d[v]+1 of
//                          ident[w] * (1 + delta[w]) / sigma[w]
//             (Eq. (3) in pull form: the stack of Algorithm 1 becomes a
//             deepest-level-first sweep and the predecessor lists become a
//             level test on the neighbours)
//   accumulate bc'[v] += ident[s] * reach[s] * delta[v] for v != s.
// The backward coefficient ident[w]*(1+delta[w])/sigma[w] overwrites
// sigma[w]: once delta[w] is known no one needs sigma[w] again.
//
// Kernels are persistent: a grid of resident workgroups drains a device work
// queue with an atomic counter, so thousands of uneven items share one launch.
//
// This header holds only device code.  It is compiled for gfx950 by
// kernels.hip; SBC_DYNAMIC_LDS(name) must be defined by the includer to
// declare the dynamic LDS array.
#pragma once

#include <cfloat>
#include <cstdint>

#include "kernel_types.hpp"

#ifndef SBC_KERNEL_BOUNDS
#define SBC_KERNEL_BOUNDS(block, eu) \
  __attribute__((amdgpu_flat_work_group_size(1, block), amdgpu_waves_per_eu((eu) > 0 ? (eu) : 1)))
#endif

namespace sbc {
namespace dev {

__device__ __forceinline__ void raise_flag(int32_t* flags, int32_t bit) {
  __hip_atomic_fetch_or(flags, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Load of a value that another wave produced with an atomic (atomics execute
// in L2): an agent-scope atomic load cannot be served from a stale per-CU L1
// line.  On LDS it is an ordinary LDS read.
template <typename T>
__device__ __forceinline__ T coherent_load(T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Load of a value that a wave of the same workgroup produced (with an atomic
// or a plain store) before a workgroup barrier.  The waves of a workgroup share
// one CU and its L1, so workgroup scope suffices; unlike an agent-scope load it
// carries no cache-bypass bits and can hit in L2.
#ifndef SBC_MASK_SCOPE
#define SBC_MASK_SCOPE __HIP_MEMORY_SCOPE_WORKGROUP
#endif
template <typename T>
__device__ __forceinline__ T group_load(T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, SBC_MASK_SCOPE);
}

// Neighbour rows loaded together by one wave in the pull loops.
#ifndef SBC_PULL_UNROLL
#define SBC_PULL_UNROLL 4
#endif
constexpr int kPullUnroll = SBC_PULL_UNROLL;
static_assert(kPullUnroll >= 1 && (kPullUnroll & (kPullUnroll - 1)) == 0, "power of two");

// Loads of sigma / coefficient rows and of adjacency: optionally streaming
// (non-temporal), so that they do not push the per-vertex masks out of L2.
#ifndef SBC_STREAM_ROWS
#define SBC_STREAM_ROWS 0
#endif
#ifndef SBC_STREAM_COL
#define SBC_STREAM_COL 0
#endif
template <typename T>
__device__ __forceinline__ T row_load(const T* p) {
#if SBC_STREAM_ROWS
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}
template <typename T>
__device__ __forceinline__ T col_load(const T* p) {
#if SBC_STREAM_COL
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int k) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, k);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), k);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

__device__ __forceinline__ int wave_incl_scan(int x, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// Exclusive scan over the block; returns the thread's prefix and the block total.
// Contains two barriers; s_wtot holds one int per wave.
template <int BLOCK>
__device__ __forceinline__ int block_excl_scan(int x, int* s_wtot, int* total) {
  constexpr int WAVES = BLOCK / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int incl = wave_incl_scan(x, lane);
  if (lane == 63) s_wtot[wave] = incl;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) {
    const int t = s_wtot[w];
    before += (w < wave) ? t : 0;
    all += t;
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

// Checks shared by the persistent kernels: the item, its piece and its
// source range.  All values are read by every thread from the same address,
// so the verdict is uniform across the workgroup.
__device__ __forceinline__ bool item_ok(const DevPieces& P, const QueueArgs& Q, const WorkItem& W, int64_t cap,
                                        int32_t* vb, int32_t* np) {
  if (W.piece < 0 || W.piece >= P.npieces) {
    if (threadIdx.x == 0) raise_flag(Q.flags, kFlagBadItem);
    return false;
  }
  const int32_t b = P.vtx_off[W.piece], e = P.vtx_off[W.piece + 1];
  if (b < 0 || e < b || e > P.nverts || (int64_t)(e - b) > cap) {
    if (threadIdx.x == 0) raise_flag(Q.flags, kFlagBadPiece);
    return false;
  }
  if (W.s0 < 0 || W.s1 < W.s0 || W.s1 > e - b) {
    if (threadIdx.x == 0) raise_flag(Q.flags, kFlagBadItem);
    return false;
  }
  *vb = b;
  *np = e - b;
  return true;
}

// ---------------------------------------------------------------------------
// 64 sources per workgroup, one per lane of every wavefront.
//
// Per vertex v and lane j the slot keeps sg[v*64+j] (sigma, later the
// backward coefficient) so that the 64 sources' values of one vertex are one
// contiguous 512-byte row: a neighbour visit reads one coalesced row for all
// sources instead of 64 scattered words.  Reachability is tracked with 64-bit
// lane masks (vis, frontier), and the BFS order is a list of (vertex, lanes)
// entries: a vertex appears once for every distinct level its lanes reach it
// at, so the backward sweep visits exactly the (vertex, level) pairs that
// exist.
// ---------------------------------------------------------------------------
constexpr int kHubArcs = kMsHubArcs;  // rows longer than this are split over all waves
constexpr int kSliceArcs = kMsSliceArcs;  // arcs per split slice
constexpr int kHeavyMax = kMsHeavyMax;   // split rows per level

// Sum over the neighbours c of a vertex (arcs [e0, e1)) of sg[c*64+lane] for
// the lanes in need & mk[c] (scaled by ident[c] when `scale` is set).  The
// wave gathers 64 neighbour masks at a time, then visits the neighbours with
// any wanted lane kPullUnroll at a time, so that that many row loads are in
// flight together instead of one after another.
__device__ __forceinline__ double pull_row(const int32_t* __restrict__ col, int32_t e0, int32_t e1, int32_t np,
                                           uint64_t* __restrict__ mk, const uint64_t need,
                                           const double* __restrict__ sg, const int32_t* __restrict__ idn,
                                           const bool scale, const int lane, int32_t* flags) {
  double acc = 0.0;
  for (int32_t eb = e0; eb < e1; eb += 64) {
    const int32_t e = eb + lane;
    int32_t c = 0;
    uint64_t m = 0;
    if (e < e1) {
      c = col_load(&col[e]);
      if (c >= 0 && c < np) {
        m = group_load(&mk[c]) & need;
      } else {
        raise_flag(flags, kFlagBadArc);
        c = 0;
      }
    }
    uint64_t act = __ballot(m != 0);
    while (act) {
      // Up to kPullUnroll neighbours at a time: their row loads are issued
      // together, then summed in a fixed pairwise order.
      double x[kPullUnroll];
#pragma unroll
      for (int j = 0; j < kPullUnroll; ++j) {
        x[j] = 0.0;
        if (act) {  // wave-uniform
          const int k = __builtin_ctzll(act);
          act &= act - 1;
          const int32_t u = __builtin_amdgcn_readlane(c, k);
          const uint64_t mu = readlane64(m, k);
          if ((mu >> lane) & 1) x[j] = row_load(&sg[(size_t)u * 64 + lane]);
          if (scale) x[j] *= (double)idn[u];
        }
      }
#pragma unroll
      for (int w = 1; w < kPullUnroll; w <<= 1)
#pragma unroll
        for (int j = 0; j + w < kPullUnroll; j += 2 * w) x[j] += x[j + w];
      acc += x[0];
    }
  }
  return acc;
}

// Row bounds for a wave-uniform vertex; false (flagged once) when out of range.
__device__ __forceinline__ bool wave_row(const int32_t* __restrict__ rowp, int32_t v, int32_t np, int32_t narcs,
                                         int32_t* e0, int32_t* e1, int32_t* flags, int lane) {
  if (v < 0 || v >= np) {
    if (lane == 0) raise_flag(flags, kFlagBadArc);
    return false;
  }
  *e0 = rowp[v];
  *e1 = rowp[v + 1];
  if (*e0 < 0 || *e1 < *e0 || *e1 > narcs) {
    if (lane == 0) raise_flag(flags, kFlagBadArc);
    return false;
  }
  return true;
}

// Entries one wave pulls together (pull_entries).
#ifndef SBC_PULL_GROUP
#define SBC_PULL_GROUP 1
#endif
constexpr int kGroup = SBC_PULL_GROUP;

// pull_row for G entries whose rows have at most 64 arcs (deg[e] = 0 skips
// entry e): their neighbour ids, then their neighbour masks, then their rows
// are loaded together, so that a wave has G dependent chains in flight instead
// of one.  acc[e] gets the sum for entry e, in a fixed order.
template <int G>
__device__ __forceinline__ void pull_group(const int32_t* __restrict__ col, const int32_t (&e0)[G],
                                           const int32_t (&deg)[G], const int32_t np, uint64_t* __restrict__ mk,
                                           const uint64_t (&need)[G], const double* __restrict__ sg,
                                           const int32_t* __restrict__ idn, const bool scale, const int lane,
                                           int32_t* flags, double (&acc)[G]) {
  int32_t c[G];
  uint64_t m[G], act[G];
#pragma unroll
  for (int e = 0; e < G; ++e) {
    c[e] = -1;
    if (lane < deg[e]) {
      c[e] = col_load(&col[e0[e] + lane]);
      if (c[e] < 0 || c[e] >= np) {
        raise_flag(flags, kFlagBadArc);
        c[e] = -1;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < G; ++e) m[e] = c[e] >= 0 ? group_load(&mk[c[e]]) & need[e] : 0;
  uint64_t any = 0;
#pragma unroll
  for (int e = 0; e < G; ++e) {
    act[e] = __ballot(m[e] != 0);
    any |= act[e];
    acc[e] = 0.0;
  }
  // Rounds: up to kPer neighbours of every entry per round (four rows in
  // flight for a single entry, two per entry for groups).
  constexpr int kPer = G == 1 ? 4 : 2;
  while (any) {  // wave-uniform
    double x[G][kPer];
#pragma unroll
    for (int e = 0; e < G; ++e)
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        x[e][j] = 0.0;
        if (act[e]) {  // wave-uniform
          const int k = __builtin_ctzll(act[e]);
          act[e] &= act[e] - 1;
          const int32_t u = __builtin_amdgcn_readlane(c[e], k);
          const uint64_t mu = readlane64(m[e], k);
          if ((mu >> lane) & 1) x[e][j] = row_load(&sg[(size_t)u * 64 + lane]);
          if (scale) x[e][j] *= (double)idn[u];
        }
      }
    any = 0;
#pragma unroll
    for (int e = 0; e < G; ++e) {
      double r = 0.0;
#pragma unroll
      for (int j = 0; j < kPer; j += 2) r += x[e][j] + x[e][j + 1];
      acc[e] += r;
      any |= act[e];
    }
  }
}

// ---------------------------------------------------------------------------
// Compact value layout (batch kernel).  Deep and sparse pieces give a batch
// many (vertex, level) entries per vertex with a few lanes each; in 64-lane
// rows every such lane's value costs its own memory sector.  In the compact
// layout entry e's values lie together, lane j of mask m at
// eoff[e] + lane_rank(m, j), and a neighbour u on the level being read is
// found through ob[u], the offset of u's entry on that level.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_rank(uint64_t m, int j) { return __builtin_popcountll(m & ((1ull << j) - 1)); }

// pull_group<1> / pull_row for the compact layout: the neighbour's full
// lane mask and its entry offset are gathered together, and lane j of the
// wave reads value rank_j of the neighbour's entry.
// The sum continues from acc in the order pull_group and pull_row use (four
// neighbours' values added pairwise, then to the running sum), so both
// layouts give the same bits.
__device__ __forceinline__ double pull_short_c(const int32_t* __restrict__ col, int32_t e0, int32_t deg, int32_t np,
                                               uint64_t* __restrict__ mk, const int32_t* __restrict__ ob,
                                               const uint64_t need, const double* __restrict__ sg,
                                               const int32_t* __restrict__ idn, const bool scale, const int lane,
                                               int32_t* flags, double acc) {
  int32_t c = -1, o = 0;
  uint64_t mf = 0;
  if (lane < deg) {
    c = col_load(&col[e0 + lane]);
    if (c < 0 || c >= np) {
      raise_flag(flags, kFlagBadArc);
      c = -1;
    } else {
      mf = group_load(&mk[c]);
      o = ob[c];
    }
  }
  uint64_t act = __ballot((mf & need) != 0);
  constexpr int kPer = 4;  // rows in flight
  static_assert(kPer == kPullUnroll, "the row layout's pull adds four at a time");
  while (act) {  // wave-uniform
    double x[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      x[j] = 0.0;
      if (act) {  // wave-uniform
        const int k = __builtin_ctzll(act);
        act &= act - 1;
        const int32_t u = __builtin_amdgcn_readlane(c, k);
        const uint64_t mu = readlane64(mf, k);
        const int32_t ou = __builtin_amdgcn_readlane(o, k);
        if (((mu & need) >> lane) & 1) x[j] = row_load(&sg[(size_t)ou + lane_rank(mu, lane)]);
        if (scale) x[j] *= (double)idn[u];
      }
    }
    acc += (x[0] + x[1]) + (x[2] + x[3]);
  }
  return acc;
}

__device__ __forceinline__ double pull_row_c(const int32_t* __restrict__ col, int32_t e0, int32_t e1, int32_t np,
                                             uint64_t* __restrict__ mk, const int32_t* __restrict__ ob,
                                             const uint64_t need, const double* __restrict__ sg,
                                             const int32_t* __restrict__ idn, const bool scale, const int lane,
                                             int32_t* flags) {
  double acc = 0.0;
  for (int32_t eb = e0; eb < e1; eb += 64)
    acc = pull_short_c(col, eb, min(64, e1 - eb), np, mk, ob, need, sg, idn, scale, lane, flags, acc);
  return acc;
}

// pair_sum for the compact layout.  With U > 1 the arcs go U at a time:
// their neighbour ids, then masks and entry offsets, then values are loaded
// together, so a lane waits for three round trips per U arcs instead of per
// arc.  The values are added one by one in arc order, as with U = 1, so the
// bits do not depend on U.
template <int U>
__device__ __forceinline__ double pair_sum_c(const int32_t* __restrict__ col, int32_t e0, int32_t e1, int32_t np,
                                             uint64_t* __restrict__ mk, const int32_t* __restrict__ ob,
                                             const double* __restrict__ sg, const int32_t* __restrict__ idn,
                                             bool scale, int j, int32_t* flags) {
  double acc = 0.0;
  for (int32_t e = e0; e < e1; e += U) {
    int32_t u[U], o[U];
    uint64_t m[U];
    double x[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      u[k] = -1;
      if (e + k < e1) {
        u[k] = col_load(&col[e + k]);
        if (u[k] < 0 || u[k] >= np) {
          raise_flag(flags, kFlagBadArc);
          u[k] = -1;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      m[k] = 0;
      o[k] = 0;
      if (u[k] >= 0) {
        m[k] = group_load(&mk[u[k]]);
        o[k] = ob[u[k]];
      }
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      x[k] = 0.0;
      if ((m[k] >> j) & 1) {
        x[k] = row_load(&sg[(size_t)o[k] + lane_rank(m[k], j)]);
        if (scale) x[k] *= (double)idn[u[k]];
      }
    }
#pragma unroll
    for (int k = 0; k < U; ++k)
      if ((m[k] >> j) & 1) acc += x[k];
  }
  return acc;
}

// One wave's pull of the entries [i0, min(i0 + G, iend)) of the queue q.
// need_of(i, v) gives an entry's lanes; defer(i, v, e0, e1, need) takes a row
// the caller splits over many waves and returns true (it must be
// wave-uniform); early(i, v, need) issues, before the pull, the loads that
// finish needs; finish(i, v, need, acc, early's result) consumes each other
// entry's sum.  Rows of at most 64 arcs go through pull_group together,
// longer ones through pull_row one by one.
template <int G, typename NeedOf, typename Defer, typename Early, typename Finish>
__device__ __forceinline__ void pull_entries(const int i0, const int iend, const int32_t* __restrict__ q,
                                             const int32_t* __restrict__ rowp, const int32_t np, const int32_t narcs,
                                             const int32_t* __restrict__ col, uint64_t* __restrict__ mk,
                                             const double* __restrict__ sg, const int32_t* __restrict__ idn,
                                             const bool scale, const int lane, int32_t* flags, NeedOf need_of,
                                             Defer defer, Early early, Finish finish) {
  int32_t v[G], e0[G], e1[G], dg[G];
  uint64_t need[G];
  bool live[G];
  decltype(early(0, 0, 0ull)) pre[G];
#pragma unroll
  for (int e = 0; e < G; ++e) {
    live[e] = false;
    v[e] = 0;
    e0[e] = 0;
    e1[e] = 0;
    need[e] = 0;
    const int i = i0 + e;
    if (i < iend) {
      v[e] = q[i];
      if (wave_row(rowp, v[e], np, narcs, &e0[e], &e1[e], flags, lane)) {
        need[e] = need_of(i, v[e]);
        live[e] = !defer(i, v[e], e0[e], e1[e], need[e]);
        if (live[e]) pre[e] = early(i, v[e], need[e]);
      }
    }
    dg[e] = (live[e] && e1[e] - e0[e] <= 64) ? e1[e] - e0[e] : 0;
  }
  double acc[G];
  pull_group<G>(col, e0, dg, np, mk, need, sg, idn, scale, lane, flags, acc);
#pragma unroll
  for (int e = 0; e < G; ++e)
    if (live[e] && e1[e] - e0[e] > 64) acc[e] = pull_row(col, e0[e], e1[e], np, mk, need[e], sg, idn, scale, lane, flags);
#pragma unroll
  for (int e = 0; e < G; ++e)
    if (live[e]) finish(i0 + e, v[e], need[e], acc[e], pre[e]);
}

#ifndef SBC_XCD_FENCES
// This wave's stores and atomics have reached L2.
__device__ __forceinline__ void xcd_release() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// Hardware id of the XCD this wave runs on.
__device__ __forceinline__ int xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15; }
// Lanes of one wave see each other's LDS writes made before this point.
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }
#endif


// One wave's LDS slots for pull_list: vertex, row bounds and lanes of up to
// 64 entries, and for the pair path each entry's first pair and its per-entry
// sum.
struct EntrySlots {
  int32_t* v;
  int32_t* e0;
  int32_t* e1;
  uint64_t* need;
  int32_t* poff;
  double* pacc;
};

// Pair path of pull_list: an entry whose row has at most kPairMaxDeg arcs and
// whose lanes number at most `pairs` is pulled as (entry, lane) pairs,
// one pair per lane, instead of by a whole wave of which only the entry's few
// lanes would load anything.  On deep, sparse pieces the sources of a batch
// reach a vertex at many different levels, so most entries carry a handful of
// lanes: pairs keep every lane of the wave busy and issue the loads of many
// entries at once.
constexpr int kPairMaxDeg = 32;
__device__ __forceinline__ bool pair_entry(int32_t e0, int32_t e1, uint64_t need, int max_lanes) {
  return e1 - e0 <= kPairMaxDeg && __builtin_popcountll(need) <= max_lanes;
}

// One lane's sum over the arcs [e0, e1) of sg[u*64 + j] for the neighbours u
// whose mask mk[u] holds lane j (scaled by ident[u] when `scale`), added in
// arc order.  With U > 1 the arcs go U at a time (their neighbour ids, then
// masks, then values loaded together); on MI355X U = 1 measured as fast on a
// deep grid and faster on the block tree (fewer registers).
template <int U>
__device__ __forceinline__ double pair_sum(const int32_t* __restrict__ col, int32_t e0, int32_t e1, int32_t np,
                                           uint64_t* __restrict__ mk, const double* __restrict__ sg,
                                           const int32_t* __restrict__ idn, bool scale, int j, int32_t* flags) {
  double acc = 0.0;
  for (int32_t e = e0; e < e1; e += U) {
    int32_t u[U];
    uint64_t m[U];
    double x[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      u[k] = -1;
      if (e + k < e1) {
        u[k] = col_load(&col[e + k]);
        if (u[k] < 0 || u[k] >= np) {
          raise_flag(flags, kFlagBadArc);
          u[k] = -1;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < U; ++k) m[k] = u[k] >= 0 ? group_load(&mk[u[k]]) : 0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
      x[k] = 0.0;
      if ((m[k] >> j) & 1) {
        x[k] = row_load(&sg[(size_t)u[k] * 64 + j]);
        if (scale) x[k] *= (double)idn[u[k]];
      }
    }
#pragma unroll
    for (int k = 0; k < U; ++k) acc += x[k];
  }
  return acc;
}

__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// A work item every lane read alike, in scalar registers (so are the piece
// bounds and pointers derived from it).
__device__ __forceinline__ WorkItem uniform_item(const WorkItem& w) {
  return {__builtin_amdgcn_readfirstlane(w.piece), __builtin_amdgcn_readfirstlane(w.s0),
          __builtin_amdgcn_readfirstlane(w.s1), __builtin_amdgcn_readfirstlane(w.kind)};
}

// One wave's pull of the n <= 64 entries first, first + step, ...,
// first + (n-1)*step of the queue q, with the callbacks of pull_entries and
// early(i, v, need), whose result finish gets as a fifth argument: the loads
// an entry's finish needs are issued before its pull, not after it.
// pull(e0, e1, need) is the wave's sum over the row for the entry's lanes.
// Lane k first gathers entry k's vertex, row bounds and lanes into the
// wave's slots: one round of loads for all n entries, where an entry alone
// costs three dependent rounds (queue slot, then row bounds, then lanes).
// The entries are then pulled one after another; a bad vertex or row is
// flagged and skipped.
//
// With `pairs` > 0, entries that pass pair_entry are instead done first, as
// pairs: the wave's pairs are numbered entry by entry (a scan of the entries'
// lane counts), lane t takes pairs t, t+64, ..., finds its entry by binary
// search and its lane j as the entry's r-th lane, and calls pair(k, i, v, e0,
// e1, j).  Then lane k calls pair_done(k, i, v, need) for each such entry k.
template <typename NeedOf, typename Defer, typename Early, typename Finish, typename Pair, typename PairDone,
          typename Pull>
__device__ __forceinline__ void pull_list(const int first, const int step, const int n, const EntrySlots& sl,
                                          const int32_t* __restrict__ q, const int32_t* __restrict__ rowp,
                                          const int32_t np, const int32_t narcs, const int lane, int32_t* flags,
                                          NeedOf need_of, Defer defer, Early early, Finish finish, const int pairs,
                                          Pair pair, PairDone pair_done, Pull pull) {
  if (lane < n) {
    const int i = first + lane * step;
    int32_t v = q[i], e0 = 0, e1 = 0;
    uint64_t need = 0;
    if (v >= 0 && v < np) {
      e0 = rowp[v];
      e1 = rowp[v + 1];
      if (e0 < 0 || e1 < e0 || e1 > narcs) {
        raise_flag(flags, kFlagBadArc);
        v = -1;
      } else {
        need = need_of(i, v);
      }
    } else {
      raise_flag(flags, kFlagBadArc);
      v = -1;
    }
    sl.v[lane] = v;
    sl.e0[lane] = e0;
    sl.e1[lane] = e1;
    sl.need[lane] = need;
  }
  if (pairs > 0) {  // wave-uniform
    int cnt = 0;
    bool mine = false;
    if (lane < n) {
      const int32_t v = sl.v[lane];
      const uint64_t need = sl.need[lane];
      mine = v >= 0 && pair_entry(sl.e0[lane], sl.e1[lane], need, pairs);
      if (mine) cnt = __builtin_popcountll(need);
    }
    const int incl = wave_incl_scan(cnt, lane);
    const int total = __builtin_amdgcn_readlane(incl, 63);
    sl.poff[lane] = incl - cnt;
    sl.pacc[lane] = 0.0;
    wave_sync();
    for (int t = lane; t < total; t += 64) {
      int lo = 0, hi = n - 1;  // the last entry whose first pair is at most t
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sl.poff[mid] <= t) lo = mid;
        else hi = mid - 1;
      }
      uint64_t m = sl.need[lo];
      for (int r = t - sl.poff[lo]; r > 0; --r) m &= m - 1;
      pair(lo, first + lo * step, sl.v[lo], sl.e0[lo], sl.e1[lo], __builtin_ctzll(m));
    }
    wave_sync();
    if (mine) pair_done(lane, first + lane * step, sl.v[lane], sl.need[lane]);
  } else {
    wave_sync();
  }
  for (int k = 0; k < n; ++k) {
    const int32_t v = __builtin_amdgcn_readfirstlane(sl.v[k]);
    if (v < 0) continue;
    const int i = first + k * step;
    const int32_t e0 = __builtin_amdgcn_readfirstlane(sl.e0[k]);
    const int32_t e1 = __builtin_amdgcn_readfirstlane(sl.e1[k]);
    const uint64_t need = uniform64(sl.need[k]);
    if (pairs > 0 && pair_entry(e0, e1, need, pairs)) continue;  // done as pairs
    if (defer(i, v, e0, e1, need)) continue;
    const auto pre = early(i, v, need);
    const double acc = pull(e0, e1, need);
    finish(i, v, need, acc, pre);
  }
  wave_sync();  // every lane has read the slots before the wave's next list fills them
}

// What the backward finish of entry (v, level) reads besides the pulled sum:
// the lane's sigma of v (lanes outside the entry get 1), reach[v]-1 and
// ident[v].
//
// Piece-vertex attributes: ident[v] members (identical vertices merged into
// one, Section 3.3.3) whose reaches sum to reach[v].  A source's weight is
// that sum (every member's hung vertices are sources alike), and the
// dependency of v starts at the members' mean reach minus one (the targets
// hung below a member): with equal reaches, reach[s] * ident[s] and
// reach[v] - 1 of the per-member form; with unequal ones the host adds each
// member's difference from the mean.
template <bool REACH, bool IDENT>
__device__ __forceinline__ double src_weight(const int32_t* __restrict__ rch, const int32_t* __restrict__ idn,
                                             int32_t s) {
  return REACH ? (double)rch[s] : (IDENT ? (double)idn[s] : 1.0);
}
template <bool REACH, bool IDENT>
__device__ __forceinline__ double reach_m1(const int32_t* __restrict__ rch, const int32_t* __restrict__ idn,
                                           int32_t v) {
  if constexpr (!REACH) return 0.0;
  else if constexpr (IDENT) return (double)rch[v] / (double)idn[v] - 1.0;
  else return (double)(rch[v] - 1);
}

struct BackEarly {
  double sv, rm1, id;
};

// idx: where the lane's value of the entry lies in sg.
template <bool REACH, bool IDENT>
__device__ __forceinline__ BackEarly back_early_at(const double* __restrict__ sg, size_t idx,
                                                   const int32_t* __restrict__ rch, const int32_t* __restrict__ idn,
                                                   int32_t v, uint64_t amask, int lane) {
  BackEarly r;
  r.sv = ((amask >> lane) & 1) ? sg[idx] : 1.0;
  r.rm1 = reach_m1<REACH, IDENT>(rch, idn, v);
  r.id = IDENT ? (double)idn[v] : 1.0;
  return r;
}

template <bool REACH, bool IDENT>
__device__ __forceinline__ BackEarly back_early(const double* __restrict__ sg, const int32_t* __restrict__ rch,
                                                const int32_t* __restrict__ idn, int32_t v, uint64_t amask,
                                                int lane) {
  BackEarly r;
  r.sv = ((amask >> lane) & 1) ? sg[(size_t)v * 64 + lane] : 1.0;
  r.rm1 = reach_m1<REACH, IDENT>(rch, idn, v);
  r.id = IDENT ? (double)idn[v] : 1.0;
  return r;
}

// A lane's contribution of delta dv at vertex v to bc'.  In a side piece
// (srank >= 0: the lane's source, a side vertex, whose id is its removal
// rank) it is Algorithm 3's reach[s]*(delta + (delta - (reach[v]-1))), and a
// side vertex removed before the source (v < srank) is absent from the
// source's graph: it adds nothing and passes nothing back (coefficient 0).
// It is never on a shortest path between other vertices, so the forward
// sweep needs no change.
__device__ __forceinline__ bool side_absent(int32_t v, int32_t srank) { return v < srank; }
__device__ __forceinline__ double side_contrib(double wsrc, double dv, double rm1, int32_t srank) {
  return srank >= 0 ? wsrc * (2.0 * dv - rm1) : wsrc * dv;
}

// Backward finish of entry (v, level) with lanes amask and pulled sum acc:
// delta (Eq. (3) in pull form), the coefficient that replaces sigma, the
// wave's contribution to bc'[v] (weighted by ident[s]*reach[s] in wsrc) and
// the level's backward mask.  drow, when not null, is the lane's row of the
// dependency dump; srank is the lane's side rank (-1 outside side pieces).
__device__ __forceinline__ void back_finish_at(double* __restrict__ sg, size_t idx, double* __restrict__ bcp,
                                               uint64_t* __restrict__ bw, int32_t v, uint64_t amask, double acc,
                                               const BackEarly& pre, double wsrc, int lane, int32_t* flags,
                                               double* drow, int32_t srank) {
  double contrib = 0.0;
  if ((amask >> lane) & 1) {
    const double dv = pre.rm1 + pre.sv * acc;
    if (side_absent(v, srank)) {
      sg[idx] = 0.0;
    } else {
      sg[idx] = pre.id * (1.0 + dv) / pre.sv;
      contrib = side_contrib(wsrc, dv, pre.rm1, srank);
    }
    if (drow) drow[v] = dv;
    if (!(pre.sv <= DBL_MAX) || !(dv <= DBL_MAX)) raise_flag(flags, kFlagSigmaOverflow);
  }
  contrib = wave_sum(contrib);
  if (lane == 0) {
    atomicAdd(&bcp[v], contrib);
    bw[v] = amask;
  }
}

__device__ __forceinline__ void back_finish(double* __restrict__ sg, double* __restrict__ bcp,
                                            uint64_t* __restrict__ bw, int32_t v, uint64_t amask, double acc,
                                            const BackEarly& pre, double wsrc, int lane, int32_t* flags,
                                            double* drow, int32_t srank) {
  double contrib = 0.0;
  if ((amask >> lane) & 1) {
    const double dv = pre.rm1 + pre.sv * acc;
    if (side_absent(v, srank)) {
      sg[(size_t)v * 64 + lane] = 0.0;
    } else {
      sg[(size_t)v * 64 + lane] = pre.id * (1.0 + dv) / pre.sv;
      contrib = side_contrib(wsrc, dv, pre.rm1, srank);
    }
    if (drow) drow[v] = dv;
    if (!(pre.sv <= DBL_MAX) || !(dv <= DBL_MAX)) raise_flag(flags, kFlagSigmaOverflow);
  }
  contrib = wave_sum(contrib);
  if (lane == 0) {
    atomicAdd(&bcp[v], contrib);
    bw[v] = amask;
  }
}

// EU > 0 asks the compiler for at least EU resident waves per SIMD (it then
// keeps the kernel within 512/EU VGPRs); the kernel is latency-bound, so more
// waves in flight can matter more than registers.
// DUMP builds the verification variant: it also writes every source's
// levels, path counts and dependencies to `dump` (null otherwise).
template <int WAVES, int EU, bool REACH, bool IDENT, bool DUMP = false, bool CMP = false>
__global__ SBC_KERNEL_BOUNDS(WAVES * 64, EU) void ms_kernel(DevPieces P, QueueArgs Q, MsState st, DumpOut dump) {
  if (Q.magic != kArgMagic) return;
  constexpr int BLOCK = WAVES * 64;
  // Arcs a pair loads together (compact layout): four where the compiler
  // chooses the register count, one under an occupancy target's budget.
  constexpr int kPairU = EU == 0 ? 4 : 1;
  __shared__ int s_item;
  __shared__ int s_cnt[3];
  __shared__ int s_wtot[WAVES];
  __shared__ int s_scan[BLOCK];
  __shared__ int s_e0[BLOCK];
  __shared__ int s_e1[BLOCK];
  __shared__ uint64_t s_f[BLOCK];
  __shared__ int s_poff[BLOCK];
  __shared__ double s_pacc[BLOCK];
  __shared__ double s_wsrc[64];  // ident[s]*reach[s] of lane s's source (pair path)
  __shared__ int32_t s_srank[64];  // side rank of lane s's source, -1 outside side pieces (pair path)
  __shared__ int s_nheavy, s_nslices;
  __shared__ int s_heavy[kHeavyMax];
  __shared__ int s_hoff[kHeavyMax];

  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: scalar registers
  // The pull phases gather entries in the phase-A scratch arrays (free then).
  const EntrySlots slots{s_scan + wave * 64, s_e0 + wave * 64, s_e1 + wave * 64,
                         s_f + wave * 64,    s_poff + wave * 64, s_pacc + wave * 64};
  const int pairs = st.pairs;
  const size_t slot = blockIdx.x;
  double* sg = st.sg + slot * (size_t)st.stride * 64;
  int32_t* q = st.q + slot * (size_t)st.stride * 64;
  uint64_t* qm = st.qm + slot * (size_t)st.stride * 64;
  uint64_t* vis = st.vis + slot * (size_t)st.stride;
  uint64_t* bufa = st.fa + slot * (size_t)st.stride;
  uint64_t* bufb = st.fb + slot * (size_t)st.stride;
  uint64_t* bme = st.ba + slot * (size_t)st.stride;  // backward masks of even levels
  uint64_t* bmo = st.bb + slot * (size_t)st.stride;  // backward masks of odd levels
  int32_t* lvl = st.lvl + slot * (size_t)(st.stride + 3);
  double* part = st.part + slot * (size_t)st.part_cap * 64;
  const int64_t qcap = st.stride * 64;
  // Compact layout (CMP): per-entry value offsets, and per level parity and
  // vertex the offset of the vertex's entry on the level being read.
  int32_t* eoff = CMP ? st.eoff + slot * (size_t)st.stride * 64 : nullptr;
  int32_t* ob2 = CMP ? st.ob + slot * (size_t)st.stride * 2 : nullptr;
  auto obp = [&](int lev) -> int32_t* { return ob2 + (size_t)(lev & 1) * st.stride; };
  // Where entry i's (vertex v, lanes m) value for lane j lies in sg.
  auto own = [&](int i, int32_t v, uint64_t m, int j) -> size_t {
    if constexpr (CMP) return (size_t)eoff[i] + lane_rank(m, j);
    else return (size_t)v * 64 + j;
  };
  const int32_t narcs = P.narcs;
  // Phase timers: thread 0 charges the wall-clock time since its last mark to
  // one counter of this slot.
  uint64_t* prof = st.prof ? st.prof + slot * kProfCounters : nullptr;
  long long tmark = prof ? wall_clock64() : 0;
  auto mark = [&](int idx) {
    if (prof && tid == 0) {
      const long long now = wall_clock64();
      prof[idx] += (uint64_t)(now - tmark);
      tmark = now;
    }
  };

  while (true) {
    if (tid == 0) s_item = atomicAdd(Q.head, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it < 0 || it >= Q.nitems) break;
    const WorkItem W = uniform_item(Q.items[it]);
    int32_t vb, np;
    const bool item_good = item_ok(P, Q, W, st.stride, &vb, &np) && W.s1 - W.s0 >= 1 && W.s1 - W.s0 <= 64;
    if (!item_good) {
      if (tid == 0) {
        raise_flag(Q.flags, kFlagBadItem);
        atomicAdd(Q.done, 1);
      }
      continue;
    }
    vb = __builtin_amdgcn_readfirstlane(vb);
    np = __builtin_amdgcn_readfirstlane(np);
    const int32_t* rowp = P.row + vb;
    const int32_t* col = P.col;
    const int32_t* rch = REACH ? P.reach + vb : nullptr;
    const int32_t* idn = IDENT ? P.ident + vb : nullptr;
    // the item's own area when deterministic
    double* bcp = Q.item_base ? Q.item_out + (int64_t)uniform64((uint64_t)Q.item_base[it]) : P.bcp + vb;
    const int nsrc = W.s1 - W.s0;  // 1..64

    // Lane j runs source src_order[vb + s0 + j].
    int32_t s = -1;
    if (lane < nsrc) s = P.src_order[vb + W.s0 + lane];
    if (__ballot(lane < nsrc && (s < 0 || s >= np)) != 0) {  // same verdict in every wave
      if (tid == 0) {
        raise_flag(Q.flags, kFlagBadSource);
        atomicAdd(Q.done, 1);
      }
      continue;
    }
    double wsrc = 0.0;
    const bool side_item = P.nside && P.nside[W.piece] > 0;
    const int32_t srank = (side_item && lane < nsrc) ? s : -1;  // Algorithm 3 items: the source's removal rank
    if (lane < nsrc) {
      wsrc = src_weight<REACH, IDENT>(rch, idn, s);
      if (wave == 0) {
        q[lane] = s;
        qm[lane] = 1ull << lane;
        bufa[s] = 1ull << lane;
        vis[s] = 1ull << lane;
        if constexpr (CMP) {  // level 0: entry j holds lane j alone
          eoff[lane] = lane;
          obp(0)[s] = lane;
          sg[lane] = 1.0;
        } else {
          sg[(size_t)s * 64 + lane] = 1.0;
        }
      }
    }
    if (wave == 0) {
      s_wsrc[lane] = wsrc;
      s_srank[lane] = srank;
    }
    if (tid == 0) {
      lvl[0] = 0;
      lvl[1] = nsrc;
      s_cnt[0] = s_cnt[1] = s_cnt[2] = 0;
    }
    __syncthreads();
    mark(kProfFetch);

    uint64_t* fcur = bufa;
    uint64_t* fnxt = bufb;
    int qs = 0, qe = nsrc, L = 0;
    int64_t cbase = nsrc;  // compact layout: values placed so far
    // ---------------- forward sweep ----------------
    while (true) {
      if (tid == 0) {
        s_cnt[(L + 1) % 3] = 0;
        s_nheavy = 0;
        s_nslices = 0;
      }
      // Phase A: discover the (vertex, new lanes) pairs of level L+1 with the
      // arcs of level L spread evenly over the whole workgroup.
      for (int cb = qs; cb < qe; cb += BLOCK) {
        const int i = cb + tid;
        int e0 = 0, deg = 0;
        uint64_t fu = 0;
        if (i < qe) {
          const int32_t u = q[i];
          if (u >= 0 && u < np) {
            e0 = rowp[u];
            const int32_t e1 = rowp[u + 1];
            if (e0 >= 0 && e1 >= e0 && e1 <= narcs) {
              deg = e1 - e0;
              fu = qm[i];
            } else {
              raise_flag(Q.flags, kFlagBadArc);
              e0 = 0;
            }
          } else {
            raise_flag(Q.flags, kFlagBadArc);
          }
        }
        int total;
        const int ex = block_excl_scan<BLOCK>(deg, s_wtot, &total);
        s_scan[tid] = ex;
        s_e0[tid] = e0;
        s_f[tid] = fu;
        __syncthreads();
        const int nv = min(BLOCK, qe - cb);
        for (int t = tid; t < total; t += BLOCK) {
          int lo = 0, hi = nv - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_scan[mid] <= t) lo = mid;
            else hi = mid - 1;
          }
          const int32_t w = col[s_e0[lo] + (t - s_scan[lo])];
          if (w < 0 || w >= np) {
            raise_flag(Q.flags, kFlagBadArc);
            continue;
          }
          const uint64_t nw = s_f[lo] & ~vis[w];
          if (nw) {
            const uint64_t old = atomicOr((unsigned long long*)&fnxt[w], (unsigned long long)nw);
            if (old == 0) {
              const int pos = atomicAdd(&s_cnt[L % 3], 1);
              if (qe + pos < qcap) q[qe + pos] = w;
              else raise_flag(Q.flags, kFlagQueueOverflow);
            }
          }
        }
        __syncthreads();
      }
      const int nt = (int)min((int64_t)(qe + s_cnt[L % 3]), qcap);
      mark(kProfPhaseA);
      if (nt == qe) break;
      if constexpr (CMP) {
        // Level L+1's entries get their value offsets: their lane counts, scanned.
        int32_t* obn = obp(L + 1);
        for (int cb = qe; cb < nt; cb += BLOCK) {
          const int i = cb + tid;
          int cnt = 0;
          int32_t w = -1;
          if (i < nt) {
            w = q[i];
            if (w >= 0 && w < np) cnt = __builtin_popcountll(group_load(&fnxt[w]));
            else w = -1;
          }
          int total;
          const int ex = block_excl_scan<BLOCK>(cnt, s_wtot, &total);
          if (i < nt) {
            // Each (vertex, lane) is reached once, so the values of a batch
            // fit the slot's stride*64; a run that would not is reported.
            const int64_t o = cbase + ex;
            const int32_t at = o + cnt <= qcap ? (int32_t)o : 0;
            if (o + cnt > qcap) raise_flag(Q.flags, kFlagQueueOverflow);
            eoff[i] = at;
            if (w >= 0) obn[w] = at;
          }
          cbase += total;
        }
        __syncthreads();
      }
      // Phase B: sigma of the new lanes, one wave per vertex, pulling from the
      // neighbours on level L (their frontier masks); long rows are deferred.
      const bool scale = IDENT && L > 0;
      auto defer_long = [&](int i, int32_t, int32_t e0, int32_t e1, uint64_t) -> bool {
        if (e1 - e0 <= kHubArcs) return false;
        int reg = 0;
        if (lane == 0) {
          const int ns = (e1 - e0 + kSliceArcs - 1) / kSliceArcs;
          const int h = atomicAdd(&s_nheavy, 1);
          const int o = atomicAdd(&s_nslices, ns);
          if (h < kHeavyMax && o + ns <= st.part_cap) {
            s_heavy[h] = i;
            s_hoff[h] = o;
            reg = 1;
          } else if (h < kHeavyMax) {
            s_heavy[h] = -1;
          }
        }
        return __builtin_amdgcn_readfirstlane(reg) != 0;
      };
      auto need_f = [&](int, int32_t w) { return group_load(&fnxt[w]); };  // built with atomicOr
      // The new lanes are marked visited in phase C, all entries at once.
      auto early_f = [](int, int32_t, uint64_t) { return 0; };
      auto finish_f = [&](int i, int32_t w, uint64_t need, double acc, int) {
        if ((need >> lane) & 1) sg[own(i, w, need, lane)] = acc;
        if (lane == 0) qm[i] = need;
      };
      const int32_t* obL = CMP ? obp(L) : nullptr;  // compact: offsets of level L's entries
      // Pair (w, lane j): sigma of w for source j from the neighbours on level L.
      auto pair_f = [&](int k, int i, int32_t w, int32_t e0, int32_t e1, int j) {
        double acc;
        if constexpr (CMP) acc = pair_sum_c<kPairU>(col, e0, e1, np, fcur, obL, sg, idn, scale, j, Q.flags);
        else acc = pair_sum<1>(col, e0, e1, np, fcur, sg, idn, scale, j, Q.flags);
        sg[own(i, w, slots.need[k], j)] = acc;
      };
      auto pair_done_f = [&](int, int i, int32_t, uint64_t need) { qm[i] = need; };
      auto pull_f = [&](int32_t e0, int32_t e1, uint64_t need) -> double {
        if constexpr (CMP) return pull_row_c(col, e0, e1, np, fcur, obL, need, sg, idn, scale, lane, Q.flags);
        if (e1 - e0 <= 64) {
          const int32_t a[1] = {e0}, d[1] = {e1 - e0};
          const uint64_t nd[1] = {need};
          double r[1];
          pull_group<1>(col, a, d, np, fcur, nd, sg, idn, scale, lane, Q.flags, r);
          return r[0];
        }
        return pull_row(col, e0, e1, np, fcur, need, sg, idn, scale, lane, Q.flags);
      };
      for (int first = qe + wave; first < nt; first += WAVES * 64)
        pull_list(first, WAVES, min(64, (nt - first + WAVES - 1) / WAVES), slots, q, rowp, np, narcs, lane, Q.flags,
                  need_f, defer_long, early_f, finish_f, pairs, pair_f, pair_done_f, pull_f);
      __syncthreads();
      mark(kProfPhaseB);
      const int nh = min(s_nheavy, kHeavyMax);
      if (nh > 0) {
        for (int h = 0; h < nh; ++h) {
          const int i = s_heavy[h];
          if (i < 0) continue;
          const int32_t w = q[i];
          int32_t e0, e1;
          if (!wave_row(rowp, w, np, narcs, &e0, &e1, Q.flags, lane)) continue;
          const uint64_t need = group_load(&fnxt[w]);
          const int ns = (e1 - e0 + kSliceArcs - 1) / kSliceArcs;
          for (int sl = wave; sl < ns; sl += WAVES) {
            const int32_t a = e0 + sl * kSliceArcs;
            const int32_t b = min(e1, a + kSliceArcs);
            part[(size_t)(s_hoff[h] + sl) * 64 + lane] =
                CMP ? pull_row_c(col, a, b, np, fcur, obL, need, sg, idn, scale, lane, Q.flags)
                    : pull_row(col, a, b, np, fcur, need, sg, idn, scale, lane, Q.flags);
          }
        }
        __syncthreads();
        for (int h = wave; h < nh; h += WAVES) {
          const int i = s_heavy[h];
          if (i < 0) continue;
          const int32_t w = q[i];
          int32_t e0, e1;
          if (!wave_row(rowp, w, np, narcs, &e0, &e1, Q.flags, lane)) continue;
          const uint64_t need = group_load(&fnxt[w]);
          const int ns = (e1 - e0 + kSliceArcs - 1) / kSliceArcs;
          double acc = 0.0;
          for (int sl = 0; sl < ns; ++sl) acc += part[(size_t)(s_hoff[h] + sl) * 64 + lane];
          if ((need >> lane) & 1) sg[own(i, w, need, lane)] = acc;
          if (lane == 0) qm[i] = need;
        }
        __syncthreads();
        mark(kProfPhaseBHeavy);
      }
      // Phase C: retire level L's frontier masks, mark level L+1's lanes
      // visited; level L+1 becomes current.
      for (int i = qs + tid; i < qe; i += BLOCK) {
        const int32_t u = q[i];
        if (u >= 0 && u < np) fcur[u] = 0;
      }
      for (int i = qe + tid; i < nt; i += BLOCK) {
        const int32_t w = q[i];
        if (w >= 0 && w < np) vis[w] |= group_load(&fnxt[w]);
      }
      if (tid == 0) lvl[L + 2] = nt;
      __syncthreads();
      mark(kProfPhaseC);
      uint64_t* t = fcur;
      fcur = fnxt;
      fnxt = t;
      qs = qe;
      qe = nt;
      ++L;
    }
    for (int i = qs + tid; i < qe; i += BLOCK) {
      const int32_t u = q[i];
      if (u >= 0 && u < np) fcur[u] = 0;
    }
    __syncthreads();
    mark(kProfPhaseC);
    const int total = qe;
    const int Lmax = L;
    // Lane j's dump row is that of source ordinal s0 + j.
    double* drow = nullptr;
    if constexpr (DUMP) {
      if (lane < nsrc) drow = dump.delta + (size_t)(W.s0 + lane) * dump.np;
      // Levels and path counts of every entry, before the backward sweep
      // overwrites sigma with coefficients.
      for (int l = 0; l <= Lmax; ++l)
        for (int i = lvl[l] + wave; i < lvl[l + 1]; i += WAVES) {
          const int32_t v = q[i];
          const uint64_t m = qm[i];
          if (v >= 0 && v < np && lane < nsrc && ((m >> lane) & 1)) {
            const size_t o = (size_t)(W.s0 + lane) * dump.np + v;
            dump.dist[o] = l;
            dump.sigma[o] = sg[own(i, v, m, lane)];
          }
        }
      __syncthreads();
    }

    // ---------------- backward sweep ----------------
    for (int l = Lmax; l >= 1; --l) {
      uint64_t* bw = (l & 1) ? bmo : bme;  // masks of level l, written now
      uint64_t* br = (l & 1) ? bme : bmo;  // masks of level l+1, read now
      if (l + 2 <= Lmax)
        for (int i = lvl[l + 2] + tid; i < lvl[l + 3]; i += BLOCK) {
          const int32_t u = q[i];
          if (u >= 0 && u < np) bw[u] = 0;
        }
      const int32_t* obR = CMP ? obp(l + 1) : nullptr;  // compact: offsets of level l+1's entries
      if constexpr (CMP) {
        if (l + 1 <= Lmax) {
          int32_t* obw = obp(l + 1);
          for (int i = lvl[l + 1] + tid; i < lvl[l + 2]; i += BLOCK) {
            const int32_t u = q[i];
            if (u >= 0 && u < np) obw[u] = eoff[i];
          }
        }
      }
      if (tid == 0) {
        s_nheavy = 0;
        s_nslices = 0;
      }
      __syncthreads();
      const int b = lvl[l], e = lvl[l + 1];
      auto defer_long_b = [&](int i, int32_t, int32_t e0, int32_t e1, uint64_t) -> bool {
        if (e1 - e0 <= kHubArcs) return false;
        int reg = 0;
        if (lane == 0) {
          const int ns = (e1 - e0 + kSliceArcs - 1) / kSliceArcs;
          const int h = atomicAdd(&s_nheavy, 1);
          const int o = atomicAdd(&s_nslices, ns);
          if (h < kHeavyMax && o + ns <= st.part_cap) {
            s_heavy[h] = i;
            s_hoff[h] = o;
            reg = 1;
          } else if (h < kHeavyMax) {
            s_heavy[h] = -1;
          }
        }
        return __builtin_amdgcn_readfirstlane(reg) != 0;
      };
      auto need_b = [&](int i, int32_t) { return qm[i]; };
      auto early_b = [&](int i, int32_t v, uint64_t amask) {
        return back_early_at<REACH, IDENT>(sg, own(i, v, amask, lane), rch, idn, v, amask, lane);
      };
      auto finish_b = [&](int i, int32_t v, uint64_t amask, double acc, const BackEarly& pre) {
        back_finish_at(sg, own(i, v, amask, lane), bcp, bw, v, amask, acc, pre, wsrc, lane, Q.flags, drow, srank);
      };
      // Pair (v, lane j): the dependency of v for source j from the
      // coefficients of its neighbours on level l+1 (Eq. (3) in pull form),
      // the coefficient that replaces sigma, and the weighted contribution
      // to bc'[v], summed per entry in LDS.
      auto pair_b = [&](int k, int i, int32_t v, int32_t e0, int32_t e1, int j) {
        const size_t at = own(i, v, slots.need[k], j);
        const double sv = sg[at];
        const double rm1 = reach_m1<REACH, IDENT>(rch, idn, v);
        const double id = IDENT ? (double)idn[v] : 1.0;
        double acc;
        if constexpr (CMP) acc = pair_sum_c<kPairU>(col, e0, e1, np, br, obR, sg, idn, false, j, Q.flags);
        else acc = pair_sum<1>(col, e0, e1, np, br, sg, idn, false, j, Q.flags);
        const double dv = rm1 + sv * acc;
        const int32_t sr = s_srank[j];
        if (side_absent(v, sr)) {
          sg[at] = 0.0;
        } else {
          sg[at] = id * (1.0 + dv) / sv;
          atomicAdd(&s_pacc[wave * 64 + k], side_contrib(s_wsrc[j], dv, rm1, sr));  // LDS (the array itself)
        }
        if constexpr (DUMP) dump.delta[(size_t)(W.s0 + j) * dump.np + v] = dv;
        if (!(sv <= DBL_MAX) || !(dv <= DBL_MAX)) raise_flag(Q.flags, kFlagSigmaOverflow);
      };
      auto pair_done_b = [&](int k, int, int32_t v, uint64_t amask) {
        atomicAdd(&bcp[v], s_pacc[wave * 64 + k]);
        bw[v] = amask;
      };
      auto pull_b = [&](int32_t e0, int32_t e1, uint64_t need) -> double {
        if constexpr (CMP) return pull_row_c(col, e0, e1, np, br, obR, need, sg, idn, false, lane, Q.flags);
        if (e1 - e0 <= 64) {
          const int32_t a[1] = {e0}, d[1] = {e1 - e0};
          const uint64_t nd[1] = {need};
          double r[1];
          pull_group<1>(col, a, d, np, br, nd, sg, idn, false, lane, Q.flags, r);
          return r[0];
        }
        return pull_row(col, e0, e1, np, br, need, sg, idn, false, lane, Q.flags);
      };
      for (int first = b + wave; first < e; first += WAVES * 64)
        pull_list(first, WAVES, min(64, (e - first + WAVES - 1) / WAVES), slots, q, rowp, np, narcs, lane, Q.flags,
                  need_b, defer_long_b, early_b, finish_b, pairs, pair_b, pair_done_b, pull_b);
      __syncthreads();
      mark(kProfBackward);
      const int nh = min(s_nheavy, kHeavyMax);
      if (nh > 0) {
        for (int h = 0; h < nh; ++h) {
          const int i = s_heavy[h];
          if (i < 0) continue;
          const int32_t v = q[i];
          int32_t e0, e1;
          if (!wave_row(rowp, v, np, narcs, &e0, &e1, Q.flags, lane)) continue;
          const uint64_t amask = qm[i];
          const int ns = (e1 - e0 + kSliceArcs - 1) / kSliceArcs;
          for (int sl = wave; sl < ns; sl += WAVES) {
            const int32_t a = e0 + sl * kSliceArcs;
            const int32_t bnd = min(e1, a + kSliceArcs);
            part[(size_t)(s_hoff[h] + sl) * 64 + lane] =
                CMP ? pull_row_c(col, a, bnd, np, br, obR, amask, sg, idn, false, lane, Q.flags)
                    : pull_row(col, a, bnd, np, br, amask, sg, idn, false, lane, Q.flags);
          }
        }
        __syncthreads();
        for (int h = wave; h < nh; h += WAVES) {
          const int i = s_heavy[h];
          if (i < 0) continue;
          const int32_t v = q[i];
          int32_t e0, e1;
          if (!wave_row(rowp, v, np, narcs, &e0, &e1, Q.flags, lane)) continue;
          const uint64_t amask = qm[i];
          const int ns = (e1 - e0 + kSliceArcs - 1) / kSliceArcs;
          const size_t at = own(i, v, amask, lane);
          const BackEarly pre = back_early_at<REACH, IDENT>(sg, at, rch, idn, v, amask, lane);
          double acc = 0.0;
          for (int sl = 0; sl < ns; ++sl) acc += part[(size_t)(s_hoff[h] + sl) * 64 + lane];
          back_finish_at(sg, at, bcp, bw, v, amask, acc, pre, wsrc, lane, Q.flags, drow, srank);
        }
        __syncthreads();
        mark(kProfBackHeavy);
      }
    }
    // Restore the slot: clear the backward masks of the two lowest levels and
    // the visit masks of every entry.
    for (int l = 1; l <= 2 && l <= Lmax; ++l) {
      uint64_t* bw = (l & 1) ? bmo : bme;
      for (int i = lvl[l] + tid; i < lvl[l + 1]; i += BLOCK) {
        const int32_t u = q[i];
        if (u >= 0 && u < np) bw[u] = 0;
      }
    }
    for (int i = tid; i < total; i += BLOCK) {
      const int32_t u = q[i];
      if (u >= 0 && u < np) vis[u] = 0;
    }
    __syncthreads();
    mark(kProfRestore);
    if (prof && tid == 0) {
      prof[kProfItems] += 1;
      prof[kProfLevels] += (uint64_t)Lmax;
      prof[kProfEntries] += (uint64_t)total;
    }
    if (tid == 0) atomicAdd(Q.done, 1);
  }
}

// ---------------------------------------------------------------------------
// Team kernel: the same traversal as ms_kernel, for large pieces.  Instead of
// one workgroup per 64-source item, the workgroups of a launch form teams by
// the XCD they run on (read from the hardware XCC id when the launch starts),
// and all workgroups of a team work on the team's current item, with the
// (vertex, level) entries of each level spread over every wave of the team.
// One item's per-vertex lane masks (about 0.5 MB per mask for a piece of
// 64K vertices) then stay in that XCD's L2, instead of one cold copy per
// workgroup.
//
// Phases are separated by team barriers: release, an arrival counter, a spin
// on the generation word bounded by T.spin_ticks, acquire.  Acquire is an
// agent-scope fence (it invalidates the CU's L1).  When all of a team's
// workgroups run on one XCD (so share its L2), release only waits for the
// wave's own stores, which the per-CU L1 writes through to that L2; a team
// spread over several XCDs releases with an agent-scope fence, which also
// writes back L2.  (A workgroup-scope L1 invalidate is not enough here: a
// launch without thread-group split need not perform it.)  A timed-out wait aborts the team and raises
// kFlagTeamTimeout, so every wave still leaves the kernel.  The kernel needs
// all of its workgroups resident at once; the host launches it cooperatively.
// ---------------------------------------------------------------------------
template <int BLOCK>
struct TeamShared {
  int scan[BLOCK];
  int e0[BLOCK];
  uint64_t f[BLOCK];
  int ok, team, rank, tsize, local;
};

constexpr int kTeamChunk = 16;  // frontier entries per wave-sized chunk of phase A
constexpr int kTeamGrab = 4;  // entries a wave takes at a time in the pull phases

// The team control block is only ever accessed with agent-scope atomics and
// atomic loads/stores, so it is coherent whatever fences a team uses (a plain
// store could sit in one XCD's L2 while an agent-scope load reads memory).
template <typename T>
__device__ __forceinline__ T ctl_load(T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void ctl_store(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int WAVES, int EU, bool REACH, bool IDENT, bool DUMP = false>
__global__ SBC_KERNEL_BOUNDS(WAVES * 64, EU) void ms_team_kernel(DevPieces P, QueueArgs Q, MsState st, TeamArgs T,
                                                                 DumpOut dump) {
  if (Q.magic != kArgMagic) return;
  constexpr int BLOCK = WAVES * 64;
  SBC_DYNAMIC_LDS(lds_raw);
  TeamShared<BLOCK>& S = *reinterpret_cast<TeamShared<BLOCK>*>(lds_raw);
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: scalar registers
  const int nteams = T.nteams;
  if (nteams < 1 || T.heavy_max < 1) return;  // every workgroup takes this exit together
  // Join a team by XCD: with nteams a multiple of 8, XCD x hosts teams
  // x, x+8, ...; otherwise teams span XCDs.  Then wait until every workgroup
  // of the launch has joined, so that team sizes are final.
  if (tid == 0) {
    const int x = xcc_id();
    int team;
    if (nteams % 8 == 0) {
      const int k = atomicAdd(&T.ctl[x % 8].xjoin, 1);
      team = x % 8 + 8 * (k % (nteams / 8));
    } else {
      team = x % nteams;
    }
    S.team = team;
    S.rank = atomicAdd(&T.ctl[team].join, 1);
    atomicOr(&T.ctl[team].xccmask, 1 << x);
    atomicAdd(&T.ctl[0].gjoin, 1);
    int ok = 1;
    const long long t0 = wall_clock64();
    while (ctl_load(&T.ctl[0].gjoin) < (int)gridDim.x) {
      if (wall_clock64() - t0 > T.spin_ticks) {
        raise_flag(Q.flags, kFlagTeamTimeout);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    S.ok = ok;
    S.tsize = ctl_load(&T.ctl[team].join);
    S.local = T.allow_local && __builtin_popcount(ctl_load(&T.ctl[team].xccmask)) == 1;
  }
  __syncthreads();
  if (!S.ok) return;  // every workgroup that timed out leaves; the others time out too
  const int team = S.team, rank = S.rank, tsize = S.tsize;
  const bool local = S.local != 0;
  const int gwave = rank * WAVES + wave, twaves = tsize * WAVES;
  const int gthr = rank * BLOCK + tid, tthr = tsize * BLOCK;
  const bool leader = rank == 0 && tid == 0;
  TeamCtl* ctl = T.ctl + team;
  const int hmax = T.heavy_max;
  const int split = T.split_arcs;  // rows longer than this are split into slices
  int32_t* hv_i = T.heavy + (size_t)team * 2 * hmax;  // queue index of each split row
  int32_t* hv_off = hv_i + hmax;                      // its first slice in part[]
  const size_t slot = team;
  double* sg = st.sg + slot * (size_t)st.stride * 64;
  int32_t* q = st.q + slot * (size_t)st.stride * 64;
  uint64_t* qm = st.qm + slot * (size_t)st.stride * 64;
  uint64_t* vis = st.vis + slot * (size_t)st.stride;
  uint64_t* bufa = st.fa + slot * (size_t)st.stride;
  uint64_t* bufb = st.fb + slot * (size_t)st.stride;
  uint64_t* bufc = st.fc + slot * (size_t)st.stride;
  uint64_t* bm0 = st.ba + slot * (size_t)st.stride;  // backward masks of levels = 0 mod 3
  uint64_t* bm1 = st.bb + slot * (size_t)st.stride;  // ... = 1 mod 3
  uint64_t* bm2 = st.bc + slot * (size_t)st.stride;  // ... = 2 mod 3
  auto bmask = [&](int l) { return (l % 3 == 0) ? bm0 : ((l % 3 == 1) ? bm1 : bm2); };
  int32_t* lvl = st.lvl + slot * (size_t)(st.stride + 3);
  double* part = st.part + slot * (size_t)st.part_cap * 64;
  const int64_t qcap = st.stride * 64;
  const int32_t narcs = P.narcs;
  uint64_t* prof = st.prof ? st.prof + (size_t)blockIdx.x * kProfCounters : nullptr;
  long long tmark = prof ? wall_clock64() : 0;
  auto mark = [&](int idx) {
    if (prof && tid == 0) {
      const long long now = wall_clock64();
      prof[idx] += (uint64_t)(now - tmark);
      tmark = now;
    }
  };
  int gen = 0;
  // Team barrier; false once the team has been aborted.
  auto team_sync = [&](int phase) -> bool {
    mark(phase);
    if (local) xcd_release();
    else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) {
      const int arrived = __hip_atomic_fetch_add(&ctl->arrive, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (arrived == tsize - 1) {
        __hip_atomic_store(&ctl->arrive, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->gen, gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        const long long t0 = wall_clock64();
        while (ctl_load(&ctl->gen) == gen && !ctl_load(&ctl->abort)) {
          if (wall_clock64() - t0 > T.spin_ticks) {
            __hip_atomic_store(&ctl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            raise_flag(Q.flags, kFlagTeamTimeout);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      S.ok = ctl_load(&ctl->abort) ? 0 : 1;
      // One invalidation serves the workgroup: its waves share the CU's L1.
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      xcd_release();
    }
    __syncthreads();
    ++gen;
    mark(kProfSync);
    return S.ok != 0;
  };

  // Entries [b, e) of a pull phase, handed to the team's waves kTeamGrab at a
  // time from the phase's counter; a wave asks for its next share before it
  // works on the current one.  body(i, i1) pulls the kGroup entries from i
  // (up to i1).
  auto grabbed = [&](int slot, int b, int e, auto&& body) {
    int next = 0;
    if (lane == 0) next = atomicAdd(&ctl->grab[slot], kTeamGrab);
    while (true) {
      const int i0 = b + __builtin_amdgcn_readfirstlane(next);
      if (i0 >= e) break;
      if (lane == 0) next = atomicAdd(&ctl->grab[slot], kTeamGrab);
      const int i1 = min(e, i0 + kTeamGrab);
      for (int i = i0; i < i1; i += kGroup) body(i, i1);
    }
  };

  for (int iter = 0;; ++iter) {
    if (leader) ctl_store(&ctl->item[iter & 1], atomicAdd(Q.head, 1));
    if (!team_sync(kProfFetch)) break;
    const int it = __builtin_amdgcn_readfirstlane(ctl_load(&ctl->item[iter & 1]));
    if (it < 0 || it >= Q.nitems) break;  // the same verdict in the whole team
    const WorkItem W = uniform_item(Q.items[it]);
    int32_t vb, np;
    const bool item_good = item_ok(P, Q, W, st.stride, &vb, &np) && W.s1 - W.s0 >= 1 && W.s1 - W.s0 <= 64;
    if (!item_good) {
      if (leader) {
        raise_flag(Q.flags, kFlagBadItem);
        atomicAdd(Q.done, 1);
      }
      continue;
    }
    vb = __builtin_amdgcn_readfirstlane(vb);
    np = __builtin_amdgcn_readfirstlane(np);
    const int32_t* rowp = P.row + vb;
    const int32_t* col = P.col;
    const int32_t* rch = REACH ? P.reach + vb : nullptr;
    const int32_t* idn = IDENT ? P.ident + vb : nullptr;
    // the item's own area when deterministic
    double* bcp = Q.item_base ? Q.item_out + (int64_t)uniform64((uint64_t)Q.item_base[it]) : P.bcp + vb;
    const int nsrc = W.s1 - W.s0;

    // Lane j runs source src_order[vb + s0 + j].
    int32_t s = -1;
    if (lane < nsrc) s = P.src_order[vb + W.s0 + lane];
    if (__ballot(lane < nsrc && (s < 0 || s >= np)) != 0) {  // the same verdict in every wave of the team
      if (leader) {
        raise_flag(Q.flags, kFlagBadSource);
        atomicAdd(Q.done, 1);
      }
      continue;
    }
    double wsrc = 0.0;
    const int32_t srank = (P.nside && P.nside[W.piece] > 0 && lane < nsrc) ? s : -1;  // Algorithm 3 items
    if (lane < nsrc) {
      wsrc = src_weight<REACH, IDENT>(rch, idn, s);
      if (rank == 0 && wave == 0) {
        q[lane] = s;
        qm[lane] = 1ull << lane;
        bufa[s] = 1ull << lane;
        vis[s] = 1ull << lane;
        sg[(size_t)s * 64 + lane] = 1.0;
      }
    }
    if (leader) {
      lvl[0] = 0;
      lvl[1] = nsrc;
      ctl_store(&ctl->qtail, nsrc);
      ctl_store(&ctl->hcnt[0], 0);
      ctl_store(&ctl->scnt[0], 0);
      ctl_store(&ctl->grab[0], 0);
      ctl_store(&ctl->agrab[0], 0);
    }
    if (!team_sync(kProfFetch)) break;

    // Frontier masks rotate over three arrays: level L's in fmask(L), level
    // L+1's built in fmask(L+1), while fmask(L+2) = fmask(L-1) is cleared of
    // level L-1's entries.
    auto fmask = [&](int l) { return (l % 3 == 0) ? bufa : ((l % 3 == 1) ? bufb : bufc); };
    int qprev = 0, qs = 0, qe = nsrc, L = 0, hstep = 0;
    bool alive = true;
    // ---------------- forward sweep ----------------
    // Per level: A (discover level L+1, finish the split rows of level L,
    // clear level L-1's masks) | B (sigma of level L+1; long rows registered,
    // their masks set at once) | the slices of the long rows, if any.
    while (true) {
      uint64_t* fcur = fmask(L);
      uint64_t* fnxt = fmask(L + 1);
      uint64_t* fold = fmask(L + 2);
      if (leader) {  // counters of the next registering phase (last used three phases ago)
        ctl_store(&ctl->hcnt[(hstep + 1) % 3], 0);
        ctl_store(&ctl->scnt[(hstep + 1) % 3], 0);
        ctl_store(&ctl->grab[(hstep + 1) % 3], 0);
      }
      const int nhp = L > 0 ? min(ctl_load(&ctl->hcnt[(hstep + 2) % 3]), hmax) : 0;  // level L's split rows
      // Phase A: waves take chunks of kTeamChunk level-L entries (from the
      // phase's counter, so that fast waves take more) and spread each
      // chunk's arcs over their lanes; the split rows of level L are expanded
      // slice by slice over all waves of the team instead.
      {
        // Reached-first vertices get queue slots, one reservation per wave.
        auto discover = [&](int32_t w, uint64_t fu, bool valid) {
          uint64_t nw = 0;
          if (valid) {
            if (w < 0 || w >= np) raise_flag(Q.flags, kFlagBadArc);
            else nw = fu & ~vis[w];
          }
          bool isnew = false;
          if (nw) isnew = atomicOr((unsigned long long*)&fnxt[w], (unsigned long long)nw) == 0;
          const uint64_t bal = __ballot(isnew);
          if (bal) {
            const int first = __builtin_ctzll(bal);
            int base = 0;
            if (lane == first) base = atomicAdd(&ctl->qtail, (int)__builtin_popcountll(bal));
            base = __builtin_amdgcn_readlane(base, first);
            if (isnew) {
              const int64_t pos = (int64_t)base + __builtin_popcountll(bal & ((1ull << lane) - 1));
              if (pos < qcap) q[pos] = w;
              else raise_flag(Q.flags, kFlagQueueOverflow);
            }
          }
        };
        int* wscan = S.scan + wave * 64;
        int* we0 = S.e0 + wave * 64;
        uint64_t* wf = S.f + wave * 64;
        int next = 0;
        if (lane == 0) next = atomicAdd(&ctl->agrab[L & 1], kTeamChunk);
        while (true) {
          const int cb = qs + __builtin_amdgcn_readfirstlane(next);
          if (cb >= qe) break;
          if (lane == 0) next = atomicAdd(&ctl->agrab[L & 1], kTeamChunk);
          const int i = cb + lane;
          int e0 = 0, deg = 0;
          uint64_t fu = 0;
          if (lane < kTeamChunk && i < qe) {
            const int32_t u = q[i];
            if (u >= 0 && u < np) {
              e0 = rowp[u];
              const int32_t e1 = rowp[u + 1];
              if (e0 >= 0 && e1 >= e0 && e1 <= narcs) {
                deg = e1 - e0;
                fu = qm[i];
                if (L > 0 && deg > split) deg = 0;  // expanded by slices below
              } else {
                raise_flag(Q.flags, kFlagBadArc);
                e0 = 0;
              }
            } else {
              raise_flag(Q.flags, kFlagBadArc);
            }
          }
          const int incl = wave_incl_scan(deg, lane);
          const int total = __builtin_amdgcn_readlane(incl, 63);
          wscan[lane] = incl - deg;
          we0[lane] = e0;
          wf[lane] = fu;
          wave_sync();
          const int nv = min(kTeamChunk, qe - cb);
          for (int tb = 0; tb < total; tb += 64) {  // wave-uniform trip count
            const int t = tb + lane;
            int32_t w = -1;
            uint64_t f = 0;
            if (t < total) {
              int lo = 0, hi = nv - 1;
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (wscan[mid] <= t) lo = mid;
                else hi = mid - 1;
              }
              w = col_load(&col[we0[lo] + (t - wscan[lo])]);
              f = wf[lo];
            }
            discover(w, f, t < total);
          }
          wave_sync();
        }
        for (int h = 0; h < nhp; ++h) {
          const int i = hv_i[h];
          if (i < 0) continue;
          const int32_t u = q[i];
          int32_t e0, e1;
          if (!wave_row(rowp, u, np, narcs, &e0, &e1, Q.flags, lane)) continue;
          const uint64_t fu = qm[i];
          const int ns = (e1 - e0 + kSliceArcs - 1) / kSliceArcs;
          const int o = hv_off[h];
          for (int sl = ((gwave - o) % twaves + twaves) % twaves; sl < ns; sl += twaves) {
            const int32_t a = e0 + sl * kSliceArcs;
            const int32_t b = min(e1, a + kSliceArcs);
            for (int32_t eb = a; eb < b; eb += 64) {
              const int32_t e = eb + lane;
              discover(e < b ? col_load(&col[e]) : -1, fu, e < b);
            }
          }
        }
        // Sigma of level L's split rows: the sum of their slices.
        for (int h = gwave; h < nhp; h += twaves) {
          const int i = hv_i[h];
          if (i < 0) continue;
          const int32_t w = q[i];
          int32_t e0, e1;
          if (!wave_row(rowp, w, np, narcs, &e0, &e1, Q.flags, lane)) continue;
          const uint64_t need = qm[i];
          const int ns = (e1 - e0 + kSliceArcs - 1) / kSliceArcs;
          double acc = 0.0;
          for (int sl = 0; sl < ns; ++sl) acc += part[(size_t)(hv_off[h] + sl) * 64 + lane];
          if ((need >> lane) & 1) sg[(size_t)w * 64 + lane] = acc;
        }
        for (int i = qprev + gthr; i < qs; i += tthr) {  // level L-1's masks
          const int32_t u = q[i];
          if (u >= 0 && u < np) fold[u] = 0;
        }
      }
      if (!team_sync(kProfPhaseA)) {
        alive = false;
        break;
      }
      const int nt = (int)min((int64_t)ctl_load(&ctl->qtail), qcap);
      if (nt == qe) break;  // the same verdict in the whole team
      if (leader) {
        lvl[L + 2] = nt;
        ctl_store(&ctl->agrab[(L + 1) & 1], 0);  // for the next discovery phase
      }
      // Phase B: sigma of the new lanes, one wave per entry, spread over the
      // team.  Long rows are registered for splitting; their masks are set
      // now, their sigma when the next level is discovered.
      const bool scale = IDENT && L > 0;
      const int hs = hstep % 3;
      // Register a long row for splitting (the host sizes the lists for every
      // long row of the piece, so registration cannot run out).
      auto register_long = [&](int i, int32_t e0, int32_t e1) {
        const int ns = (e1 - e0 + kSliceArcs - 1) / kSliceArcs;
        const int h = atomicAdd(&ctl->hcnt[hs], 1);
        const int o = atomicAdd(&ctl->scnt[hs], ns);
        if (h < hmax && o + ns <= st.part_cap) {
          hv_i[h] = i;
          hv_off[h] = o;
        } else {
          raise_flag(Q.flags, kFlagHeavyOverflow);
          if (h < hmax) hv_i[h] = -1;
        }
      };
      auto need_f = [&](int, int32_t w) { return fnxt[w]; };
      auto defer_f = [&](int i, int32_t w, int32_t e0, int32_t e1, uint64_t need) -> bool {
        if (e1 - e0 <= split) return false;
        if (lane == 0) {
          register_long(i, e0, e1);
          vis[w] |= need;
          qm[i] = need;
        }
        return true;
      };
      // The visit mask is read before the pull, so that its update is a store.
      auto early_f = [&](int, int32_t w, uint64_t) {
        uint64_t old = 0;
        if (lane == 0) old = vis[w];
        return old;
      };
      auto finish_f = [&](int i, int32_t w, uint64_t need, double acc, uint64_t old) {
        if ((need >> lane) & 1) sg[(size_t)w * 64 + lane] = acc;
        if (lane == 0) {
          vis[w] = old | need;
          qm[i] = need;
        }
      };
      grabbed(hs, qe, nt, [&](int i0, int i1) {
        pull_entries<kGroup>(i0, i1, q, rowp, np, narcs, col, fcur, sg, idn, scale, lane, Q.flags, need_f, defer_f,
                             early_f, finish_f);
      });
      if (!team_sync(kProfPhaseB)) {
        alive = false;
        break;
      }
      const int nh = min(ctl_load(&ctl->hcnt[hs]), hmax);
      if (nh > 0) {  // the same verdict in the whole team
        // Slice u of all registered slices goes to team wave u mod twaves.
        for (int h = 0; h < nh; ++h) {
          const int i = hv_i[h];
          if (i < 0) continue;
          const int32_t w = q[i];
          int32_t e0, e1;
          if (!wave_row(rowp, w, np, narcs, &e0, &e1, Q.flags, lane)) continue;
          const uint64_t need = qm[i];
          const int ns = (e1 - e0 + kSliceArcs - 1) / kSliceArcs;
          const int o = hv_off[h];
          for (int sl = ((gwave - o) % twaves + twaves) % twaves; sl < ns; sl += twaves) {
            const int32_t a = e0 + sl * kSliceArcs;
            const int32_t b = min(e1, a + kSliceArcs);
            part[(size_t)(o + sl) * 64 + lane] = pull_row(col, a, b, np, fcur, need, sg, idn, scale, lane, Q.flags);
          }
        }
        if (!team_sync(kProfPhaseBHeavy)) {
          alive = false;
          break;
        }
      }
      qprev = qs;
      qs = qe;
      qe = nt;
      ++L;
      ++hstep;
    }
    if (!alive) break;
    // The last phase A finished level L's split rows and cleared level L-1's
    // masks; clear level L's.
    {
      uint64_t* fcur = fmask(L);
      for (int i = qs + gthr; i < qe; i += tthr) {
        const int32_t u = q[i];
        if (u >= 0 && u < np) fcur[u] = 0;
      }
    }
    const int total = qe;
    const int Lmax = L;
    double* drow = nullptr;  // lane j's dump row: source ordinal s0 + j
    if constexpr (DUMP) {
      if (lane < nsrc) drow = dump.delta + (size_t)(W.s0 + lane) * dump.np;
      for (int l = 0; l <= Lmax; ++l)
        for (int i = lvl[l] + gwave; i < lvl[l + 1]; i += twaves) {
          const int32_t v = q[i];
          const uint64_t m = qm[i];
          if (v >= 0 && v < np && lane < nsrc && ((m >> lane) & 1)) {
            const size_t o = (size_t)(W.s0 + lane) * dump.np + v;
            dump.dist[o] = l;
            dump.sigma[o] = sg[(size_t)v * 64 + lane];
          }
        }
      // the backward sweep overwrites sigma only after every wave has dumped it
      if (!team_sync(kProfPhaseC)) break;
    }

    // ---------------- backward sweep ----------------
    // Level l writes the masks of array l mod 3 and reads those of level l+1;
    // meanwhile the idle array (l+2) mod 3 is cleared for level l-1.
    for (int l = Lmax; l >= 1 && alive; --l) {
      uint64_t* bw = bmask(l);
      uint64_t* br = bmask(l + 1);
      uint64_t* bz = bmask(l + 2);
      if (leader) {
        ctl_store(&ctl->hcnt[(hstep + 1) % 3], 0);
        ctl_store(&ctl->scnt[(hstep + 1) % 3], 0);
        ctl_store(&ctl->grab[(hstep + 1) % 3], 0);
      }
      const int hs = hstep % 3;
      if (l + 2 <= Lmax)
        for (int i = lvl[l + 2] + gthr; i < lvl[l + 3]; i += tthr) {
          const int32_t u = q[i];
          if (u >= 0 && u < np) bz[u] = 0;
        }
      const int b = lvl[l], e = lvl[l + 1];
      auto need_b = [&](int i, int32_t) { return qm[i]; };
      auto defer_b = [&](int i, int32_t, int32_t e0, int32_t e1, uint64_t) -> bool {
        if (e1 - e0 <= split) return false;
        if (lane == 0) {
          const int ns = (e1 - e0 + kSliceArcs - 1) / kSliceArcs;
          const int h = atomicAdd(&ctl->hcnt[hs], 1);
          const int o = atomicAdd(&ctl->scnt[hs], ns);
          if (h < hmax && o + ns <= st.part_cap) {
            hv_i[h] = i;
            hv_off[h] = o;
          } else {  // the host sizes the lists for every long row of the piece
            raise_flag(Q.flags, kFlagHeavyOverflow);
            if (h < hmax) hv_i[h] = -1;
          }
        }
        return true;
      };
      // Here the finish loads after the pull: loaded before it, the values
      // would hold registers through the pull and cost more spills.
      auto early_b = [](int, int32_t, uint64_t) { return 0; };
      auto finish_b = [&](int, int32_t v, uint64_t amask, double acc, int) {
        back_finish(sg, bcp, bw, v, amask, acc, back_early<REACH, IDENT>(sg, rch, idn, v, amask, lane), wsrc, lane,
                    Q.flags, drow, srank);
      };
      grabbed(hs, b, e, [&](int i0, int i1) {
        pull_entries<kGroup>(i0, i1, q, rowp, np, narcs, col, br, sg, idn, false, lane, Q.flags, need_b, defer_b,
                             early_b, finish_b);
      });
      if (!team_sync(kProfBackward)) {
        alive = false;
        break;
      }
      const int nh = min(ctl_load(&ctl->hcnt[hs]), hmax);
      if (nh > 0) {
        for (int h = 0; h < nh; ++h) {
          const int i = hv_i[h];
          if (i < 0) continue;
          const int32_t v = q[i];
          int32_t e0, e1;
          if (!wave_row(rowp, v, np, narcs, &e0, &e1, Q.flags, lane)) continue;
          const uint64_t amask = qm[i];
          const int ns = (e1 - e0 + kSliceArcs - 1) / kSliceArcs;
          const int o = hv_off[h];
          for (int sl = ((gwave - o) % twaves + twaves) % twaves; sl < ns; sl += twaves) {
            const int32_t a = e0 + sl * kSliceArcs;
            const int32_t bnd = min(e1, a + kSliceArcs);
            part[(size_t)(o + sl) * 64 + lane] = pull_row(col, a, bnd, np, br, amask, sg, idn, false, lane, Q.flags);
          }
        }
        if (!team_sync(kProfBackHeavy)) {
          alive = false;
          break;
        }
        for (int h = gwave; h < nh; h += twaves) {
          const int i = hv_i[h];
          if (i < 0) continue;
          const int32_t v = q[i];
          int32_t e0, e1;
          if (!wave_row(rowp, v, np, narcs, &e0, &e1, Q.flags, lane)) continue;
          const uint64_t amask = qm[i];
          const int ns = (e1 - e0 + kSliceArcs - 1) / kSliceArcs;
          const BackEarly pre = back_early<REACH, IDENT>(sg, rch, idn, v, amask, lane);
          double acc = 0.0;
          for (int sl = 0; sl < ns; ++sl) acc += part[(size_t)(hv_off[h] + sl) * 64 + lane];
          back_finish(sg, bcp, bw, v, amask, acc, pre, wsrc, lane, Q.flags, drow, srank);
        }
        if (!team_sync(kProfBackHeavy)) {
          alive = false;
          break;
        }
      }
      ++hstep;
    }
    if (!alive) break;
    // Restore the slot: the backward masks of levels 1 and 2 and the visit
    // masks of every entry.  The next item starts after a team barrier.
    for (int l = 1; l <= 2 && l <= Lmax; ++l) {
      uint64_t* bw = bmask(l);
      for (int i = lvl[l] + gthr; i < lvl[l + 1]; i += tthr) {
        const int32_t u = q[i];
        if (u >= 0 && u < np) bw[u] = 0;
      }
    }
    for (int i = gthr; i < total; i += tthr) {
      const int32_t u = q[i];
      if (u >= 0 && u < np) vis[u] = 0;
    }
    mark(kProfRestore);
    if (leader) {
      if (prof) {
        prof[kProfItems] += 1;
        prof[kProfLevels] += (uint64_t)Lmax;
        prof[kProfEntries] += (uint64_t)total;
      }
      atomicAdd(Q.done, 1);
    }
  }
}

// ---------------------------------------------------------------------------
// Small pieces: one source per wavefront, the piece and every source's state
// in LDS.  A workgroup of WAVES waves takes an item (a piece and up to 64 of
// its sources), copies the piece's rows, column ids (16-bit, piece-local),
// reach and ident into LDS, and each wave runs the item's sources
// j = wave, wave + WAVES, ... one after another with the source's levels,
// path counts (then backward coefficients) and BFS order in its own LDS
// slice.  A level is one wave's work: the lanes share the level's arcs, and
// the wave's LDS fences order one level after the other, so waves never wait
// for each other inside an item.  bc' contributions are summed per vertex in
// LDS by all waves and added to global memory once per item.
// Forward: the frontier's arcs are spread over the lanes (prefix sums of the
// row lengths); a lane that reaches an unseen vertex claims it with a
// compare-and-swap on its level and appends it to the BFS order, and every
// arc into the next level adds the frontier vertex's weighted path count
// (sigma[u] * ident[u], the source unweighted) to the target's sigma with an
// LDS atomic add (path counts are integers, so the order of the additions
// does not change them).  Backward: one lane per vertex of the level pulls
// the coefficients of its neighbours one level deeper (Eq. (3) in pull
// form).
// ---------------------------------------------------------------------------
// LDS writes of the wave's lanes before this point are seen by its lanes after it.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  wave_sync();
}

template <int WAVES, bool REACH, bool IDENT, bool DUMP = false>
__global__ __launch_bounds__(WAVES * 64) void wave_kernel(DevPieces P, QueueArgs Q, int32_t np_max, int32_t arcs_max,
                                                          DumpOut dump) {
  if (Q.magic != kArgMagic) return;
  if (np_max < 1 || np_max > kWaveMaxVertices || arcs_max < 0) return;  // every workgroup leaves together
  constexpr int BLOCK = WAVES * 64;
  SBC_DYNAMIC_LDS(lds);
  __shared__ int s_item, s_bad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const WaveLds Lo = wave_lds_layout(np_max, arcs_max, WAVES);
  double* s_bc = reinterpret_cast<double*>(lds + Lo.bc);
  int32_t* s_row = reinterpret_cast<int32_t*>(lds + Lo.row);
  int32_t* s_rch = reinterpret_cast<int32_t*>(lds + Lo.rch);
  int32_t* s_idn = reinterpret_cast<int32_t*>(lds + Lo.idn);
  uint16_t* s_col = reinterpret_cast<uint16_t*>(lds + Lo.col);
  unsigned char* ws = lds + Lo.wave0 + (size_t)wave * Lo.wave_bytes;
  double* sig = reinterpret_cast<double*>(ws + Lo.sig);
  double* fsu = reinterpret_cast<double*>(ws + Lo.fsu);
  int32_t* d = reinterpret_cast<int32_t*>(ws + Lo.d);
  int32_t* scan = reinterpret_cast<int32_t*>(ws + Lo.scan);
  int32_t* fe0 = reinterpret_cast<int32_t*>(ws + Lo.fe0);
  uint16_t* q = reinterpret_cast<uint16_t*>(ws + Lo.q);
  uint16_t* lvl = reinterpret_cast<uint16_t*>(ws + Lo.lvl);

  while (true) {
    if (tid == 0) {
      s_item = atomicAdd(Q.head, 1);
      s_bad = 0;
    }
    __syncthreads();
    const int it = s_item;
    if (it < 0 || it >= Q.nitems) break;  // the same verdict in the whole workgroup
    const WorkItem W = Q.items[it];
    int32_t vb, np;
    bool good = item_ok(P, Q, W, np_max, &vb, &np) && W.s1 - W.s0 >= 1 && W.s1 - W.s0 <= 64;
    int32_t a0 = 0, na = 0;
    if (good) {
      a0 = P.row[vb];
      const int32_t a1 = P.row[vb + np];
      na = a1 - a0;
      if (a0 < 0 || a1 > P.narcs || na < 0 || na > arcs_max) {
        if (tid == 0) raise_flag(Q.flags, kFlagBadPiece);
        good = false;
      }
    }
    if (!good) {
      if (tid == 0) {
        raise_flag(Q.flags, kFlagBadItem);
        atomicAdd(Q.done, 1);
      }
      __syncthreads();  // s_item is read by every thread before thread 0 takes the next item
      continue;
    }
    // Stage the piece: rows relative to the piece's first arc, checked to be
    // nondecreasing and within its arcs; column ids checked to be in range.
    for (int v = tid; v <= np; v += BLOCK) {
      const int32_t r = P.row[vb + v] - a0;
      const int32_t rn = v < np ? P.row[vb + v + 1] - a0 : na;
      if (r < 0 || rn < r || rn > na) s_bad = 1;
      s_row[v] = r;
      if (v < np) {
        s_bc[v] = 0.0;
        if (REACH) s_rch[v] = P.reach[vb + v];
        if (IDENT) s_idn[v] = P.ident[vb + v];
      }
    }
    for (int e = tid; e < na; e += BLOCK) {
      const int32_t c = P.col[a0 + e];
      if (c < 0 || c >= np) s_bad = 1;
      s_col[e] = (uint16_t)(c >= 0 && c < np ? c : 0);
    }
    for (int v = lane; v < np; v += 64) {
      d[v] = -1;
      sig[v] = 0.0;
    }
    __syncthreads();
    if (s_bad) {  // the same verdict in the whole workgroup
      if (tid == 0) {
        raise_flag(Q.flags, kFlagBadArc);
        atomicAdd(Q.done, 1);
      }
      __syncthreads();
      continue;
    }
    const int nsrc = W.s1 - W.s0;
    for (int j = wave; j < nsrc; j += WAVES) {
      const int32_t s = P.src_order[vb + W.s0 + j];  // the same in every lane
      if (s < 0 || s >= np) {
        if (lane == 0) raise_flag(Q.flags, kFlagBadSource);
        continue;
      }
      const double wsrc = src_weight<REACH, IDENT>(s_rch, s_idn, s);
      const int32_t srank = (P.nside && P.nside[W.piece] > 0) ? s : -1;  // Algorithm 3 items
      if (lane == 0) {
        d[s] = 0;
        sig[s] = 1.0;
        q[0] = (uint16_t)s;
        lvl[0] = 0;
        lvl[1] = 1;
      }
      wave_lds_sync();
      // ---------------- forward sweep ----------------
      int qs = 0, qe = 1, L = 0;
      while (true) {
        int cnt = 0;  // vertices of level L+1 found so far (wave-uniform)
        for (int cb = qs; cb < qe; cb += 64) {
          const int i = cb + lane;
          int32_t e0 = 0, deg = 0;
          double su = 0.0;
          if (i < qe) {
            const int u = q[i];
            e0 = s_row[u];
            deg = s_row[u + 1] - e0;
            su = sig[u];
            if (IDENT && L > 0) su *= (double)s_idn[u];
          }
          const int incl = wave_incl_scan(deg, lane);
          const int total = __builtin_amdgcn_readlane(incl, 63);
          scan[lane] = incl - deg;
          fe0[lane] = e0;
          fsu[lane] = su;
          wave_lds_sync();
          const int nv = min(64, qe - cb);
          for (int tb = 0; tb < total; tb += 64) {  // wave-uniform trip count
            const int t = tb + lane;
            bool won = false;
            int w = 0;
            if (t < total) {
              int lo = 0, hi = nv - 1;
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (scan[mid] <= t) lo = mid;
                else hi = mid - 1;
              }
              w = s_col[fe0[lo] + (t - scan[lo])];
              int dw = d[w];
              if (dw < 0) {
                const int old = atomicCAS(&d[w], -1, L + 1);
                won = old == -1;
                dw = won ? L + 1 : old;
              }
              if (dw == L + 1) atomicAdd(&sig[w], fsu[lo]);
            }
            const uint64_t bal = __ballot(won);
            if (won) {
              const int pos = qe + cnt + (int)__builtin_popcountll(bal & ((1ull << lane) - 1));
              if (pos < np) q[pos] = (uint16_t)w;
              else raise_flag(Q.flags, kFlagQueueOverflow);
            }
            cnt += (int)__builtin_popcountll(bal);
          }
          wave_lds_sync();  // the scratch is refilled by the next chunk
        }
        if (cnt == 0) break;
        qs = qe;
        qe = min(np, qe + cnt);
        ++L;
        if (lane == 0) lvl[L + 1] = (uint16_t)qe;
        wave_lds_sync();
      }
      double* drow = nullptr;  // this source's dump row
      if constexpr (DUMP) {
        const size_t o = (size_t)(W.s0 + j) * dump.np;
        drow = dump.delta + o;
        for (int i = lane; i < qe; i += 64) {
          const int v = q[i];
          dump.dist[o + v] = d[v];
          dump.sigma[o + v] = sig[v];
        }
        wave_lds_sync();  // every lane has read sigma before the backward sweep overwrites it
      }
      // ---------------- backward sweep ----------------
      for (int l = L; l >= 1; --l) {
        const int b = lvl[l], e = lvl[l + 1];
        for (int i = b + lane; i < e; i += 64) {
          const int v = q[i];
          double acc = 0.0;
          const int32_t x1 = s_row[v + 1];
          for (int32_t x = s_row[v]; x < x1; ++x) {
            const int w = s_col[x];
            if (d[w] == l + 1) acc += sig[w];
          }
          const double sv = sig[v];
          const double rm1 = reach_m1<REACH, IDENT>(s_rch, s_idn, v);
          const double dv = rm1 + sv * acc;
          if (side_absent(v, srank)) {
            sig[v] = 0.0;
          } else {
            sig[v] = (IDENT ? (double)s_idn[v] : 1.0) * (1.0 + dv) / sv;
            atomicAdd(&s_bc[v], side_contrib(wsrc, dv, rm1, srank));
          }
          if constexpr (DUMP) drow[v] = dv;
          if (!(sv <= DBL_MAX) || !(dv <= DBL_MAX)) raise_flag(Q.flags, kFlagSigmaOverflow);
        }
        wave_lds_sync();
      }
      // Restore the unseen state of every vertex this source reached.
      for (int i = lane; i < qe; i += 64) {
        const int v = q[i];
        d[v] = -1;
        sig[v] = 0.0;
      }
      wave_lds_sync();
    }
    __syncthreads();
    for (int v = tid; v < np; v += BLOCK) {
      const double x = s_bc[v];
      if (x != 0.0) atomicAdd(Q.item_base ? &Q.item_out[Q.item_base[it] + v] : &P.bcp[vb + v], x);
    }
    if (tid == 0) atomicAdd(Q.done, 1);
    __syncthreads();  // LDS is refilled by the next item
  }
}

// ---------------------------------------------------------------------------
// Weighted farness of 64 sources at a time, for closeness on the shattered
// pieces: the breadth-first discovery of ms_kernel's forward sweep without
// path counts.  Lane j runs the piece-local source src_order[vb + s0 + j]
// (s0 + j when src_order is null).  Every level's new
// (vertex, lanes) entries add reach[v] x level to their lanes' sums; a wave
// adds 64 entries into its 64 lanes by visiting the entries in turn (lane j
// takes an entry's weight when bit j of its mask is set), so the sums need no
// atomics, and out[] gets each source's exact int64 sum.
// ---------------------------------------------------------------------------
template <int WAVES, bool REACH>
__global__ __launch_bounds__(WAVES * 64) void far_kernel(DevPieces P, QueueArgs Q, FarState st,
                                                         int64_t* __restrict__ out) {
  if (Q.magic != kArgMagic) return;
  constexpr int BLOCK = WAVES * 64;
  __shared__ int s_item;
  __shared__ int s_cnt;
  __shared__ int s_wtot[WAVES];
  __shared__ int s_scan[BLOCK];
  __shared__ int s_e0[BLOCK];
  __shared__ uint64_t s_f[BLOCK];
  __shared__ long long s_sum[WAVES * 64];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const size_t slot = blockIdx.x;
  int32_t* q = st.q + slot * (size_t)st.qcap;
  uint64_t* vis = st.vis + slot * (size_t)st.stride;
  uint64_t* bufa = st.fa + slot * (size_t)st.stride;
  uint64_t* bufb = st.fb + slot * (size_t)st.stride;
  const int64_t qcap = st.qcap;
  const int32_t narcs = P.narcs;

  while (true) {
    if (tid == 0) s_item = atomicAdd(Q.head, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it < 0 || it >= Q.nitems) break;
    const WorkItem W = Q.items[it];
    int32_t vb, np;
    if (!(item_ok(P, Q, W, st.stride, &vb, &np) && W.s1 - W.s0 >= 1 && W.s1 - W.s0 <= 64 && qcap >= 64)) {
      if (tid == 0) {
        raise_flag(Q.flags, kFlagBadItem);
        atomicAdd(Q.done, 1);
      }
      continue;
    }
    const int32_t* rowp = P.row + vb;
    const int32_t* col = P.col;
    const int32_t* rch = REACH ? P.reach + vb : nullptr;
    const int nsrc = W.s1 - W.s0;  // 1..64
    int32_t s = -1;
    if (lane < nsrc) s = P.src_order ? P.src_order[vb + W.s0 + lane] : W.s0 + lane;
    if (__ballot(lane < nsrc && (s < 0 || s >= np)) != 0) {  // same verdict in every wave
      if (tid == 0) {
        raise_flag(Q.flags, kFlagBadSource);
        atomicAdd(Q.done, 1);
      }
      continue;
    }
    if (wave == 0 && lane < nsrc) {
      q[lane] = s;
      bufa[s] = 1ull << lane;
      vis[s] = 1ull << lane;
    }
    if (tid == 0) s_cnt = 0;
    __syncthreads();

    uint64_t* fcur = bufa;
    uint64_t* fnxt = bufb;
    int qs = 0, qe = nsrc, L = 0;
    long long sum = 0;  // this wave's part of lane `lane`'s source's sum
    while (true) {
      // Discover level L+1: the arcs of level L's entries spread evenly over
      // the workgroup; a vertex's first new lane bit queues it.
      for (int cb = qs; cb < qe; cb += BLOCK) {
        const int i = cb + tid;
        int e0 = 0, deg = 0;
        uint64_t fu = 0;
        if (i < qe) {
          const int32_t u = q[i];
          if (u >= 0 && u < np) {
            e0 = rowp[u];
            const int32_t e1 = rowp[u + 1];
            if (e0 >= 0 && e1 >= e0 && e1 <= narcs) {
              deg = e1 - e0;
              fu = fcur[u];
            } else {
              raise_flag(Q.flags, kFlagBadArc);
              e0 = 0;
            }
          } else {
            raise_flag(Q.flags, kFlagBadArc);
          }
        }
        int total;
        const int ex = block_excl_scan<BLOCK>(deg, s_wtot, &total);
        s_scan[tid] = ex;
        s_e0[tid] = e0;
        s_f[tid] = fu;
        __syncthreads();
        const int nv = min(BLOCK, qe - cb);
        for (int t = tid; t < total; t += BLOCK) {
          int lo = 0, hi = nv - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_scan[mid] <= t) lo = mid;
            else hi = mid - 1;
          }
          const int32_t w = col[s_e0[lo] + (t - s_scan[lo])];
          if (w < 0 || w >= np) {
            raise_flag(Q.flags, kFlagBadArc);
            continue;
          }
          const uint64_t nw = s_f[lo] & ~vis[w];
          if (nw) {
            const uint64_t old = atomicOr((unsigned long long*)&fnxt[w], (unsigned long long)nw);
            if (old == 0) {
              const int pos = atomicAdd(&s_cnt, 1);
              if (qe + pos < qcap) q[qe + pos] = w;
              else raise_flag(Q.flags, kFlagQueueOverflow);
            }
          }
        }
        __syncthreads();
      }
      const int nt = (int)min((int64_t)qe + s_cnt, qcap);
      if (nt == qe) break;
      // Level L+1's entries: mark their lanes visited and add reach x level
      // to those lanes, 64 entries per wave at a time.
      const long long lev = L + 1;
      for (int base = qe + wave * 64; base < nt; base += BLOCK) {
        const int i = base + lane;
        uint64_t m = 0;
        int wt = 0;
        if (i < nt) {
          const int32_t w = q[i];
          if (w >= 0 && w < np) {
            m = fnxt[w];
            vis[w] |= m;
            wt = REACH ? rch[w] : 1;
          }
        }
        const int cnt = min(64, nt - base);
        long long acc = 0;
        for (int k = 0; k < cnt; ++k) {
          const uint64_t mk = readlane64(m, k);
          const int wk = __builtin_amdgcn_readlane(wt, k);
          if ((mk >> lane) & 1) acc += wk;
        }
        sum += lev * acc;
      }
      // Retire level L's frontier masks; level L+1 becomes current.
      for (int i = qs + tid; i < qe; i += BLOCK) {
        const int32_t u = q[i];
        if (u >= 0 && u < np) fcur[u] = 0;
      }
      __syncthreads();
      if (tid == 0) s_cnt = 0;  // every thread has read it; the next discovery adds after a barrier
      uint64_t* t = fcur;
      fcur = fnxt;
      fnxt = t;
      qs = qe;
      qe = nt;
      ++L;
    }
    // Restore the slot: the last level's frontier and every entry's visit mask.
    for (int i = qs + tid; i < qe; i += BLOCK) {
      const int32_t u = q[i];
      if (u >= 0 && u < np) fcur[u] = 0;
    }
    for (int i = tid; i < qe; i += BLOCK) {
      const int32_t u = q[i];
      if (u >= 0 && u < np) vis[u] = 0;
    }
    s_sum[wave * 64 + lane] = sum;
    __syncthreads();
    if (wave == 0) {
      long long tot = 0;
      for (int w = 0; w < WAVES; ++w) tot += s_sum[w * 64 + lane];
      if (lane < nsrc) out[(size_t)vb + s] = (int64_t)tot;
    }
    __syncthreads();
    if (tid == 0) atomicAdd(Q.done, 1);
  }
}


__global__ void mapback_kernel(int32_t n, int32_t nverts, int32_t nmap, const int32_t* __restrict__ map_off,
                               const int32_t* __restrict__ map_idx, const double* __restrict__ bcp,
                               const double* __restrict__ corr, const double* __restrict__ bcx, double scale,
                               double* __restrict__ out) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double acc = bcx ? bcx[v] : 0.0;
  const int32_t j0 = max(map_off[v], 0), j1 = min(map_off[v + 1], nmap);
  for (int32_t j = j0; j < j1; ++j) {
    const int32_t x = map_idx[j];
    if (x < 0 || x >= nverts) continue;
    acc += bcp[x] + (corr ? corr[x] : 0.0);
  }
  out[v] = acc * scale;
}

// Deterministic runs: bc'[x] of packed piece vertex x is the sum, in item
// order (the order of the sources), of x's value in the areas of its piece's
// items; piece p's c_p items own consecutive areas of n_p values from
// area_base[p].
__global__ void det_reduce_kernel(int32_t nverts, int32_t npieces, const int32_t* __restrict__ vtx_off,
                                  const int64_t* __restrict__ area_base, const int32_t* __restrict__ piece_items,
                                  const double* __restrict__ item_out, double* __restrict__ bcp) {
  const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nverts) return;
  int32_t lo = 0, hi = npieces - 1;  // the piece holding x
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (vtx_off[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  const int32_t np = vtx_off[lo + 1] - vtx_off[lo];
  const double* a = item_out + area_base[lo] + (x - vtx_off[lo]);
  double acc = 0.0;
  for (int32_t j = 0; j < piece_items[lo]; ++j) acc += a[(size_t)j * np];
  bcp[x] = acc;
}

// Streaming copy of 16-byte words: a kernel of known traffic (read n*16
// bytes, write n*16 bytes) for bandwidth calibration.
__global__ void copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

template <typename T>
__global__ void fill_kernel(T* p, T v, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

}  // namespace dev
}  // namespace sbc
