// Plain data shared by the device code and the host runtime (no HIP types).
#pragma once

#include <cstdint>

namespace sbc {

constexpr int kMsSliceArcs = 256;  // arcs per split slice of a long row (multi-source kernel)
constexpr int kMsHeavyMax = 128;   // split rows per level (multi-source kernel)

// Packed pieces in device memory.  Piece p owns global piece vertices
// [vtx_off[p], vtx_off[p+1]); row[] holds absolute arc offsets into col[],
// col[] holds piece-local neighbour ids.
struct DevPieces {
  const int32_t* vtx_off;
  const int32_t* row;
  const int32_t* col;
  const int32_t* reach;      // may be null when no piece uses reach
  const int32_t* ident;      // may be null when no piece uses ident
  const int32_t* src_order;  // per piece, local source order
  double* bcp;               // accumulated bc' per piece vertex
};

// One work item: sources src_order[vtx_off[piece] + s0 .. + s1) of `piece`.
struct WorkItem {
  int32_t piece;
  int32_t s0;
  int32_t s1;
  int32_t kind;
};

// Optional per-source outputs for the verification entry point.
struct DebugOut {
  int32_t* dist;
  double* sigma;
  double* delta;
};

// Per-slot state of the one-source-per-workgroup kernel in global memory.
struct WgState {
  int32_t* d;      // [slots][stride]   BFS level, -1 unseen
  double* sig;     // [slots][stride]   sigma, then the backward coefficient
  int32_t* q;      // [slots][stride]   BFS order
  int32_t* lvl;    // [slots][stride+2] level starts
  int64_t stride;  // vertices per slot
};

// Per-slot state of the 64-source batch kernel in global memory.
struct MsState {
  double* sg;      // [slots][stride*64]  per (vertex, lane): sigma, then coefficient
  int32_t* q;      // [slots][stride*64]  (vertex, level) entries in level order
  uint64_t* qm;    // [slots][stride*64]  lanes of the entry at its level
  uint64_t* vis;   // [slots][stride]     lanes that reached the vertex
  uint64_t* fa;    // [slots][stride]     frontier masks, double buffered
  uint64_t* fb;
  uint64_t* ba;    // [slots][stride]     backward level masks, by level parity
  uint64_t* bb;
  int32_t* lvl;    // [slots][stride+3]   level starts in q
  double* part;    // [slots][part_cap*64] partial sums of split high-degree rows
  int64_t stride;
  int32_t part_cap;
};

struct QueueArgs {
  const WorkItem* items;
  int32_t nitems;
  int32_t* head;      // next item to take (device counter, zero before launch)
  int32_t* flags;     // bit 0: sigma overflow, bit 1: level overflow, bit 2: queue overflow
  int32_t* done;      // items finished (device counter)
};

}  // namespace sbc
