// Plain data shared by the device code and the host runtime (no HIP types).
#pragma once

#include <cstdint>

namespace sbc {

constexpr int kMsSliceArcs = 256;  // arcs per split slice of a long row (multi-source kernel)
constexpr int kMsHeavyMax = 128;   // split rows per level (multi-source kernel)
constexpr int kMsHubArcs = 1024;   // rows longer than this are split (multi-source kernels)

// Kernel arguments carry this word; a kernel that sees anything else returns
// at once instead of dereferencing pointers it cannot trust.
constexpr int32_t kArgMagic = 0x5BC0DE01;

// Device error flags (QueueArgs::flags).
constexpr int32_t kFlagSigmaOverflow = 1;   // a path count left the binary64 range
constexpr int32_t kFlagQueueOverflow = 4;   // a traversal queue would have overrun its slot
constexpr int32_t kFlagBadItem = 8;         // work item index or source range out of bounds
constexpr int32_t kFlagBadPiece = 16;       // piece offsets out of bounds or larger than the slot
constexpr int32_t kFlagBadArc = 32;         // row bounds, neighbour id or queue entry out of range
constexpr int32_t kFlagBadSource = 64;      // a source id outside its piece
constexpr int32_t kFlagTeamTimeout = 128;   // a team barrier wait exceeded its bound (team aborted)
constexpr int32_t kFlagHeavyOverflow = 256; // more long rows in a level than the team's split lists hold
constexpr int32_t kFlagRangeMask = kFlagBadItem | kFlagBadPiece | kFlagBadArc | kFlagBadSource;

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
  // per piece: 0, or k > 0 for a side piece (sources: its side vertices
  // 0..k-1, each running Algorithm 3 without the side vertices before it);
  // null when no piece is a side piece
  const int32_t* nside;
  double* bcp;               // accumulated bc' per piece vertex
  int32_t npieces;           // P: entries of vtx_off are P+1
  int32_t nverts;            // V: entries of row are V+1
  int32_t narcs;             // A: entries of col
  int32_t pad_;
};

// One work item: sources src_order[vtx_off[piece] + s0 .. + s1) of `piece`.
struct WorkItem {
  int32_t piece;
  int32_t s0;
  int32_t s1;
  int32_t kind;
};

// Per-source state written by the dump variants of the traversal kernels
// (the verification entry point).  The source with ordinal k in the run's
// source list and piece vertex v share index k*np + v.  The host fills dist
// with -1 and delta with 0 first; a kernel writes the level and path count of
// every vertex a source reaches, and the dependency of every vertex but the
// source itself.
struct DumpOut {
  int32_t* dist;
  double* sigma;
  double* delta;
  int32_t np;
  int32_t pad_;
};

// Per-slot state of the 64-source batch kernel in global memory.
struct MsState {
  double* sg;      // [slots][stride*64]  per (vertex, lane): sigma, then coefficient
  int32_t* q;      // [slots][stride*64]  (vertex, level) entries in level order
  uint64_t* qm;    // [slots][stride*64]  lanes of the entry at its level
  uint64_t* vis;   // [slots][stride]     lanes that reached the vertex
  uint64_t* fa;    // [slots][stride]     frontier masks, double buffered
  uint64_t* fb;    //                     (the team kernel rotates three)
  uint64_t* fc;    //                     team kernel only
  uint64_t* ba;    // [slots][stride]     backward level masks, by level parity
  uint64_t* bb;    //                     (the team kernel rotates three: level mod 3)
  uint64_t* bc;    //                     team kernel only
  int32_t* lvl;    // [slots][stride+3]   level starts in q
  double* part;    // [slots][part_cap*64] partial sums of split high-degree rows
  uint64_t* prof;  // [slots][kProfCounters] phase timers, or null
  // Compact value layout of the batch kernel (null: sg holds 64-lane rows):
  // an entry's values, one per lane of its mask, lie together in sg at
  // eoff[entry], and ob holds per vertex the offset of its entry on the level
  // of each parity that is being read.
  int32_t* eoff;   // [slots][stride*64]  per entry: offset of its values in sg
  int32_t* ob;     // [slots][2*stride]   per level parity and vertex: offset of the vertex's entry
  int64_t stride;
  int32_t part_cap;
  int32_t pairs;   // batch kernel: entries with short rows and at most this many lanes are pulled as
                   // (entry, lane) pairs (0: never)
};

// Per-slot phase timers of the batch kernel (wall-clock ticks, or counts).
enum ProfCounter {
  kProfFetch = 0,      // taking items and setting up a batch
  kProfPhaseA = 1,     // forward: discovering the next level
  kProfPhaseB = 2,     // forward: path counts of the new level
  kProfPhaseBHeavy = 3,
  kProfPhaseC = 4,     // forward: retiring the frontier
  kProfBackward = 5,   // backward: dependencies and accumulation
  kProfBackHeavy = 6,
  kProfRestore = 7,    // clearing the slot for the next batch
  kProfItems = 8,      // count
  kProfLevels = 9,     // count
  kProfEntries = 10,   // count of (vertex, level) entries
  kProfSync = 11,      // team kernel: waiting at team barriers
  kProfCounters = 12
};

// Team kernel: the workgroups of a launch form `nteams` teams by the XCD they
// run on (the hardware XCC id), so that the workgroups of a team share one L2;
// each team works on one 64-source item at a time in one MsState slot.
// TeamCtl is a team's control block in global memory (zero before launch).
struct TeamCtl {
  int32_t arrive;    // barrier arrivals of the current phase
  int32_t gen;       // barrier generation
  int32_t abort;     // set once a barrier wait timed out
  int32_t qtail;     // entries in the team's queue
  int32_t item[2];   // items taken by the team's leader, by iteration parity
  int32_t hcnt[3];   // long rows registered, by registering phase mod 3
  int32_t scnt[3];   // slices registered, by registering phase mod 3
  int32_t join;      // workgroups in the team
  int32_t xccmask;   // XCDs the team's workgroups run on
  int32_t xjoin;     // (block of XCD x) workgroups that arrived on XCD x
  int32_t gjoin;     // (block 0) workgroups of the whole launch that arrived
  int32_t grab[3];   // entries handed out in a pull phase, by registering phase mod 3
  int32_t agrab[2];  // frontier entries handed out in a discovery phase, by level parity
  int32_t pad[11];   // 128 bytes
};

struct TeamArgs {
  TeamCtl* ctl;         // [nteams]
  int32_t* heavy;       // [nteams][2][heavy_max]: queue index, first slice
  int32_t nteams;
  int32_t heavy_max;    // long rows per level a team can register (host-sized: never exceeded)
  int64_t spin_ticks;   // bound of one barrier wait, in wall-clock ticks
  int32_t allow_local;  // 1: teams on one XCD release without writing back L2
  int32_t split_arcs;   // rows with more arcs are pulled in slices over the team
  int32_t cooperative;  // 1: cooperative launch (the runtime guarantees residency); 0: ordinary launch
};

// Dynamic LDS of the small-piece kernel (one source per wavefront, the piece
// in LDS) for pieces of at most np vertices and `arcs` arcs, with `waves`
// waves per workgroup.  Shared by the workgroup: per-vertex bc' sums (f64),
// row offsets, reach and ident (i32), column ids (u16).  Then one slice per
// wave: sigma / backward coefficient (f64), level (i32), BFS order and level
// starts (u16), and a 64-entry scratch of the frontier's arc prefix sums, row
// starts and weighted path counts.  Offsets are multiples of 16 bytes.
struct WaveLds {
  uint64_t bc, row, rch, idn, col;  // shared arrays
  uint64_t wave0, wave_bytes;       // first wave slice, bytes per slice
  uint64_t sig, d, q, lvl, scan, fe0, fsu;  // offsets inside a slice
  uint64_t total;
};
constexpr uint64_t wave_lds_align(uint64_t x) { return (x + 15) & ~uint64_t(15); }
constexpr WaveLds wave_lds_layout(int64_t np, int64_t arcs, int64_t waves) {
  WaveLds L{};
  uint64_t o = 0;
  L.bc = o;
  o = wave_lds_align(o + 8 * (uint64_t)np);
  L.row = o;
  o = wave_lds_align(o + 4 * (uint64_t)(np + 1));
  L.rch = o;
  o = wave_lds_align(o + 4 * (uint64_t)np);
  L.idn = o;
  o = wave_lds_align(o + 4 * (uint64_t)np);
  L.col = o;
  o = wave_lds_align(o + 2 * (uint64_t)arcs);
  L.wave0 = o;
  uint64_t w = 0;
  L.sig = w;
  w = wave_lds_align(w + 8 * (uint64_t)np);
  L.fsu = w;
  w += 8 * 64;
  L.d = w;
  w = wave_lds_align(w + 4 * (uint64_t)np);
  L.scan = w;
  w += 4 * 64;
  L.fe0 = w;
  w += 4 * 64;
  L.q = w;
  w = wave_lds_align(w + 2 * (uint64_t)np);
  L.lvl = w;
  w = wave_lds_align(w + 2 * (uint64_t)(np + 2));
  L.wave_bytes = w;
  L.total = o + (uint64_t)waves * w;
  return L;
}
// Largest piece the small-piece kernel takes (its BFS order is 16-bit).
constexpr int32_t kWaveMaxVertices = 4096;

// Per-slot state of the farness kernel: the (vertex, lanes) entries of every
// level (qcap per slot), and per-vertex visit and frontier lane masks.
struct FarState {
  int32_t* q;
  uint64_t* vis;
  uint64_t* fa;
  uint64_t* fb;
  int64_t stride;  // vertices per slot (the largest piece)
  int64_t qcap;    // entries per slot
};

struct QueueArgs {
  const WorkItem* items;
  int32_t nitems;
  int32_t magic;      // kArgMagic
  int32_t* head;      // next item to take (device counter, zero before launch)
  int32_t* flags;     // kFlag* bits
  int32_t* done;      // items finished (device counter)
  // Deterministic runs: item i accumulates its bc' into its own area
  // item_out[item_base[i] .. + piece vertices) instead of the shared bc'
  // (null otherwise); a later reduction sums the areas in a fixed order.
  const int64_t* item_base;
  double* item_out;
};

}  // namespace sbc
