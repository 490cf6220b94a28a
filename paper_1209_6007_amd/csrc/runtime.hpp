// Runtime objects behind the C interface: context, graph, plan.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "prep.hpp"
#include "shatterbc.h"

namespace sbc {

void set_error(const std::string& msg);
sbc_status fail(sbc_status code, const std::string& msg);
sbc_status hip_fail(hipError_t e, const char* what);

// Device memory, pinned host staging, streams and events a plan borrows
// instead of creating its own: the serving loop keeps one set per slot, so
// a job neither allocates nor frees device memory (whose release waits for
// the whole device) nor creates streams.  Device buffers are bump-allocated
// from `arena`, uploads go through `staging` with asynchronous copies on
// `own`; reset() makes both empty again once the slot's job is done.
struct SlotResources {
  char* arena = nullptr;
  size_t arena_bytes = 0, arena_used = 0;
  char* staging = nullptr;  // pinned host memory
  size_t staging_bytes = 0, staging_used = 0;
  int32_t* h_ctl = nullptr;  // pinned copy of a plan's control block
  hipStream_t own = nullptr;
  hipStream_t side[5] = {};
  hipEvent_t ev_start = nullptr, ev_trav = nullptr, ev_end = nullptr, ev_fork = nullptr;
  hipEvent_t ev_kc_start[5] = {}, ev_kc_end[5] = {};
  void reset() { arena_used = staging_used = 0; }
  hipError_t create(size_t arena_b, size_t staging_b);
  void destroy();
};

// While a BorrowScope lives, device buffers of this thread come from the
// given slot's arena and uploads go through its staging memory.
struct BorrowScope {
  explicit BorrowScope(SlotResources* r);
  ~BorrowScope();
  SlotResources* prev;
};
SlotResources* borrowed_resources();

// Device buffer owned by one object (or borrowed from a slot's arena, then
// returned with the arena).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = false;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  hipError_t alloc(size_t b);
  void release();
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

struct Params {
  int64_t wave_max_vertices = 256;    // pieces up to this size: small-piece kernel (0: never)
  int64_t wave_wg_waves = 4;          // wavefronts per small-piece workgroup (4 or 8)
  int64_t batch_wg_waves = 8;         // wavefronts per multi-source workgroup
  int64_t batch_waves_per_eu = 8;     // occupancy target of the batch kernel (0, 6 or 8 waves per SIMD)
  int64_t wave_sources_per_item = 64; // sources per small-piece work item (at most 64)
  int64_t slots = 0;                  // resident workgroups per kernel (0: from occupancy)
  int64_t cluster_sources = 2;        // batch source order: 0 as is, 1 balls, 2 common-hub groups then balls
  int64_t batch_pairs = 16;           // batch kernel: rows of <= 32 arcs with at most this many lanes pulled as pairs
  int64_t batch_compact = 1;          // batch kernel: 1 an entry's values lie together (compact), 0 64-lane rows
  int64_t deep_min_levels = 64;       // pieces deeper than this (BFS from the highest-degree vertex): deep class
  int64_t deep_wg_waves = 16;         // wavefronts per workgroup of the deep class's batch kernel
  int64_t deep_waves_per_eu = 0;      // occupancy target of the deep class's batch kernel
  int64_t mem_budget_mb = 0;          // traversal state budget (0: 60% of free memory)
  int64_t profile_phases = 0;         // 1: per-phase timers in the batch kernel
  int64_t order_plain = 0;            // 1: plain problems renumbered breadth-first
  int64_t team_min_vertices = 16384;  // pieces from this size: team kernel (0: never)
  int64_t team_count = 64;            // teams of the team kernel (a multiple of 8: that many per XCD / 8)
  int64_t team_wg_waves = 16;         // wavefronts per workgroup of the team kernel (4, 8 or 16)
  int64_t team_waves_per_eu = 8;      // occupancy target of the team kernel (0 or 8)
  int64_t team_spin_ms = 20000;       // bound of one team barrier wait
  int64_t team_local_fences = 1;      // 1: teams on one XCD fence through L2 only
  int64_t team_cooperative = 1;       // 1: cooperative launch of the team kernel; 0: ordinary launch
  int64_t team_split_arcs = 2048;     // team kernel: rows with more arcs are split into slices
  int64_t team_max_levels = 0;        // pieces deeper than this stay off the team kernel (0: no limit)
  int64_t sample_items = 0;           // tuning only: run an evenly spaced sample of this many items per class
  int64_t far_wg_waves = 16;          // wavefronts per workgroup of the farness kernel
  int64_t server_order = 1;           // serving: 0 oldest job first, 1 least estimated work first
  int64_t server_max_wait_ms = 30000; // serving, order 1: a job waiting longer is taken first
};

}  // namespace sbc

struct sbc_context_s {
  int device = 0;
  hipDeviceProp_t prop{};
  int cus = 0;
  size_t lds_limit = 64 * 1024;  // dynamic LDS one workgroup may use
  double wall_khz = 100000.0;    // device wall-clock rate
  sbc::Params params;
  std::mutex mu;
};

struct sbc_graph_s {
  sbc::HostGraph g;
  bool prepared = false;
  std::string ops;
  sbc::Prepared prep;
  sbc_prep_stats stats{};
};

namespace sbc {

// KC_WAVE: small-piece kernel (one source per wavefront, the piece in LDS).
// KC_BATCH: 64-source batches, one workgroup per batch.  KC_DEEP: the same
// kernel for deep pieces (many levels), launched separately in its own
// workgroup shape.  KC_TEAM: 64-source batches, one team of workgroups per
// batch.  Class 1 is not used (its slots in sbc_run_stats stay zero).
enum KernelClass { KC_WAVE = 0, KC_BATCH = 2, KC_DEEP = 3, KC_TEAM = 4, KC_COUNT = 5 };

// Per-slot state of one launch of the 64-source batch kernel.
struct BatchState {
  DevBuf sg, q, qm, vis, fa, fb, ba, bb, lvl, part, prof, eoff, ob;
  MsState ms{};
  int waves = 8, eu = 8;  // workgroup shape of the launch
};

struct PlanOptions {
  int force_kernel = 0;                 // 0 automatic, 3 batch, 4 team, 5 small-piece
  const int32_t* sources = nullptr;     // one-piece problems: source subset (host), or null for all
  int64_t nsrc = 0;
  bool dump = false;                    // keep every listed source's levels, path counts and dependencies
};

struct Plan {
  sbc_context ctx = nullptr;
  int32_t n = 0;            // output length (original vertices)
  int32_t P = 0;            // pieces
  int64_t V = 0, A = 0;
  bool reach = false, ident = false;
  double scale = 1.0;
  bool has_map = true;
  int32_t nmap = 0;         // entries of map_idx
  // device problem
  DevBuf d_vtx_off, d_row, d_col, d_reach, d_ident, d_src, d_bcp, d_corr, d_bcx, d_map_off, d_map_idx, d_out;
  DevBuf d_nside;           // per piece: side vertices of a side piece (Algorithm 3), when any piece has them
  bool has_side = false;
  DevBuf d_items[KC_COUNT];
  // deterministic runs: per-item bc' areas (see QueueArgs::item_base)
  bool det = false;
  int64_t det_values = 0;   // doubles in d_item_out
  DevBuf d_item_base[KC_COUNT], d_area_base, d_piece_items, d_item_out;
  DevBuf d_ctl;             // int32: heads[KC_COUNT] at 0, done[KC_COUNT] at 8, flags at 16
  int32_t* h_ctl = nullptr; // pinned copy of the control block
  int32_t nitems[KC_COUNT] = {0, 0, 0, 0, 0};
  int32_t max_np[KC_COUNT] = {0, 0, 0, 0, 0};
  int grid[KC_COUNT] = {0, 0, 0, 0, 0};
  int block[KC_COUNT] = {256, 0, 512, 0, 512};
  int64_t sources_in[KC_COUNT] = {0, 0, 0, 0, 0};
  // slot state: the batch kernel's launches (batch and deep classes)
  BatchState bst[2];
  std::vector<uint64_t> h_prof;  // last execution's phase timers, summed over slots
  int64_t prof_slots = 0;        // workgroups whose timers h_prof sums
  // team kernel state: one slot per team, plus control blocks and split-row lists
  DevBuf tm_sg, tm_q, tm_qm, tm_vis, tm_fa, tm_fb, tm_fc, tm_ba, tm_bb, tm_bc, tm_lvl, tm_part, tm_prof, tm_ctl,
      tm_heavy;
  MsState tm{};
  TeamArgs targs{};
  int team_waves = 8, team_eu = 8;
  int wave_waves = 4;                       // small-piece kernel: waves per workgroup
  int32_t wave_np = 0, wave_arcs = 0;       // its LDS is sized for these
  DumpOut dump{};                           // verification dump (dump.dist null when off)
  DevBuf dump_dist, dump_sigma, dump_delta;
  int64_t dump_rows = 0;
  // streams and timing
  hipStream_t own = nullptr;
  hipStream_t side[KC_COUNT] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_start = nullptr, ev_trav = nullptr, ev_end = nullptr;
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_kc_start[KC_COUNT] = {}, ev_kc_end[KC_COUNT] = {};
  bool borrowed = false;  // streams, events and control-block copy belong to a serving slot
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool use_graph = false;
  hipStream_t graph_stream = nullptr;
  hipStream_t last_stream = nullptr;  // stream of the last execute (may be the caller's)
  double* graph_out = nullptr;
  bool ran = false;
  double teps = 0, algo_bytes = 0;
  double teps_k[KC_COUNT] = {0, 0, 0, 0, 0}, bytes_k[KC_COUNT] = {0, 0, 0, 0, 0};
  int64_t total_items = 0;
  double last_host_ms = 0;

  ~Plan();
  // BatchState of a batch-kernel class (KC_BATCH or KC_DEEP)
  BatchState& batch_of(int k) { return bst[k == KC_DEEP ? 1 : 0]; }
  sbc_status build(sbc_context c, const Prepared& prob, uint32_t mode, const PlanOptions& opt);
  sbc_status build_impl(sbc_context c, const Prepared& prob, uint32_t mode, const PlanOptions& opt);
  // Wait for everything this plan enqueued; called before any buffer is freed.
  void quiesce();
  sbc_status enqueue(double* out, hipStream_t s);
  sbc_status execute(double* out, hipStream_t s);
  sbc_status sync(sbc_run_stats* st);
  size_t device_bytes() const;
};

// Rough device footprint of a plan for admission control.
size_t estimate_plan_bytes(sbc_context c, const Prepared& prob);

}  // namespace sbc

struct sbc_plan_s {
  sbc::Plan plan;
};
