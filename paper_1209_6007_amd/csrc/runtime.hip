// Plan construction and execution: uploads a prepared problem, sorts pieces
// into kernel classes, builds the device work queues, sizes the per-workgroup
// traversal state, and runs every class concurrently on its own stream.
#include "runtime.hpp"

#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstring>
#include <numeric>

namespace sbc {

namespace {
thread_local std::string g_last_error;

// Control block: work-queue heads, items done per class, error flags.
constexpr int kCtlHeads = 0, kCtlDone = 8, kCtlFlags = 16, kCtlInts = 32;

double wall_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

thread_local SlotResources* t_borrow = nullptr;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// A device copy of v.  With borrowed slot resources, the bytes go through
// the slot's pinned staging memory with an asynchronous copy on its stream
// (the plan waits for that stream before it runs); otherwise, or when the
// staging memory is full, a synchronous copy.
template <typename T>
hipError_t upload(DevBuf& b, const std::vector<T>& v) {
  size_t bytes = std::max<size_t>(v.size() * sizeof(T), sizeof(T));
  hipError_t e = b.alloc(bytes);
  if (e != hipSuccess || v.empty()) return e;
  const size_t n = v.size() * sizeof(T);
  SlotResources* r = t_borrow;
  if (r && r->staging && r->staging_used + align256(n) <= r->staging_bytes) {
    char* h = r->staging + r->staging_used;
    r->staging_used += align256(n);
    std::memcpy(h, v.data(), n);
    return hipMemcpyAsync(b.p, h, n, hipMemcpyHostToDevice, r->own);
  }
  return hipMemcpy(b.p, v.data(), n, hipMemcpyHostToDevice);
}
}  // namespace

SlotResources* borrowed_resources() { return t_borrow; }
BorrowScope::BorrowScope(SlotResources* r) : prev(t_borrow) { t_borrow = r; }
BorrowScope::~BorrowScope() { t_borrow = prev; }

hipError_t SlotResources::create(size_t arena_b, size_t staging_b) {
  hipError_t e;
  arena_bytes = arena_b;
  staging_bytes = staging_b;
  if ((e = hipMalloc((void**)&arena, arena_b)) != hipSuccess) return e;
  if ((e = hipHostMalloc((void**)&staging, staging_b, hipHostMallocDefault)) != hipSuccess) return e;
  if ((e = hipHostMalloc((void**)&h_ctl, 256, hipHostMallocDefault)) != hipSuccess) return e;
  if ((e = hipStreamCreateWithFlags(&own, hipStreamNonBlocking)) != hipSuccess) return e;
  for (auto& st : side)
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) return e;
  for (hipEvent_t* ev : {&ev_start, &ev_trav, &ev_end})
    if ((e = hipEventCreate(ev)) != hipSuccess) return e;
  if ((e = hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming)) != hipSuccess) return e;
  for (int k = 0; k < 5; ++k) {
    if ((e = hipEventCreate(&ev_kc_start[k])) != hipSuccess) return e;
    if ((e = hipEventCreate(&ev_kc_end[k])) != hipSuccess) return e;
  }
  return hipSuccess;
}

void SlotResources::destroy() {
  if (own) (void)hipStreamSynchronize(own);
  for (auto st : side)
    if (st) (void)hipStreamSynchronize(st);
  for (auto ev : {ev_start, ev_trav, ev_end, ev_fork})
    if (ev) (void)hipEventDestroy(ev);
  for (int k = 0; k < 5; ++k) {
    if (ev_kc_start[k]) (void)hipEventDestroy(ev_kc_start[k]);
    if (ev_kc_end[k]) (void)hipEventDestroy(ev_kc_end[k]);
  }
  for (auto st : side)
    if (st) (void)hipStreamDestroy(st);
  if (own) (void)hipStreamDestroy(own);
  if (h_ctl) (void)hipHostFree(h_ctl);
  if (staging) (void)hipHostFree(staging);
  if (arena) (void)hipFree(arena);
  *this = SlotResources();
}

void set_error(const std::string& msg) { g_last_error = msg; }
const std::string& last_error() { return g_last_error; }

sbc_status fail(sbc_status code, const std::string& msg) {
  set_error(msg);
  return code;
}

sbc_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? SBC_E_OOM : SBC_E_DEVICE;
}

hipError_t DevBuf::alloc(size_t b) {
  release();
  if (b == 0) b = 8;
  if (SlotResources* r = t_borrow) {  // from the slot's arena: no device allocation
    if (r->arena_used + align256(b) > r->arena_bytes) return hipErrorOutOfMemory;
    p = r->arena + r->arena_used;
    r->arena_used += align256(b);
    bytes = b;
    owned = false;
    return hipSuccess;
  }
  hipError_t e = hipMalloc(&p, b);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    return e;
  }
  bytes = b;
  owned = true;
  return hipSuccess;
}

void DevBuf::release() {
  if (p && owned) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
  owned = false;
}

void Plan::quiesce() {
  if (own) (void)hipStreamSynchronize(own);
  for (int c = 0; c < KC_COUNT; ++c)
    if (side[c]) (void)hipStreamSynchronize(side[c]);
  if (graph_stream) (void)hipStreamSynchronize(graph_stream);
  if (last_stream) (void)hipStreamSynchronize(last_stream);
  (void)hipGetLastError();
}

Plan::~Plan() {
  // Device buffers are freed by the members' destructors after this body:
  // nothing the plan launched may still be running then.
  if (ctx) {
    (void)hipSetDevice(ctx->device);
    quiesce();
  }
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (borrowed) return;  // the streams, events and control-block copy are the slot's
  for (auto e : {ev_start, ev_trav, ev_end, ev_fork})
    if (e) (void)hipEventDestroy(e);
  for (int c = 0; c < KC_COUNT; ++c) {
    if (ev_kc_start[c]) (void)hipEventDestroy(ev_kc_start[c]);
    if (ev_kc_end[c]) (void)hipEventDestroy(ev_kc_end[c]);
    if (side[c]) (void)hipStreamDestroy(side[c]);
  }
  if (own) (void)hipStreamDestroy(own);
  if (h_ctl) (void)hipHostFree(h_ctl);
}

size_t Plan::device_bytes() const {
  size_t t = 0;
  for (const DevBuf* b : {&d_vtx_off, &d_row, &d_col, &d_reach, &d_ident, &d_src, &d_bcp, &d_corr, &d_bcx,
                          &d_map_off, &d_map_idx, &d_out, &d_ctl, &d_area_base, &d_piece_items, &d_item_out,
                          &d_nside, &tm_sg, &tm_q, &tm_qm, &tm_vis, &tm_fa, &tm_fb,
                          &tm_fc, &tm_ba, &tm_bb, &tm_bc, &tm_lvl, &tm_part, &tm_prof, &tm_ctl, &tm_heavy, &dump_dist,
                          &dump_sigma, &dump_delta})
    t += b->bytes;
  for (const BatchState& b : bst)
    for (const DevBuf* d : {&b.sg, &b.q, &b.qm, &b.vis, &b.fa, &b.fb, &b.ba, &b.bb, &b.lvl, &b.part, &b.prof})
      t += d->bytes;
  for (int c = 0; c < KC_COUNT; ++c) t += d_items[c].bytes + d_item_base[c].bytes;
  return t;
}

namespace {

// Per-slot bytes of the 64-source batch kernel for pieces of up to `stride`
// vertices and `arcs` arcs.
size_t ms_slot_bytes(int64_t stride, int64_t part_cap) {
  return (size_t)stride * 64 * (8 + 4 + 8) + (size_t)stride * 8 * 5 + (size_t)(stride + 3) * 4 +
         (size_t)part_cap * 64 * 8;
}

// Long rows (more than `split` arcs) of piece p and their slices: the team
// kernel registers at most that many per level, since a vertex has at most
// one entry per level.
void long_rows(const Prepared& prob, int32_t p, int64_t split, int64_t* rows, int64_t* slices) {
  *rows = 0;
  *slices = 0;
  for (int32_t v = prob.vtx_off[p]; v < prob.vtx_off[p + 1]; ++v) {
    const int64_t d = (int64_t)prob.row[v + 1] - prob.row[v];
    if (d > split) {
      ++*rows;
      *slices += (d + kMsSliceArcs - 1) / kMsSliceArcs;
    }
  }
}

// Levels of a breadth-first search of piece p from its highest-degree vertex
// (a lower bound on the piece's diameter, and at least half of it).
int64_t bfs_depth(const Prepared& prob, int32_t p) {
  const int32_t vb = prob.vtx_off[p], np = prob.vtx_off[p + 1] - vb;
  if (np <= 0) return 0;
  int32_t start = 0;
  for (int32_t v = 1; v < np; ++v)
    if (prob.row[vb + v + 1] - prob.row[vb + v] > prob.row[vb + start + 1] - prob.row[vb + start]) start = v;
  std::vector<int32_t> d(np, -1), q;
  q.reserve(np);
  q.push_back(start);
  d[start] = 0;
  int64_t depth = 0;
  for (size_t h = 0; h < q.size(); ++h) {
    const int32_t v = q[h];
    for (int32_t e = prob.row[vb + v]; e < prob.row[vb + v + 1]; ++e) {
      const int32_t w = prob.col[e];
      if (w >= 0 && w < np && d[w] < 0) {
        d[w] = d[v] + 1;
        depth = std::max<int64_t>(depth, d[w]);
        q.push_back(w);
      }
    }
  }
  return depth;
}

// Kernel class of a piece of np vertices (before the LDS-size checks).
int classify(const Params& pr, int32_t np, int force) {
  if (force == 5) return KC_WAVE;
  if (force == 4) return KC_TEAM;
  if (force == 3) return KC_BATCH;
  const bool team = pr.team_min_vertices > 0 && np >= pr.team_min_vertices;
  // The team threshold wins where the two overlap.
  if (!team && np <= pr.wave_max_vertices) return KC_WAVE;
  return team ? KC_TEAM : KC_BATCH;
}

// LDS the small-piece kernel may give one workgroup (at most 64 KB, so that
// at least two workgroups fit a compute unit).
size_t wave_lds_budget(const sbc_context_s* c) { return std::min<size_t>(c->lds_limit, 64 * 1024); }

}  // namespace

size_t estimate_plan_bytes(sbc_context c, const Prepared& prob) {
  size_t t = (size_t)prob.V() * (4 * 4 + 8 * 2) + prob.A() * 4 + (size_t)prob.n * (8 * 2 + 4) +
             prob.map_idx.size() * 4 + (size_t)prob.pieces() * 4;
  int64_t max_batch = 0, max_batch_arcs = 0, max_team = 0, max_team_slices = 1;
  for (int32_t p = 0; p < prob.pieces(); ++p) {
    int32_t np = prob.vtx_off[p + 1] - prob.vtx_off[p];
    const int64_t arcs = prob.row[prob.vtx_off[p + 1]] - prob.row[prob.vtx_off[p]];
    int k = classify(c->params, np, 0);
    if (k == KC_BATCH) {
      max_batch = std::max<int64_t>(max_batch, np);
      max_batch_arcs = std::max<int64_t>(max_batch_arcs, arcs);
    }
    if (k == KC_TEAM) {
      int64_t rows = 0, slices = 0;
      long_rows(prob, p, c->params.team_split_arcs, &rows, &slices);
      max_team = std::max<int64_t>(max_team, np);
      max_team_slices = std::max<int64_t>(max_team_slices, slices);
    }
  }
  if (max_batch)
    t += (ms_slot_bytes(max_batch, max_batch_arcs / kMsSliceArcs + 2 * kMsHeavyMax) +
          (size_t)max_batch * (64 * 4 + 2 * 4)) * 4;  // with the compact layout's offsets
  if (max_team)
    t += (ms_slot_bytes(max_team, max_team_slices) + (size_t)max_team * 16) *
         std::max<int64_t>(1, c->params.team_count);
  return t;
}

sbc_status Plan::build(sbc_context c, const Prepared& prob, uint32_t mode, const PlanOptions& opt) {
  const sbc_status rc = build_impl(c, prob, mode, opt);
  if (rc != SBC_OK) quiesce();  // an early return must not leave set-up kernels running
  return rc;
}

sbc_status Plan::build_impl(sbc_context c, const Prepared& prob_in, uint32_t mode, const PlanOptions& opt) {
  ctx = c;
  if (opt.force_kernel != 0 && opt.force_kernel != 3 && opt.force_kernel != 4 && opt.force_kernel != 5)
    return fail(SBC_E_INVALID_ARG, "kernel must be 0 (automatic), 3 (batch), 4 (team) or 5 (small-piece)");
  if ((opt.sources || opt.dump) && prob_in.pieces() != 1)
    return fail(SBC_E_INVALID_ARG, "a source list needs a one-piece problem");
  const Params& pr = c->params;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  // Streams and events first: every set-up kernel runs on `own`, so any
  // return path can wait for it before buffers are released.  A serving
  // slot lends its own.
  if (SlotResources* r = borrowed_resources()) {
    borrowed = true;
    own = r->own;
    for (int k = 0; k < KC_COUNT; ++k) {
      side[k] = r->side[k];
      ev_kc_start[k] = r->ev_kc_start[k];
      ev_kc_end[k] = r->ev_kc_end[k];
    }
    ev_start = r->ev_start;
    ev_trav = r->ev_trav;
    ev_end = r->ev_end;
    ev_fork = r->ev_fork;
  } else {
    if ((e = hipStreamCreateWithFlags(&own, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
    for (int k = 0; k < KC_COUNT; ++k)
      if ((e = hipStreamCreateWithFlags(&side[k], hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
    for (hipEvent_t* ev : {&ev_start, &ev_trav, &ev_end})
      if ((e = hipEventCreate(ev)) != hipSuccess) return hip_fail(e, "event");
    if ((e = hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event");
    for (int k = 0; k < KC_COUNT; ++k) {
      if ((e = hipEventCreate(&ev_kc_start[k])) != hipSuccess) return hip_fail(e, "event");
      if ((e = hipEventCreate(&ev_kc_end[k])) != hipSuccess) return hip_fail(e, "event");
    }
  }
  const bool plain = !(mode & SBC_COMPRESSED);
  // Deterministic runs: every item sums into its own area, reduced in a fixed
  // order afterwards.  Small pieces go to the batch kernel (the small-piece
  // kernel's waves add into shared LDS sums in no fixed order), and the batch
  // kernel pulls every entry with a whole wave (the pair path's per-entry LDS
  // sums have no fixed order either).
  det = (mode & SBC_DETERMINISTIC) != 0;
  const Prepared* probp = &prob_in;
  Prepared local;
  if (opt.sources || (pr.cluster_sources && prob_in.pieces() > 0)) {
    local = prob_in;
    probp = &local;
    if (pr.cluster_sources && !opt.sources) cluster_sources(&local, 64, (int)pr.cluster_sources);
    if (opt.sources) {
      // plain graph, one piece: the listed sources first
      std::vector<uint8_t> seen(local.n, 0);
      for (int64_t i = 0; i < opt.nsrc; ++i) {
        int32_t s = opt.sources[i];
        if (s < 0 || s >= local.n) return fail(SBC_E_INDEX_RANGE, "source out of range");
        if (seen[s]) return fail(SBC_E_INVALID_ARG, "sources must be distinct");
        seen[s] = 1;
        local.src_order[i] = s;
      }
      int64_t k = opt.nsrc;
      for (int32_t v = 0; v < local.n; ++v)
        if (!seen[v]) local.src_order[k++] = v;
    }
  }
  const Prepared& prob = *probp;
  n = prob.n;
  P = prob.pieces();
  V = prob.V();
  A = prob.A();
  reach = prob.weighted;
  ident = prob.has_ident;
  scale = (mode & SBC_UNORDERED) ? 0.5 : 1.0;

  // Work items by kernel class.
  std::vector<WorkItem> items[KC_COUNT];
  std::vector<int64_t> item_base[KC_COUNT];
  std::vector<int64_t> area_base(P, 0);
  std::vector<int32_t> piece_items(P, 0);
  det_values = 0;
  std::vector<double> item_teps[KC_COUNT], item_bytes[KC_COUNT];
  std::vector<int> piece_class(P, -1);
  teps = 0;
  algo_bytes = 0;
  for (int32_t p = 0; p < P; ++p) {
    const int32_t vb = prob.vtx_off[p], np = prob.vtx_off[p + 1] - vb;
    const int64_t arcs = (int64_t)prob.row[vb + np] - prob.row[vb];
    int k = classify(pr, np, opt.force_kernel);
    // Deep pieces (many BFS levels) pay a team barrier per phase and level:
    // with team_max_levels set they stay on the one-workgroup kernel.
    if (k == KC_TEAM && opt.force_kernel != 4 && pr.team_max_levels > 0 &&
        bfs_depth(prob, p) > pr.team_max_levels)
      k = KC_BATCH;
    // Pieces deeper than deep_min_levels run on the batch kernel in their own
    // launch and shape: most of their entries carry a few lanes, and more
    // waves per workgroup keep more of them in flight.
    if ((k == KC_BATCH || k == KC_TEAM) && opt.force_kernel == 0 && pr.deep_min_levels > 0 &&
        np > pr.deep_min_levels && bfs_depth(prob, p) > pr.deep_min_levels)
      k = KC_DEEP;
    // A small piece must fit LDS with the class's largest vertex count: then
    // any mix of the class's pieces fits one launch.
    if (k == KC_WAVE &&
        (np > kWaveMaxVertices ||
         wave_lds_layout(std::max<int64_t>(np, pr.wave_max_vertices), arcs, pr.wave_wg_waves).total >
             wave_lds_budget(c))) {
      if (opt.force_kernel == 5) return fail(SBC_E_INVALID_ARG, "piece too large for the small-piece kernel");
      k = (pr.team_min_vertices > 0 && np >= pr.team_min_vertices) ? KC_TEAM : KC_BATCH;
    }
    if (det && k == KC_WAVE) k = (pr.team_min_vertices > 0 && np >= pr.team_min_vertices) ? KC_TEAM : KC_BATCH;
    piece_class[p] = k;
    int32_t nsrc = np;
    if (opt.sources) nsrc = (int32_t)opt.nsrc;
    const bool side_piece = p < (int32_t)prob.nside.size() && prob.nside[p] > 0;
    if (side_piece) nsrc = prob.nside[p];  // Algorithm 3: only the side vertices are sources
    if (nsrc <= 0) continue;
    const int32_t chunk = k == KC_WAVE ? (int32_t)std::min<int64_t>(64, pr.wave_sources_per_item) : 64;
    const double per = 8.0 * arcs + (plain ? 48.0 : (reach || ident ? 56.0 : 48.0)) * np;
    for (int32_t s0 = 0; s0 < nsrc; s0 += chunk) {
      const int32_t s1 = std::min(nsrc, s0 + chunk);
      items[k].push_back({p, s0, s1, k});
      item_base[k].push_back(det_values + (int64_t)piece_items[p] * np);
      piece_items[p]++;
      item_teps[k].push_back((double)(s1 - s0) * (double)arcs * 0.5);
      item_bytes[k].push_back((double)(s1 - s0) * per);
    }
    area_base[p] = det_values;
    det_values += (int64_t)piece_items[p] * np;
    max_np[k] = std::max(max_np[k], np);
  }
  // Tuning runs may keep an evenly spaced sample of the items (the result
  // then covers only their sources): the class with the most items keeps at
  // most sample_items of them, and every other class the same fraction of
  // its own (at least one), so that one factor scales the whole run.
  total_items = 0;
  size_t most = 0;
  for (int k = 0; k < KC_COUNT; ++k) most = std::max(most, items[k].size());
  const double keep_frac = (pr.sample_items > 0 && most > (size_t)pr.sample_items)
                               ? (double)pr.sample_items / (double)most : 1.0;
  for (int k = 0; k < KC_COUNT; ++k) {
    if (keep_frac < 1.0 && !items[k].empty()) {
      const size_t total = items[k].size();
      const size_t keep = std::min(total, std::max<size_t>(1, (size_t)std::llround(keep_frac * (double)total)));
      std::vector<WorkItem> kept;
      std::vector<double> kt, kb;
      std::vector<int64_t> kbase;
      for (size_t j = 0; j < keep; ++j) {
        const size_t idx = j * total / keep;
        kept.push_back(items[k][idx]);
        kt.push_back(item_teps[k][idx]);
        kb.push_back(item_bytes[k][idx]);
        kbase.push_back(item_base[k][idx]);
      }
      items[k].swap(kept);
      item_base[k].swap(kbase);
      item_teps[k].swap(kt);
      item_bytes[k].swap(kb);
    }
    for (size_t j = 0; j < items[k].size(); ++j) {
      sources_in[k] += items[k][j].s1 - items[k][j].s0;
      teps_k[k] += item_teps[k][j];
      bytes_k[k] += item_bytes[k][j];
    }
    teps += teps_k[k];
    algo_bytes += bytes_k[k];
    nitems[k] = (int32_t)items[k].size();
    total_items += nitems[k];
  }

  // Upload the problem.
  if ((e = upload(d_vtx_off, prob.vtx_off)) != hipSuccess) return hip_fail(e, "upload vtx_off");
  if ((e = upload(d_row, prob.row)) != hipSuccess) return hip_fail(e, "upload row");
  if ((e = upload(d_col, prob.col)) != hipSuccess) return hip_fail(e, "upload col");
  if (reach && (e = upload(d_reach, prob.reach)) != hipSuccess) return hip_fail(e, "upload reach");
  if (ident && (e = upload(d_ident, prob.ident)) != hipSuccess) return hip_fail(e, "upload ident");
  if ((e = upload(d_src, prob.src_order)) != hipSuccess) return hip_fail(e, "upload src_order");
  has_side = false;
  for (int32_t x : prob.nside) has_side = has_side || x > 0;
  if (has_side && (e = upload(d_nside, prob.nside)) != hipSuccess) return hip_fail(e, "upload nside");
  if ((e = d_bcp.alloc(std::max<int64_t>(V, 1) * sizeof(double))) != hipSuccess) return hip_fail(e, "alloc bcp");
  has_map = !plain;
  nmap = (int32_t)prob.map_idx.size();
  if ((e = upload(d_corr, prob.corr)) != hipSuccess) return hip_fail(e, "upload corr");
  if ((e = upload(d_bcx, prob.bcx)) != hipSuccess) return hip_fail(e, "upload bcx");
  if ((e = upload(d_map_off, prob.map_off)) != hipSuccess) return hip_fail(e, "upload map_off");
  if ((e = upload(d_map_idx, prob.map_idx)) != hipSuccess) return hip_fail(e, "upload map_idx");
  if ((e = d_out.alloc(std::max<int32_t>(n, 1) * sizeof(double))) != hipSuccess) return hip_fail(e, "alloc out");
  for (int k = 0; k < KC_COUNT; ++k)
    if ((e = upload(d_items[k], items[k])) != hipSuccess) return hip_fail(e, "upload items");
  if (det) {
    for (int k = 0; k < KC_COUNT; ++k)
      if ((e = upload(d_item_base[k], item_base[k])) != hipSuccess) return hip_fail(e, "upload item areas");
    if ((e = upload(d_area_base, area_base)) != hipSuccess) return hip_fail(e, "upload item areas");
    if ((e = upload(d_piece_items, piece_items)) != hipSuccess) return hip_fail(e, "upload item areas");
    if ((e = d_item_out.alloc((size_t)std::max<int64_t>(det_values, 1) * sizeof(double))) != hipSuccess)
      return hip_fail(e, "alloc per-item areas of a deterministic run");
  }
  if ((e = d_ctl.alloc(sizeof(int32_t) * kCtlInts)) != hipSuccess) return hip_fail(e, "alloc ctl");
  if (borrowed) {
    h_ctl = borrowed_resources()->h_ctl;
  } else if ((e = hipHostMalloc((void**)&h_ctl, sizeof(int32_t) * kCtlInts, hipHostMallocDefault)) != hipSuccess) {
    return hip_fail(e, "hipHostMalloc");
  }
  std::memset(h_ctl, 0, sizeof(int32_t) * kCtlInts);

  // Traversal state, sized by occupancy and the memory budget (a serving
  // slot: what is left of its arena).
  size_t freeb = 0, totalb = 0;
  size_t budget;
  if (borrowed) {
    const SlotResources* r = borrowed_resources();
    budget = (size_t)((r->arena_bytes - r->arena_used) * 0.9);
  } else {
    (void)hipMemGetInfo(&freeb, &totalb);
    budget = pr.mem_budget_mb > 0 ? (size_t)pr.mem_budget_mb << 20 : (size_t)(freeb * 0.6);
  }
  const int cus = c->cus;
  if (nitems[KC_WAVE]) {
    // The launch's LDS holds the largest piece's vertices and the most arcs
    // of any piece of the class; each fits, and both together must too.
    wave_waves = (int)pr.wave_wg_waves;
    block[KC_WAVE] = wave_waves * 64;
    int32_t mnp = 0, marcs = 0;
    for (int32_t p = 0; p < P; ++p)
      if (piece_class[p] == KC_WAVE) {
        const int32_t vb = prob.vtx_off[p], np = prob.vtx_off[p + 1] - vb;
        mnp = std::max(mnp, np);
        marcs = std::max<int32_t>(marcs, prob.row[vb + np] - prob.row[vb]);
      }
    wave_np = mnp;
    wave_arcs = marcs;
    if (wave_lds_layout(mnp, marcs, wave_waves).total > wave_lds_budget(c))
      return fail(SBC_E_INVALID_ARG, "small-piece class does not fit LDS");
    const int occ = occupancy_wave(wave_waves, mnp, marcs);
    if (occ <= 0) return fail(SBC_E_INVALID_ARG, "small-piece kernel configuration cannot be resident");
    int g = cus * occ;
    if (pr.slots > 0) g = (int)pr.slots;
    grid[KC_WAVE] = std::max(1, std::min(g, nitems[KC_WAVE]));
  }
  for (int k : {KC_BATCH, KC_DEEP}) {
    if (!nitems[k]) continue;
    BatchState& B = batch_of(k);
    const int64_t stride = max_np[k];
    int64_t max_arcs = 0;
    for (int32_t p = 0; p < P; ++p) {
      const int32_t vb = prob.vtx_off[p], np = prob.vtx_off[p + 1] - vb;
      if (piece_class[p] == k) max_arcs = std::max<int64_t>(max_arcs, (int64_t)prob.row[vb + np] - prob.row[vb]);
    }
    const int64_t part_cap = max_arcs / kMsSliceArcs + 2 * kMsHeavyMax;
    B.waves = (int)(k == KC_DEEP ? pr.deep_wg_waves : pr.batch_wg_waves);
    // the dump variant is built at the compiler's default occupancy only
    B.eu = opt.dump ? 0 : (int)(k == KC_DEEP ? pr.deep_waves_per_eu : pr.batch_waves_per_eu);
    block[k] = B.waves * 64;
    const int occ = occupancy_ms(B.waves, B.eu);
    int g = cus * occ;
    if (pr.slots > 0) g = (int)pr.slots;
    const bool compact = pr.batch_compact != 0;
    const size_t per = ms_slot_bytes(stride, part_cap) + (compact ? (size_t)stride * (64 * 4 + 2 * 4) : 0);
    g = std::min<int64_t>(g, std::max<int64_t>(1, (int64_t)(budget / per)));
    g = std::max(1, std::min(g, nitems[k]));
    grid[k] = g;
    MsState& ms = B.ms;
    ms.stride = stride;
    ms.part_cap = (int32_t)part_cap;
    ms.pairs = det ? 0 : (int32_t)pr.batch_pairs;
    const size_t G = g;
    if ((e = B.sg.alloc(G * stride * 64 * 8)) != hipSuccess) return hip_fail(e, "alloc ms sg");
    if ((e = B.q.alloc(G * stride * 64 * 4)) != hipSuccess) return hip_fail(e, "alloc ms q");
    if ((e = B.qm.alloc(G * stride * 64 * 8)) != hipSuccess) return hip_fail(e, "alloc ms qm");
    for (DevBuf* d : {&B.vis, &B.fa, &B.fb, &B.ba, &B.bb})
      if ((e = d->alloc(G * stride * 8)) != hipSuccess) return hip_fail(e, "alloc ms masks");
    if ((e = B.lvl.alloc(G * (stride + 3) * 4)) != hipSuccess) return hip_fail(e, "alloc ms lvl");
    if ((e = B.part.alloc(G * part_cap * 64 * 8)) != hipSuccess) return hip_fail(e, "alloc ms part");
    ms.sg = B.sg.as<double>();
    ms.q = B.q.as<int32_t>();
    ms.qm = B.qm.as<uint64_t>();
    ms.vis = B.vis.as<uint64_t>();
    ms.fa = B.fa.as<uint64_t>();
    ms.fb = B.fb.as<uint64_t>();
    ms.ba = B.ba.as<uint64_t>();
    ms.bb = B.bb.as<uint64_t>();
    ms.lvl = B.lvl.as<int32_t>();
    ms.part = B.part.as<double>();
    ms.prof = nullptr;
    if (pr.profile_phases) {
      if ((e = B.prof.alloc(G * kProfCounters * 8)) != hipSuccess) return hip_fail(e, "alloc ms prof");
      ms.prof = B.prof.as<uint64_t>();
    }
    ms.eoff = nullptr;
    ms.ob = nullptr;
    if (compact) {  // written before every read: no clearing
      if ((e = B.eoff.alloc(G * stride * 64 * 4)) != hipSuccess) return hip_fail(e, "alloc ms eoff");
      if ((e = B.ob.alloc(G * stride * 2 * 4)) != hipSuccess) return hip_fail(e, "alloc ms ob");
      ms.eoff = B.eoff.as<int32_t>();
      ms.ob = B.ob.as<int32_t>();
    }
    for (uint64_t* p : {ms.vis, ms.fa, ms.fb, ms.ba, ms.bb})
      if ((e = launch_fill_u64(p, 0, (int64_t)G * stride, own)) != hipSuccess) return hip_fail(e, "fill ms");
  }
  if (nitems[KC_TEAM]) {
    // One slot per team; the grid is every workgroup that can be resident,
    // dealt round-robin to the teams.
    int64_t stride = 0, max_rows = 1, max_slices = 1;
    for (int32_t p = 0; p < P; ++p) {
      const int32_t vb = prob.vtx_off[p], np = prob.vtx_off[p + 1] - vb;
      if (piece_class[p] != KC_TEAM) continue;
      stride = std::max<int64_t>(stride, np);
      int64_t rows = 0, slices = 0;
      long_rows(prob, p, pr.team_split_arcs, &rows, &slices);
      max_rows = std::max(max_rows, rows);
      max_slices = std::max(max_slices, slices);
    }
    team_waves = (int)pr.team_wg_waves;
    team_eu = (pr.team_waves_per_eu > 0 && !opt.dump) ? 8 : 0;
    block[KC_TEAM] = team_waves * 64;
    int coop = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c->device) != hipSuccess) {
      (void)hipGetLastError();
      coop = 0;
    }
    if (!coop && pr.team_cooperative)
      return fail(SBC_E_DEVICE, "the device does not support cooperative launches (team kernel)");
    const int occ = occupancy_team(team_waves, team_eu, opt.dump);
    if (occ <= 0) return fail(SBC_E_INVALID_ARG, "team kernel configuration cannot be resident");
    const int nteams = (int)std::max<int64_t>(1, pr.team_count);
    int g = cus * occ;
    if (pr.slots > 0) g = (int)std::min<int64_t>(pr.slots, g);
    grid[KC_TEAM] = g;
    const int64_t part_cap = max_slices;
    tm.stride = stride;
    tm.part_cap = (int32_t)part_cap;
    const size_t T = nteams;
    if ((e = tm_sg.alloc(T * stride * 64 * 8)) != hipSuccess) return hip_fail(e, "alloc team sg");
    if ((e = tm_q.alloc(T * stride * 64 * 4)) != hipSuccess) return hip_fail(e, "alloc team q");
    if ((e = tm_qm.alloc(T * stride * 64 * 8)) != hipSuccess) return hip_fail(e, "alloc team qm");
    for (DevBuf* b : {&tm_vis, &tm_fa, &tm_fb, &tm_fc, &tm_ba, &tm_bb, &tm_bc})
      if ((e = b->alloc(T * stride * 8)) != hipSuccess) return hip_fail(e, "alloc team masks");
    if ((e = tm_lvl.alloc(T * (stride + 3) * 4)) != hipSuccess) return hip_fail(e, "alloc team lvl");
    if ((e = tm_part.alloc(T * part_cap * 64 * 8)) != hipSuccess) return hip_fail(e, "alloc team part");
    if ((e = tm_ctl.alloc(T * sizeof(TeamCtl))) != hipSuccess) return hip_fail(e, "alloc team ctl");
    if ((e = tm_heavy.alloc(T * 2 * (size_t)max_rows * 4)) != hipSuccess) return hip_fail(e, "alloc team heavy");
    tm.sg = tm_sg.as<double>();
    tm.q = tm_q.as<int32_t>();
    tm.qm = tm_qm.as<uint64_t>();
    tm.vis = tm_vis.as<uint64_t>();
    tm.fa = tm_fa.as<uint64_t>();
    tm.fb = tm_fb.as<uint64_t>();
    tm.fc = tm_fc.as<uint64_t>();
    tm.ba = tm_ba.as<uint64_t>();
    tm.bb = tm_bb.as<uint64_t>();
    tm.bc = tm_bc.as<uint64_t>();
    tm.lvl = tm_lvl.as<int32_t>();
    tm.part = tm_part.as<double>();
    tm.prof = nullptr;
    if (pr.profile_phases) {
      if ((e = tm_prof.alloc((size_t)g * kProfCounters * 8)) != hipSuccess) return hip_fail(e, "alloc team prof");
      tm.prof = tm_prof.as<uint64_t>();
    }
    for (uint64_t* p : {tm.vis, tm.fa, tm.fb, tm.fc, tm.ba, tm.bb, tm.bc})
      if ((e = launch_fill_u64(p, 0, (int64_t)T * stride, own)) != hipSuccess) return hip_fail(e, "fill team");
    targs.ctl = tm_ctl.as<TeamCtl>();
    targs.heavy = tm_heavy.as<int32_t>();
    targs.nteams = nteams;
    targs.heavy_max = (int32_t)max_rows;
    targs.allow_local = pr.team_local_fences ? 1 : 0;
    targs.split_arcs = (int32_t)pr.team_split_arcs;
    targs.cooperative = pr.team_cooperative ? 1 : 0;
    targs.spin_ticks = (int64_t)((double)pr.team_spin_ms * c->wall_khz);
  }
  if (opt.dump) {
    // One row of V values per listed source; rows start unreached (-1) and
    // with no dependency (0), which the traversal leaves at the source.
    dump_rows = opt.sources ? opt.nsrc : V;
    const size_t cells = (size_t)std::max<int64_t>(1, dump_rows) * (size_t)std::max<int64_t>(1, V);
    if ((e = dump_dist.alloc(cells * 4)) != hipSuccess) return hip_fail(e, "alloc dump");
    if ((e = dump_sigma.alloc(cells * 8)) != hipSuccess) return hip_fail(e, "alloc dump");
    if ((e = dump_delta.alloc(cells * 8)) != hipSuccess) return hip_fail(e, "alloc dump");
    dump = {dump_dist.as<int32_t>(), dump_sigma.as<double>(), dump_delta.as<double>(), (int32_t)V, 0};
    if ((e = launch_fill_i32(dump.dist, -1, (int64_t)cells, own)) != hipSuccess) return hip_fail(e, "fill dump");
    if ((e = launch_fill_f64(dump.sigma, 0.0, (int64_t)cells, own)) != hipSuccess) return hip_fail(e, "fill dump");
    if ((e = launch_fill_f64(dump.delta, 0.0, (int64_t)cells, own)) != hipSuccess) return hip_fail(e, "fill dump");
  }
  if ((e = hipStreamSynchronize(own)) != hipSuccess) return hip_fail(e, "plan setup");
  return SBC_OK;
}

sbc_status Plan::enqueue(double* out, hipStream_t s) {
  hipError_t e;
  int32_t* ctl = d_ctl.as<int32_t>();
  int32_t* heads = ctl + kCtlHeads;
  int32_t* done = ctl + kCtlDone;
  int32_t* flags = ctl + kCtlFlags;
  if ((e = launch_fill_f64(d_bcp.as<double>(), 0.0, V, s)) != hipSuccess) return hip_fail(e, "fill bcp");
  if (det && (e = launch_fill_f64(d_item_out.as<double>(), 0.0, det_values, s)) != hipSuccess)
    return hip_fail(e, "fill item areas");
  if ((e = launch_fill_i32(ctl, 0, kCtlInts, s)) != hipSuccess) return hip_fail(e, "fill ctl");
  for (int k : {KC_BATCH, KC_DEEP}) {
    const MsState& ms = batch_of(k).ms;
    if (nitems[k] && ms.prof && (e = launch_fill_u64(ms.prof, 0, (int64_t)grid[k] * kProfCounters, s)) != hipSuccess)
      return hip_fail(e, "fill prof");
  }
  if (nitems[KC_TEAM]) {
    if ((e = launch_fill_i32((int32_t*)targs.ctl, 0, (int64_t)targs.nteams * (int64_t)(sizeof(TeamCtl) / 4), s)) !=
        hipSuccess)
      return hip_fail(e, "fill team ctl");
    if (tm.prof && (e = launch_fill_u64(tm.prof, 0, (int64_t)grid[KC_TEAM] * kProfCounters, s)) != hipSuccess)
      return hip_fail(e, "fill prof");
  }
  DevPieces dp{d_vtx_off.as<int32_t>(), d_row.as<int32_t>(), d_col.as<int32_t>(), d_reach.as<int32_t>(),
               d_ident.as<int32_t>(), d_src.as<int32_t>(), has_side ? d_nside.as<int32_t>() : nullptr,
               d_bcp.as<double>(), P, (int32_t)V, (int32_t)A, 0};
  if ((e = hipEventRecord(ev_fork, s)) != hipSuccess) return hip_fail(e, "event");
  // Largest classes first so the long multi-source items start early.  The
  // team kernel occupies the whole device, so the other classes follow it.
  const DumpOut* dp_dump = dump.dist ? &dump : nullptr;
  const int order[4] = {KC_TEAM, KC_DEEP, KC_BATCH, KC_WAVE};
  for (int k : order) {
    if (!nitems[k]) continue;
    hipStream_t ks = side[k];
    hipEvent_t after = (k != KC_TEAM && nitems[KC_TEAM]) ? ev_kc_end[KC_TEAM] : ev_fork;
    if ((e = hipStreamWaitEvent(ks, after, 0)) != hipSuccess) return hip_fail(e, "wait");
    if (!use_graph && (e = hipEventRecord(ev_kc_start[k], ks)) != hipSuccess) return hip_fail(e, "event");
    QueueArgs qa{d_items[k].as<WorkItem>(), nitems[k], kArgMagic, heads + k, flags, done + k,
                 det ? d_item_base[k].as<int64_t>() : nullptr, det ? d_item_out.as<double>() : nullptr};
    if (k == KC_TEAM) {
      e = launch_team(dp, qa, reach, ident, team_waves, team_eu, grid[k], tm, targs, dp_dump, ks);
    } else if (k == KC_BATCH || k == KC_DEEP) {
      const BatchState& B = batch_of(k);
      e = launch_ms(dp, qa, reach, ident, B.waves, B.eu, grid[k], B.ms, dp_dump, ks);
    } else {
      e = launch_wave(dp, qa, reach, ident, wave_waves, grid[k], wave_np, wave_arcs, dp_dump, ks);
    }
    if (e != hipSuccess) return hip_fail(e, "launch traversal");
    if ((e = hipEventRecord(ev_kc_end[k], ks)) != hipSuccess) return hip_fail(e, "event");
    if ((e = hipStreamWaitEvent(s, ev_kc_end[k], 0)) != hipSuccess) return hip_fail(e, "wait");
  }
  if (det && (e = launch_det_reduce((int32_t)V, P, d_vtx_off.as<int32_t>(), d_area_base.as<int64_t>(),
                                    d_piece_items.as<int32_t>(), d_item_out.as<double>(), d_bcp.as<double>(), s)) !=
                 hipSuccess)
    return hip_fail(e, "launch deterministic reduction");
  if (!use_graph && (e = hipEventRecord(ev_trav, s)) != hipSuccess) return hip_fail(e, "event");
  double* dst = out ? out : d_out.as<double>();
  if (has_map) {
    e = launch_mapback(n, (int32_t)V, nmap, d_map_off.as<int32_t>(), d_map_idx.as<int32_t>(), d_bcp.as<double>(),
                       d_corr.as<double>(), d_bcx.as<double>(), scale, dst, s);
  } else {
    e = launch_mapback(n, (int32_t)V, nmap, d_map_off.as<int32_t>(), d_map_idx.as<int32_t>(), d_bcp.as<double>(), nullptr,
                       nullptr, scale, dst, s);
  }
  if (e != hipSuccess) return hip_fail(e, "launch mapback");
  if ((e = hipMemcpyAsync(h_ctl, ctl, sizeof(int32_t) * kCtlInts, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(e, "copy ctl");
  return SBC_OK;
}

sbc_status Plan::execute(double* out, hipStream_t s) {
  hipError_t e;
  if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  if (!s) s = own;
  last_stream = s;
  const double t0 = wall_ms();
  if ((e = hipEventRecord(ev_start, s)) != hipSuccess) return hip_fail(e, "event");
  sbc_status rc = SBC_OK;
  if (use_graph) {
    if (graph_exec && (graph_stream != s || graph_out != out)) {
      (void)hipGraphExecDestroy(graph_exec);
      (void)hipGraphDestroy(graph);
      graph_exec = nullptr;
      graph = nullptr;
    }
    if (!graph_exec) {
      hipStream_t cap = own;
      if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "begin capture");
      rc = enqueue(out, cap);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(cap, &g);
      if (rc != SBC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return hip_fail(e, "end capture");
      graph = g;
      if ((e = hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0)) != hipSuccess)
        return hip_fail(e, "graph instantiate");
      graph_stream = s;
      graph_out = out;
    }
    if ((e = hipGraphLaunch(graph_exec, s)) != hipSuccess) return hip_fail(e, "graph launch");
  } else {
    rc = enqueue(out, s);
    if (rc != SBC_OK) return rc;
  }
  if ((e = hipEventRecord(ev_end, s)) != hipSuccess) return hip_fail(e, "event");
  ran = true;
  last_host_ms = wall_ms() - t0;
  return SBC_OK;
}

sbc_status Plan::sync(sbc_run_stats* st) {
  hipError_t e;
  if (!ran) return fail(SBC_E_INVALID_ARG, "plan has not been executed");
  const double t0 = wall_ms();
  if ((e = hipEventSynchronize(ev_end)) != hipSuccess) return hip_fail(e, "sync");
  float ms_all = 0, ms_tr = 0, ms_mb = 0;
  double class_ms[KC_COUNT] = {0, 0, 0, 0, 0};
  (void)hipEventElapsedTime(&ms_all, ev_start, ev_end);
  if (!use_graph) {
    float a = 0, b = 0;
    double first = 1e30, last = 0;
    for (int k = 0; k < KC_COUNT; ++k) {
      class_ms[k] = 0;
      if (!nitems[k]) continue;
      (void)hipEventElapsedTime(&a, ev_start, ev_kc_start[k]);
      (void)hipEventElapsedTime(&b, ev_start, ev_kc_end[k]);
      first = std::min<double>(first, a);
      last = std::max<double>(last, b);
      class_ms[k] = b - a;
    }
    ms_tr = (first < 1e29) ? (float)(last - first) : 0.f;
    (void)hipEventElapsedTime(&ms_mb, ev_trav, ev_end);
  } else {
    ms_tr = ms_all;
  }
  const int32_t flags = h_ctl[kCtlFlags];
  if (bst[0].ms.prof || bst[1].ms.prof || tm.prof) {
    h_prof.assign(kProfCounters, 0);
    prof_slots = 0;
    for (int k : {KC_BATCH, KC_DEEP, KC_TEAM}) {
      uint64_t* src = (k == KC_TEAM) ? tm.prof : batch_of(k).ms.prof;
      if (!src || !nitems[k]) continue;
      std::vector<uint64_t> raw((size_t)grid[k] * kProfCounters);
      if ((e = hipMemcpy(raw.data(), src, raw.size() * 8, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "copy phase timers");
      for (size_t i = 0; i < raw.size(); ++i) h_prof[i % kProfCounters] += raw[i];
      prof_slots += grid[k];
    }
  }
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->ms_device = ms_all;
    st->ms_traverse = ms_tr;
    st->ms_mapback = ms_mb;
    st->ms_host = last_host_ms + (wall_ms() - t0);
    st->teps = teps;
    st->algo_bytes = algo_bytes;
    st->items = total_items;
    st->batched_sources = sources_in[KC_BATCH] + sources_in[KC_DEEP] + sources_in[KC_TEAM];
    st->lds_sources = sources_in[KC_WAVE];
    st->global_sources = 0;
    st->overflow = flags;
    for (int k = 0; k < KC_COUNT; ++k) {
      st->ms_class[k] = class_ms[k];
      st->bytes_class[k] = bytes_k[k];
      st->teps_class[k] = teps_k[k];
      st->grid_class[k] = nitems[k] ? grid[k] : 0;
      st->items_class[k] = nitems[k];
    }
  }
  if (flags & kFlagTeamTimeout) return fail(SBC_E_DEVICE, "a team barrier wait timed out (team kernel aborted)");
  if (flags & kFlagRangeMask)
    return fail(SBC_E_DEVICE, "device-side range check failed (flags " + std::to_string(flags) + ")");
  if (flags & kFlagQueueOverflow) return fail(SBC_E_TOO_LARGE, "traversal queue overflow");
  if (flags & kFlagHeavyOverflow) return fail(SBC_E_DEVICE, "more long rows in a level than the split lists hold");
  if (flags & kFlagSigmaOverflow)
    return fail(SBC_E_SIGMA_OVERFLOW, "a shortest-path count exceeded the binary64 range");
  int32_t done_total = 0;
  for (int k = 0; k < KC_COUNT; ++k) done_total += h_ctl[kCtlDone + k];
  if (done_total != total_items)
    return fail(SBC_E_DEVICE, "work queue drained " + std::to_string(done_total) + " of " +
                                  std::to_string(total_items) + " items");

  return SBC_OK;
}

}  // namespace sbc
