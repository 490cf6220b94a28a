// The C interface declared in include/shatterbc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <string>

#include "runtime.hpp"
#include "shatterbc.h"

namespace sbc {
const std::string& last_error();
}

using namespace sbc;

#define SBC_TRY(body)                                        \
  try {                                                      \
    body                                                     \
  } catch (const std::bad_alloc&) {                          \
    return fail(SBC_E_OOM, "host allocation failed");        \
  } catch (const std::exception& ex) {                       \
    return fail(SBC_E_INVALID_ARG, ex.what());               \
  } catch (...) {                                            \
    return fail(SBC_E_INVALID_ARG, "unexpected exception");  \
  }

extern "C" {

const char* sbc_status_string(sbc_status s) {
  switch (s) {
    case SBC_OK: return "ok";
    case SBC_E_INVALID_ARG: return "invalid argument";
    case SBC_E_NOT_SYMMETRIC: return "graph is not symmetric";
    case SBC_E_SELF_LOOP: return "graph has a self loop";
    case SBC_E_DUP_EDGE: return "graph has a duplicate arc";
    case SBC_E_INDEX_RANGE: return "index out of range";
    case SBC_E_TOO_LARGE: return "problem too large";
    case SBC_E_OOM: return "out of memory";
    case SBC_E_DEVICE: return "device error";
    case SBC_E_SIGMA_OVERFLOW: return "shortest-path count overflow";
    case SBC_E_CANCELLED: return "cancelled";
    case SBC_E_NOT_READY: return "not ready";
    case SBC_E_NO_DEVICE: return "no usable gfx950 device";
    default: return "unknown status";
  }
}

const char* sbc_last_error(void) { return sbc::last_error().c_str(); }

const char* sbc_version(void) { return "shatterbc 0.1 (gfx950)"; }

sbc_status sbc_context_create(int device, sbc_context* out) {
  if (!out) return fail(SBC_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return fail(SBC_E_NO_DEVICE, "no HIP device visible");
  }
  if (device < 0 || device >= count) return fail(SBC_E_NO_DEVICE, "device ordinal out of range");
  SBC_TRY({
    std::unique_ptr<sbc_context_s> c(new sbc_context_s());
    c->device = device;
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    if ((e = hipGetDeviceProperties(&c->prop, device)) != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(c->prop.gcnArchName, "gfx950", 6) != 0)
      return fail(SBC_E_NO_DEVICE, std::string("device is ") + c->prop.gcnArchName + ", this library is built for gfx950");
    c->cus = c->prop.multiProcessorCount;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
      c->lds_limit = std::min<size_t>((size_t)lds, kMaxLdsBytes);
    int wclk = 0;
    if (hipDeviceGetAttribute(&wclk, hipDeviceAttributeWallClockRate, device) == hipSuccess && wclk > 0)
      c->wall_khz = wclk;
    (void)hipGetLastError();  // leave no stale error behind for later launch checks
    *out = c.release();
    return SBC_OK;
  })
}

sbc_status sbc_context_destroy(sbc_context ctx) {
  delete ctx;
  return SBC_OK;
}

static int64_t* param_slot(Params& p, const char* key) {
  const std::string k(key);
  if (k == "wave_max_vertices") return &p.wave_max_vertices;
  if (k == "batch_wg_waves") return &p.batch_wg_waves;
  if (k == "batch_waves_per_eu") return &p.batch_waves_per_eu;
  if (k == "wave_sources_per_item") return &p.wave_sources_per_item;
  if (k == "wave_wg_waves") return &p.wave_wg_waves;
  if (k == "slots") return &p.slots;
  if (k == "cluster_sources") return &p.cluster_sources;
  if (k == "batch_pairs") return &p.batch_pairs;
  if (k == "batch_compact") return &p.batch_compact;
  if (k == "deep_min_levels") return &p.deep_min_levels;
  if (k == "deep_wg_waves") return &p.deep_wg_waves;
  if (k == "deep_waves_per_eu") return &p.deep_waves_per_eu;
  if (k == "mem_budget_mb") return &p.mem_budget_mb;
  if (k == "profile_phases") return &p.profile_phases;
  if (k == "order_plain") return &p.order_plain;
  if (k == "team_min_vertices") return &p.team_min_vertices;
  if (k == "team_count") return &p.team_count;
  if (k == "team_wg_waves") return &p.team_wg_waves;
  if (k == "team_waves_per_eu") return &p.team_waves_per_eu;
  if (k == "team_spin_ms") return &p.team_spin_ms;
  if (k == "team_local_fences") return &p.team_local_fences;
  if (k == "team_cooperative") return &p.team_cooperative;
  if (k == "team_split_arcs") return &p.team_split_arcs;
  if (k == "team_max_levels") return &p.team_max_levels;
  if (k == "sample_items") return &p.sample_items;
  if (k == "far_wg_waves") return &p.far_wg_waves;
  if (k == "server_order") return &p.server_order;
  if (k == "server_max_wait_ms") return &p.server_max_wait_ms;
  return nullptr;
}

sbc_status sbc_context_set_param(sbc_context ctx, const char* key, int64_t value) {
  if (!ctx || !key) return fail(SBC_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  int64_t* slot = param_slot(ctx->params, key);
  if (!slot) return fail(SBC_E_INVALID_ARG, std::string("unknown parameter ") + key);
  const std::string k(key);
  bool ok = value >= 0;
  if (k == "batch_wg_waves") ok = value == 4 || value == 8 || value == 16;
  if (k == "batch_waves_per_eu") ok = value == 0 || value == 6 || value == 8;
  if (k == "deep_wg_waves") ok = value == 4 || value == 8 || value == 16;
  if (k == "far_wg_waves") ok = value == 4 || value == 8 || value == 16;
  if (k == "deep_waves_per_eu") ok = value == 0 || value == 6 || value == 8;
  if (k == "team_waves_per_eu") ok = value == 0 || value == 8;
  if (k == "team_wg_waves") ok = value == 4 || value == 8 || value == 16;
  if (k == "team_count") ok = value >= 1 && value <= 1024;
  if (k == "cluster_sources") ok = value >= 0 && value <= 2;
  if (k == "batch_pairs") ok = value >= 0 && value <= 64;
  if (k == "batch_compact") ok = value == 0 || value == 1;
  if (k == "team_spin_ms") ok = value <= 600000;
  if (k == "team_local_fences") ok = value == 0 || value == 1;
  if (k == "team_cooperative") ok = value == 0 || value == 1;
  if (k == "server_order") ok = value == 0 || value == 1;
  if (k == "team_split_arcs") ok = value >= 64 && value <= (1 << 30);
  if (k == "wave_max_vertices") ok = value >= 0 && value <= kWaveMaxVertices;
  if (k == "wave_wg_waves") ok = value == 4 || value == 8;
  if (k == "wave_sources_per_item") ok = value >= 1 && value <= 64;
  if (!ok) return fail(SBC_E_INVALID_ARG, std::string("value out of range for ") + key);
  *slot = value;
  return SBC_OK;
}

sbc_status sbc_context_get_param(sbc_context ctx, const char* key, int64_t* value) {
  if (!ctx || !key || !value) return fail(SBC_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (std::string(key) == "cus") {
    *value = ctx->cus;
    return SBC_OK;
  }
  if (std::string(key) == "lds_limit_bytes") {
    *value = (int64_t)ctx->lds_limit;
    return SBC_OK;
  }
  int64_t* slot = param_slot(ctx->params, key);
  if (!slot) return fail(SBC_E_INVALID_ARG, std::string("unknown parameter ") + key);
  *value = *slot;
  return SBC_OK;
}

sbc_status sbc_context_device_name(sbc_context ctx, char* buf, size_t len) {
  if (!ctx || !buf || len == 0) return fail(SBC_E_INVALID_ARG, "NULL argument");
  const char* nm = ctx->prop.name[0] ? ctx->prop.name : ctx->prop.gcnArchName;
  std::strncpy(buf, nm, len - 1);
  buf[len - 1] = 0;
  return SBC_OK;
}

sbc_status sbc_graph_create(int32_t n, const int32_t* row_ptr, const int32_t* col, uint32_t flags, sbc_graph* out) {
  if (!out) return fail(SBC_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (flags & ~SBC_SANITIZE) return fail(SBC_E_INVALID_ARG, "unknown flag");
  SBC_TRY({
    std::unique_ptr<sbc_graph_s> g(new sbc_graph_s());
    std::string why;
    int rc = validate_csr(n, row_ptr, col, (flags & SBC_SANITIZE) != 0, &g->g, &why);
    if (rc != SBC_OK) return fail(rc, why);
    *out = g.release();
    return SBC_OK;
  })
}

sbc_status sbc_graph_destroy(sbc_graph g) {
  delete g;
  return SBC_OK;
}

sbc_status sbc_graph_info(sbc_graph g, int32_t* n, int64_t* arcs) {
  if (!g) return fail(SBC_E_INVALID_ARG, "graph is NULL");
  if (n) *n = g->g.n;
  if (arcs) *arcs = g->g.arcs();
  return SBC_OK;
}

sbc_status sbc_graph_preprocess(sbc_graph g, const char* ops, sbc_prep_stats* st) {
  if (!g || !ops) return fail(SBC_E_INVALID_ARG, "NULL argument");
  SBC_TRY({
    PrepStats ps;
    std::string why;
    Prepared prep;
    int rc = preprocess(g->g, ops, &prep, &ps, &why);
    if (rc != SBC_OK) return fail(rc, why);
    g->prep = std::move(prep);
    g->prepared = true;
    g->ops = ops;
    sbc_prep_stats s{};
    s.n = ps.n;
    s.m = ps.m;
    s.components = ps.components;
    s.stripped = ps.stripped;
    s.blocks = ps.blocks;
    s.bridges = ps.bridges;
    s.twin_classes = ps.twin_classes;
    s.twins_merged = ps.twins_merged;
    s.tiny_pieces = ps.tiny_pieces;
    s.pieces = ps.pieces;
    s.piece_vertices = ps.piece_vertices;
    s.piece_arcs = ps.piece_arcs;
    s.work_teps = ps.work_teps;
    s.ms_degree1 = ps.ms_degree1;
    s.ms_shatter = ps.ms_shatter;
    s.ms_twins = ps.ms_twins;
    s.ms_pack = ps.ms_pack;
    s.side_vertices = ps.side_vertices;
    s.side_pieces = ps.side_pieces;
    g->stats = s;
    if (st) *st = s;
    return SBC_OK;
  })
}

sbc_status sbc_graph_export_sizes(sbc_graph g, int64_t* P, int64_t* V, int64_t* A, int64_t* M) {
  if (!g) return fail(SBC_E_INVALID_ARG, "graph is NULL");
  if (!g->prepared) return fail(SBC_E_INVALID_ARG, "graph has not been preprocessed");
  if (P) *P = g->prep.pieces();
  if (V) *V = g->prep.V();
  if (A) *A = g->prep.A();
  if (M) *M = (int64_t)g->prep.map_idx.size();
  return SBC_OK;
}

sbc_status sbc_graph_export(sbc_graph g, int32_t* vtx_off, int32_t* row, int32_t* col, int32_t* reach,
                            int32_t* ident, double* corr, double* bcx, int32_t* map_off, int32_t* map_idx) {
  if (!g) return fail(SBC_E_INVALID_ARG, "graph is NULL");
  if (!g->prepared) return fail(SBC_E_INVALID_ARG, "graph has not been preprocessed");
  const Prepared& p = g->prep;
  auto cp = [](auto* dst, const auto& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
  };
  cp(vtx_off, p.vtx_off);
  cp(row, p.row);
  cp(col, p.col);
  cp(reach, p.reach);
  cp(ident, p.ident);
  cp(corr, p.corr);
  cp(bcx, p.bcx);
  cp(map_off, p.map_off);
  cp(map_idx, p.map_idx);
  return SBC_OK;
}

sbc_status sbc_graph_export_side(sbc_graph g, int32_t* nside) {
  if (!g || !nside) return fail(SBC_E_INVALID_ARG, "NULL argument");
  if (!g->prepared) return fail(SBC_E_INVALID_ARG, "graph has not been preprocessed");
  const Prepared& p = g->prep;
  for (int32_t i = 0; i < p.pieces(); ++i) nside[i] = i < (int32_t)p.nside.size() ? p.nside[i] : 0;
  return SBC_OK;
}

static sbc_status ensure_problem(sbc_context ctx, sbc_graph g, uint32_t mode, Prepared* plain_storage,
                                 const Prepared** out) {
  if (mode & SBC_COMPRESSED) {
    if (!g->prepared) {
      sbc_status rc = sbc_graph_preprocess(g, "odai", nullptr);
      if (rc != SBC_OK) return rc;
    }
    *out = &g->prep;
  } else {
    plain_problem(g->g, plain_storage);
    if (ctx->params.order_plain) order_pieces(plain_storage);
    *out = plain_storage;
  }
  return SBC_OK;
}

sbc_status sbc_plan_create(sbc_context ctx, sbc_graph g, uint32_t mode, sbc_plan* out) {
  if (!ctx || !g || !out) return fail(SBC_E_INVALID_ARG, "NULL argument");
  if (mode & ~(SBC_COMPRESSED | SBC_UNORDERED | SBC_DETERMINISTIC)) return fail(SBC_E_INVALID_ARG, "unknown mode bit");
  *out = nullptr;
  SBC_TRY({
    Prepared plain;
    const Prepared* prob = nullptr;
    sbc_status rc = ensure_problem(ctx, g, mode, &plain, &prob);
    if (rc != SBC_OK) return rc;
    std::unique_ptr<sbc_plan_s> p(new sbc_plan_s());
    rc = p->plan.build(ctx, *prob, mode, PlanOptions());
    if (rc != SBC_OK) return rc;
    *out = p.release();
    return SBC_OK;
  })
}

sbc_status sbc_plan_destroy(sbc_plan p) {
  if (p) {
    (void)hipSetDevice(p->plan.ctx->device);
    if (p->plan.ran) (void)hipEventSynchronize(p->plan.ev_end);
  }
  delete p;
  return SBC_OK;
}

sbc_status sbc_plan_execute(sbc_plan p, double* bc_dev, void* stream) {
  if (!p) return fail(SBC_E_INVALID_ARG, "plan is NULL");
  SBC_TRY({ return p->plan.execute(bc_dev, (hipStream_t)stream); })
}

sbc_status sbc_plan_sync(sbc_plan p, sbc_run_stats* st) {
  if (!p) return fail(SBC_E_INVALID_ARG, "plan is NULL");
  SBC_TRY({ return p->plan.sync(st); })
}

sbc_status sbc_plan_result(sbc_plan p, double* bc_host) {
  if (!p || !bc_host) return fail(SBC_E_INVALID_ARG, "NULL argument");
  sbc_status rc = p->plan.sync(nullptr);
  if (rc != SBC_OK) return rc;
  hipError_t e = hipMemcpy(bc_host, p->plan.d_out.p, sizeof(double) * p->plan.n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "copy result");
  return SBC_OK;
}

sbc_status sbc_plan_phase_profile(sbc_plan p, double* out, int32_t count) {
  if (!p || !out || count < 0) return fail(SBC_E_INVALID_ARG, "NULL argument");
  const Plan& pl = p->plan;
  if (pl.h_prof.empty()) return fail(SBC_E_INVALID_ARG, "the plan kept no phase timers");
  const double slots = pl.prof_slots > 0 ? (double)pl.prof_slots : 1.0;
  for (int32_t i = 0; i < count && i < kProfCounters; ++i) {
    const double v = (double)pl.h_prof[i];
    const bool is_time = i < kProfItems || i == kProfSync;
    out[i] = is_time ? v / pl.ctx->wall_khz / slots : v;
  }
  return SBC_OK;
}

sbc_status sbc_plan_team_layout(sbc_plan p, int32_t* sizes, int32_t* xcc_masks, int32_t cap, int32_t* nteams) {
  if (!p || !nteams || cap < 0 || (cap > 0 && (!sizes || !xcc_masks))) return fail(SBC_E_INVALID_ARG, "bad argument");
  Plan& pl = p->plan;
  *nteams = 0;
  if (!pl.nitems[KC_TEAM]) return SBC_OK;
  if (!pl.ran) return fail(SBC_E_INVALID_ARG, "plan has not been executed");
  hipError_t e = hipSetDevice(pl.ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = hipEventSynchronize(pl.ev_end)) != hipSuccess) return hip_fail(e, "sync");
  std::vector<TeamCtl> c((size_t)pl.targs.nteams);
  if ((e = hipMemcpy(c.data(), pl.targs.ctl, c.size() * sizeof(TeamCtl), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "copy team control");
  *nteams = pl.targs.nteams;
  for (int32_t t = 0; t < pl.targs.nteams && t < cap; ++t) {
    sizes[t] = c[t].join;
    xcc_masks[t] = c[t].xccmask;
  }
  return SBC_OK;
}

sbc_status sbc_plan_use_graph(sbc_plan p, int enable) {
  if (!p) return fail(SBC_E_INVALID_ARG, "plan is NULL");
  if (p->plan.ran) (void)hipEventSynchronize(p->plan.ev_end);
  p->plan.use_graph = enable != 0;
  return SBC_OK;
}

sbc_status sbc_copy_bandwidth(sbc_context ctx, size_t bytes, int reps, double* gbps) {
  if (!ctx || !gbps || reps < 1 || bytes < 16) return fail(SBC_E_INVALID_ARG, "bad argument");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  bytes &= ~(size_t)15;
  DevBuf a, b;
  if ((e = a.alloc(bytes)) != hipSuccess || (e = b.alloc(bytes)) != hipSuccess) return hip_fail(e, "alloc");
  hipStream_t s = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  sbc_status rc = SBC_OK;
  if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
  if ((e = hipEventCreate(&t0)) == hipSuccess && (e = hipEventCreate(&t1)) == hipSuccess) {
    const int grid = ctx->cus * 8;
    e = launch_fill_u64(a.as<uint64_t>(), 0x0123456789abcdefull, (int64_t)(bytes / 8), s);
    if (e == hipSuccess) e = launch_copy(a.p, b.p, (int64_t)bytes, grid, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(t0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_copy(a.p, b.p, (int64_t)bytes, grid, s);
    if (e == hipSuccess) e = hipEventRecord(t1, s);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (e == hipSuccess) *gbps = ms > 0 ? 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9 : 0.0;
  }
  if (e != hipSuccess) rc = hip_fail(e, "copy bandwidth");
  if (s) (void)hipStreamSynchronize(s);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (s) (void)hipStreamDestroy(s);
  return rc;
}

sbc_status sbc_betweenness(sbc_context ctx, sbc_graph g, uint32_t mode, double* bc_host, sbc_run_stats* st) {
  if (!ctx || !g || !bc_host) return fail(SBC_E_INVALID_ARG, "NULL argument");
  sbc_plan p = nullptr;
  sbc_status rc = sbc_plan_create(ctx, g, mode, &p);
  if (rc != SBC_OK) return rc;
  rc = sbc_plan_execute(p, nullptr, nullptr);
  if (rc == SBC_OK) rc = sbc_plan_sync(p, st);
  if (rc == SBC_OK) rc = sbc_plan_result(p, bc_host);
  sbc_plan_destroy(p);
  return rc;
}

sbc_status sbc_betweenness_device(sbc_context ctx, sbc_graph g, uint32_t mode, double* bc_dev, void* stream,
                                  sbc_run_stats* st) {
  if (!ctx || !g || !bc_dev) return fail(SBC_E_INVALID_ARG, "NULL argument");
  sbc_plan p = nullptr;
  sbc_status rc = sbc_plan_create(ctx, g, mode, &p);
  if (rc != SBC_OK) return rc;
  rc = sbc_plan_execute(p, bc_dev, stream);
  if (rc == SBC_OK) rc = sbc_plan_sync(p, st);
  sbc_plan_destroy(p);
  return rc;
}

sbc_status sbc_betweenness_sources(sbc_context ctx, sbc_graph g, int64_t nsrc, const int32_t* sources,
                                   double* bc_host, sbc_run_stats* st) {
  if (!ctx || !g || !bc_host || (nsrc > 0 && !sources) || nsrc < 0)
    return fail(SBC_E_INVALID_ARG, "NULL argument or negative count");
  if (nsrc > g->g.n) return fail(SBC_E_INVALID_ARG, "more sources than vertices");
  SBC_TRY({
    if (nsrc == 0) {
      std::memset(bc_host, 0, sizeof(double) * g->g.n);
      return SBC_OK;
    }
    Prepared plain;
    plain_problem(g->g, &plain);
    PlanOptions opt;
    opt.sources = sources;
    opt.nsrc = nsrc;
    Plan plan;
    sbc_status rc = plan.build(ctx, plain, SBC_PLAIN, opt);
    if (rc != SBC_OK) return rc;
    if ((rc = plan.execute(nullptr, nullptr)) != SBC_OK) return rc;
    if ((rc = plan.sync(st)) != SBC_OK) return rc;
    hipError_t e = hipMemcpy(bc_host, plan.d_out.p, sizeof(double) * plan.n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "copy result");
    return SBC_OK;
  })
}

// One attributed piece as a single-piece problem.
static sbc_status piece_problem(int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* reach,
                                const int32_t* ident, Prepared* out) {
  HostGraph hg;
  std::string why;
  int rc = validate_csr(n, row_ptr, col, false, &hg, &why);
  if (rc != SBC_OK) return fail(rc, why);
  if (n < 1) return fail(SBC_E_INVALID_ARG, "empty piece");
  plain_problem(hg, out);
  // Internally a piece vertex carries the reach of its members together:
  // ident[v] members of reach reach[v] each.
  for (int32_t v = 0; v < n; ++v) {
    const int64_t r = reach ? reach[v] : 1, k = ident ? ident[v] : 1;
    if (r < 1) return fail(SBC_E_INVALID_ARG, "reach must be >= 1");
    if (k < 1) return fail(SBC_E_INVALID_ARG, "ident must be >= 1");
    if (r * k > INT32_MAX) return fail(SBC_E_TOO_LARGE, "reach x ident exceeds 2^31 - 1");
    out->reach[v] = (int32_t)(r * k);
    out->ident[v] = (int32_t)k;
    if (r > 1) out->weighted = true;
    if (k > 1) out->has_ident = true;
  }
  return SBC_OK;
}

sbc_status sbc_piece_bc(sbc_context ctx, int32_t n, const int32_t* row_ptr, const int32_t* col, const int32_t* reach,
                        const int32_t* ident, int kernel, double* bc_host, sbc_run_stats* st) {
  if (!ctx || !bc_host) return fail(SBC_E_INVALID_ARG, "NULL argument");
  if (kernel == 1 || kernel == 2)
    return fail(SBC_E_INVALID_ARG, "kernels 1 and 2 (one source per workgroup) are not part of this library");
  if (kernel < 0 || kernel > 5) return fail(SBC_E_INVALID_ARG, "kernel must be 0, 3, 4 or 5");
  SBC_TRY({
    Prepared prob;
    sbc_status rc = piece_problem(n, row_ptr, col, reach, ident, &prob);
    if (rc != SBC_OK) return rc;
    PlanOptions opt;
    opt.force_kernel = kernel;
    Plan plan;
    // weighted single piece: compressed-mode kernels (REACH/IDENT picked from the data)
    rc = plan.build(ctx, prob, SBC_COMPRESSED, opt);
    if (rc != SBC_OK) return rc;
    if ((rc = plan.execute(nullptr, nullptr)) != SBC_OK) return rc;
    if ((rc = plan.sync(st)) != SBC_OK) return rc;
    hipError_t e = hipMemcpy(bc_host, plan.d_bcp.p, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "copy result");
    return SBC_OK;
  })
}

sbc_status sbc_sources_state(sbc_context ctx, int32_t n, const int32_t* row_ptr, const int32_t* col,
                             const int32_t* reach, const int32_t* ident, int32_t nsrc, const int32_t* sources,
                             int kernel, int32_t* dist, double* sigma, double* delta) {
  if (!ctx || !sources) return fail(SBC_E_INVALID_ARG, "NULL argument");
  if (n < 1 || nsrc < 1 || nsrc > n) return fail(SBC_E_INVALID_ARG, "need 1 <= nsrc <= n");
  if (kernel != 0 && kernel != 3 && kernel != 4 && kernel != 5)
    return fail(SBC_E_INVALID_ARG, "kernel must be 0, 3, 4 or 5");
  if ((int64_t)nsrc * (int64_t)n >= ((int64_t)1 << 31)) return fail(SBC_E_TOO_LARGE, "nsrc x n must stay below 2^31");
  SBC_TRY({
    Prepared prob;
    sbc_status rc = piece_problem(n, row_ptr, col, reach, ident, &prob);
    if (rc != SBC_OK) return rc;
    PlanOptions opt;
    opt.force_kernel = kernel;
    opt.sources = sources;
    opt.nsrc = nsrc;
    opt.dump = true;
    Plan plan;
    rc = plan.build(ctx, prob, SBC_COMPRESSED, opt);
    if (rc != SBC_OK) return rc;
    if ((rc = plan.execute(nullptr, nullptr)) != SBC_OK) return rc;
    if ((rc = plan.sync(nullptr)) != SBC_OK) return rc;
    const size_t cells = (size_t)nsrc * (size_t)n;
    hipError_t e = hipSuccess;
    if (dist && e == hipSuccess) e = hipMemcpy(dist, plan.dump.dist, sizeof(int32_t) * cells, hipMemcpyDeviceToHost);
    if (sigma && e == hipSuccess) e = hipMemcpy(sigma, plan.dump.sigma, sizeof(double) * cells, hipMemcpyDeviceToHost);
    if (delta && e == hipSuccess) e = hipMemcpy(delta, plan.dump.delta, sizeof(double) * cells, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "copy result");
    return SBC_OK;
  })
}

sbc_status sbc_single_source(sbc_context ctx, int32_t n, const int32_t* row_ptr, const int32_t* col,
                             const int32_t* reach, const int32_t* ident, int32_t s, int32_t* dist, double* sigma,
                             double* delta) {
  if (!ctx) return fail(SBC_E_INVALID_ARG, "NULL context");
  if (s < 0 || s >= n) return fail(SBC_E_INDEX_RANGE, "source out of range");
  return sbc_sources_state(ctx, n, row_ptr, col, reach, ident, 1, &s, 0, dist, sigma, delta);
}

}  // extern "C"
