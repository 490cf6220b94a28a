// The closeness interface (include/shatterbc.h, "farness and closeness"):
// host preparation of the shattered pieces, the device's per-piece sums and
// the host pass over the block-cut tree (far.hpp, far.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "far.hpp"
#include "runtime.hpp"
#include "shatterbc.h"

using namespace sbc;

struct sbc_far_s {
  FarPrepared F;
};

namespace {

double wall_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// The per-piece sums W on the device: one persistent launch of the farness
// kernel over 64-source items, largest pieces first.
sbc_status far_device(sbc_context ctx, const FarPrepared& F, std::vector<int64_t>* W, sbc_far_run_stats* st) {
  const int32_t P = F.pieces();
  const int64_t V = F.V(), A = F.A();
  W->assign((size_t)V, 0);
  if (P == 0 || V == 0) return SBC_OK;
  if (V >= INT32_MAX || A >= INT32_MAX) return fail(SBC_E_TOO_LARGE, "pieces exceed 32-bit offsets");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  const Params pr = [&] {
    std::lock_guard<std::mutex> lk(ctx->mu);
    return ctx->params;
  }();
  int32_t max_np = 0;
  std::vector<int32_t> order(P);
  for (int32_t p = 0; p < P; ++p) {
    order[p] = p;
    max_np = std::max(max_np, F.vtx_off[p + 1] - F.vtx_off[p]);
  }
  auto work = [&](int32_t p) {
    const int64_t np = F.vtx_off[p + 1] - F.vtx_off[p];
    return (double)np * (double)(F.row[F.vtx_off[p + 1]] - F.row[F.vtx_off[p]] + np);
  };
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return work(a) > work(b); });
  std::vector<WorkItem> items;
  for (int32_t p : order) {
    const int32_t np = F.vtx_off[p + 1] - F.vtx_off[p];
    for (int32_t s0 = 0; s0 < np; s0 += 64) items.push_back({p, s0, std::min(np, s0 + 64), 0});
  }
  const int32_t nitems = (int32_t)items.size();

  const int waves = (int)pr.far_wg_waves;
  const int occ = occupancy_far(waves);
  if (occ <= 0) return fail(SBC_E_INVALID_ARG, "farness kernel configuration cannot be resident");
  const int64_t stride = max_np;
  const int64_t qcap = stride * 64;
  const size_t per_slot = (size_t)qcap * 4 + 3 * (size_t)stride * 8;
  size_t freeb = 0, totalb = 0;
  (void)hipMemGetInfo(&freeb, &totalb);
  const size_t budget = pr.mem_budget_mb > 0 ? (size_t)pr.mem_budget_mb << 20 : (size_t)(freeb * 0.6);
  const size_t fixed = (size_t)(P + 1) * 4 + (size_t)(V + 1) * 4 + (size_t)A * 4 + (size_t)V * 8 + (size_t)V * 8 +
                       (size_t)nitems * sizeof(WorkItem) + 64;
  if (fixed + per_slot > budget) return fail(SBC_E_OOM, "farness problem does not fit the memory budget");
  int64_t grid = (int64_t)ctx->cus * occ;
  if (pr.slots > 0) grid = pr.slots;
  grid = std::min<int64_t>({grid, (int64_t)nitems, (int64_t)((budget - fixed) / per_slot)});
  grid = std::max<int64_t>(grid, 1);

  DevBuf d_vtx, d_row, d_col, d_reach, d_src, d_items, d_out, d_ctl, d_q, d_vis, d_fa, d_fb;
  if ((e = d_vtx.alloc(sizeof(int32_t) * (P + 1))) != hipSuccess || (e = d_row.alloc(sizeof(int32_t) * (V + 1))) != hipSuccess ||
      (e = d_col.alloc(sizeof(int32_t) * std::max<int64_t>(A, 1))) != hipSuccess ||
      (e = d_items.alloc(sizeof(WorkItem) * nitems)) != hipSuccess || (e = d_out.alloc(sizeof(int64_t) * V)) != hipSuccess ||
      (e = d_src.alloc(sizeof(int32_t) * V)) != hipSuccess ||
      (e = d_ctl.alloc(sizeof(int32_t) * 4)) != hipSuccess ||
      (e = d_q.alloc(sizeof(int32_t) * (size_t)qcap * grid)) != hipSuccess ||
      (e = d_vis.alloc(sizeof(uint64_t) * (size_t)stride * grid)) != hipSuccess ||
      (e = d_fa.alloc(sizeof(uint64_t) * (size_t)stride * grid)) != hipSuccess ||
      (e = d_fb.alloc(sizeof(uint64_t) * (size_t)stride * grid)) != hipSuccess)
    return hip_fail(e, "device allocation");
  if (F.weighted && (e = d_reach.alloc(sizeof(int32_t) * V)) != hipSuccess) return hip_fail(e, "device allocation");
  hipStream_t s = nullptr;
  if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  struct Guard {
    hipStream_t s;
    hipEvent_t a, b;
    ~Guard() {
      if (s) (void)hipStreamSynchronize(s);
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
      if (s) (void)hipStreamDestroy(s);
    }
  } guard{s, nullptr, nullptr};
  if ((e = hipEventCreate(&ev0)) != hipSuccess) return hip_fail(e, "event");
  guard.a = ev0;
  if ((e = hipEventCreate(&ev1)) != hipSuccess) return hip_fail(e, "event");
  guard.b = ev1;

  const double t0 = wall_ms();
  auto up = [&](DevBuf& d, const void* h, size_t bytes) {
    return bytes ? hipMemcpyAsync(d.p, h, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
  };
  if ((e = up(d_vtx, F.vtx_off.data(), sizeof(int32_t) * (P + 1))) != hipSuccess ||
      (e = up(d_row, F.row.data(), sizeof(int32_t) * (V + 1))) != hipSuccess ||
      (e = up(d_col, F.col.data(), sizeof(int32_t) * A)) != hipSuccess ||
      (e = up(d_items, items.data(), sizeof(WorkItem) * nitems)) != hipSuccess ||
      (e = up(d_src, F.src_order.data(), sizeof(int32_t) * V)) != hipSuccess ||
      (F.weighted && (e = up(d_reach, F.reach.data(), sizeof(int32_t) * V)) != hipSuccess))
    return hip_fail(e, "upload");
  // Masks start at zero (the kernel leaves them so); the control words too.
  if ((e = launch_fill_u64(d_vis.as<uint64_t>(), 0, stride * grid, s)) != hipSuccess ||
      (e = launch_fill_u64(d_fa.as<uint64_t>(), 0, stride * grid, s)) != hipSuccess ||
      (e = launch_fill_u64(d_fb.as<uint64_t>(), 0, stride * grid, s)) != hipSuccess ||
      (e = launch_fill_i32(d_ctl.as<int32_t>(), 0, 4, s)) != hipSuccess)
    return hip_fail(e, "fill");
  int32_t* ctl = d_ctl.as<int32_t>();
  DevPieces dp{d_vtx.as<int32_t>(), d_row.as<int32_t>(), d_col.as<int32_t>(),
               F.weighted ? d_reach.as<int32_t>() : nullptr, nullptr, d_src.as<int32_t>(), nullptr, nullptr, P, (int32_t)V,
               (int32_t)A, 0};
  QueueArgs qa{d_items.as<WorkItem>(), nitems, kArgMagic, ctl + 0, ctl + 1, ctl + 2, nullptr, nullptr};
  FarState fs{d_q.as<int32_t>(), d_vis.as<uint64_t>(), d_fa.as<uint64_t>(), d_fb.as<uint64_t>(), stride, qcap};
  if ((e = hipEventRecord(ev0, s)) != hipSuccess) return hip_fail(e, "event");
  if ((e = launch_far(dp, qa, F.weighted, waves, (int)grid, fs, d_out.as<int64_t>(), s)) != hipSuccess)
    return hip_fail(e, "launch farness");
  if ((e = hipEventRecord(ev1, s)) != hipSuccess) return hip_fail(e, "event");
  int32_t h_ctl[4] = {0, 0, 0, 0};
  if ((e = hipMemcpyAsync(h_ctl, ctl, sizeof(h_ctl), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(W->data(), d_out.p, sizeof(int64_t) * V, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "download");
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, ev0, ev1);
  if (st) {
    st->ms_kernel = ms;
    st->ms_device_total = wall_ms() - t0;
    st->items = nitems;
    st->grid = grid;
    st->waves = waves;
    double teps = 0;  // sources x undirected edges, over the pieces
    for (int32_t p = 0; p < P; ++p)
      teps += (double)(F.vtx_off[p + 1] - F.vtx_off[p]) * 0.5 * (double)(F.row[F.vtx_off[p + 1]] - F.row[F.vtx_off[p]]);
    st->teps = ms > 0 ? teps / (ms * 1e-3) : 0.0;
    st->flags = h_ctl[1];
  }
  if (h_ctl[1] & kFlagQueueOverflow) return fail(SBC_E_DEVICE, "farness queue overflow");
  if (h_ctl[1] & (kFlagRangeMask | kFlagBadSource)) return fail(SBC_E_DEVICE, "farness kernel saw an out-of-range index");
  if (h_ctl[2] != nitems) return fail(SBC_E_DEVICE, "farness kernel did not finish every item");
  return SBC_OK;
}

}  // namespace

extern "C" {

sbc_status sbc_far_create(sbc_graph g, const char* ops, sbc_far* out, sbc_far_stats* st) {
  if (!g || !out) return fail(SBC_E_INVALID_ARG, "NULL argument");
  *out = nullptr;
  try {
    std::unique_ptr<sbc_far_s> f(new sbc_far_s());
    std::string why;
    const int rc = far_prepare(g->g, ops ? ops : "", &f->F, &why);
    if (rc != SBC_OK) return fail(rc, why);
    if (st) {
      const FarPrepared& F = f->F;
      *st = sbc_far_stats{};
      st->n = F.n;
      st->components = (int64_t)F.comp_size.size();
      st->stripped = F.stripped;
      st->blocks = F.nblocks;
      st->bridges = F.bridges;
      st->pieces = F.pieces();
      st->piece_vertices = F.V();
      st->piece_arcs = F.A();
      st->ms_prep = F.ms_prep;
    }
    *out = f.release();
  } catch (const std::bad_alloc&) {
    return fail(SBC_E_OOM, "host allocation failed");
  } catch (...) {
    return fail(SBC_E_INVALID_ARG, "unexpected exception");
  }
  return SBC_OK;
}

sbc_status sbc_far_destroy(sbc_far f) {
  delete f;
  return SBC_OK;
}

sbc_status sbc_far_info(sbc_far f, int32_t* pieces, int64_t* vertices, int64_t* arcs) {
  if (!f) return fail(SBC_E_INVALID_ARG, "NULL argument");
  if (pieces) *pieces = f->F.pieces();
  if (vertices) *vertices = f->F.V();
  if (arcs) *arcs = f->F.A();
  return SBC_OK;
}

sbc_status sbc_far_export(sbc_far f, int32_t* vtx_off, int32_t* row, int32_t* col, int32_t* reach, int32_t* orig) {
  if (!f) return fail(SBC_E_INVALID_ARG, "NULL argument");
  const FarPrepared& F = f->F;
  if (vtx_off) std::memcpy(vtx_off, F.vtx_off.data(), sizeof(int32_t) * F.vtx_off.size());
  if (row) std::memcpy(row, F.row.data(), sizeof(int32_t) * F.row.size());
  if (col && !F.col.empty()) std::memcpy(col, F.col.data(), sizeof(int32_t) * F.col.size());
  if (reach && !F.reach.empty()) std::memcpy(reach, F.reach.data(), sizeof(int32_t) * F.reach.size());
  if (orig && !F.orig.empty()) std::memcpy(orig, F.orig.data(), sizeof(int32_t) * F.orig.size());
  return SBC_OK;
}

sbc_status sbc_far_finish(sbc_far f, const int64_t* piece_sums, int64_t* farness, double* closeness) {
  if (!f || !farness) return fail(SBC_E_INVALID_ARG, "NULL argument");
  try {
    std::string why;
    const int rc = far_finish(f->F, piece_sums, farness, closeness, &why);
    if (rc != SBC_OK) return fail(rc, why);
  } catch (const std::bad_alloc&) {
    return fail(SBC_E_OOM, "host allocation failed");
  }
  return SBC_OK;
}

sbc_status sbc_far_run(sbc_context ctx, sbc_far f, int64_t* piece_sums, int64_t* farness, double* closeness,
                       sbc_far_run_stats* st) {
  if (!ctx || !f || !farness) return fail(SBC_E_INVALID_ARG, "NULL argument");
  if (st) *st = sbc_far_run_stats{};
  try {
    const double t0 = wall_ms();
    std::vector<int64_t> W;
    sbc_status rc = far_device(ctx, f->F, &W, st);
    if (rc != SBC_OK) return rc;
    if (piece_sums && !W.empty()) std::memcpy(piece_sums, W.data(), sizeof(int64_t) * W.size());
    std::string why;
    const double t1 = wall_ms();
    const int frc = far_finish(f->F, W.data(), farness, closeness, &why);
    if (frc != SBC_OK) return fail(frc, why);
    if (st) {
      st->ms_finish = wall_ms() - t1;
      st->ms_total = wall_ms() - t0;
    }
  } catch (const std::bad_alloc&) {
    return fail(SBC_E_OOM, "host allocation failed");
  }
  return SBC_OK;
}

}  // extern "C"
