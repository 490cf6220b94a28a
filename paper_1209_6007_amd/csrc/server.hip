// Continuously batching request loop.
//
// `slots` worker threads each take a waiting job, preprocess it on the host,
// then wait until its device footprint fits in the memory budget (a job that
// arrives while others run is admitted the moment a slot and enough memory
// are free).  Admitted jobs upload, run and copy back on their slot's
// streams, so the device overlaps the work of every admitted job.
//
// Each slot owns, from sbc_server_create on, a device arena (the budget
// divided among the slots), pinned staging memory and its streams and
// events.  A job's plan takes its device buffers from the arena and its
// copies go through the staging memory asynchronously on the slot's stream,
// so a job neither allocates nor frees device memory -- a release would wait
// for every other job's kernels -- and a finished small job is not held up
// by the long jobs beside it.
//
// Which waiting job a free worker takes (context parameter server_order):
// the oldest, or the one with the least estimated work, unless the oldest
// has waited longer than server_max_wait_ms.  The estimate is sources x arcs
// scaled by the graph's breadth-first depth from its highest-degree vertex:
// every level of a traversal costs barriers and, for 64-source batches, the
// sources' levels spread wider on deep graphs.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "runtime.hpp"
#include "shatterbc.h"

using namespace sbc;

namespace {
double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// n x arcs x (1 + depth / 16), depth from a breadth-first search of the
// highest-degree vertex's component.
double work_estimate(const HostGraph& g) {
  const int32_t n = g.n;
  if (n <= 0) return 0.0;
  int32_t start = 0;
  for (int32_t v = 1; v < n; ++v)
    if (g.row_ptr[v + 1] - g.row_ptr[v] > g.row_ptr[start + 1] - g.row_ptr[start]) start = v;
  std::vector<int32_t> d(n, -1), q;
  q.reserve(n);
  d[start] = 0;
  q.push_back(start);
  int32_t depth = 0;
  for (size_t h = 0; h < q.size(); ++h) {
    const int32_t v = q[h];
    for (int32_t e = g.row_ptr[v]; e < g.row_ptr[v + 1]; ++e) {
      const int32_t w = g.col[e];
      if (d[w] < 0) {
        d[w] = d[v] + 1;
        depth = d[w];
        q.push_back(w);
      }
    }
  }
  return (double)n * (double)g.arcs() * (1.0 + depth / 16.0);
}
}  // namespace

struct sbc_job_s {
  sbc_graph g = nullptr;
  uint32_t mode = 0;
  std::vector<double> result;
  sbc_status status = SBC_E_NOT_READY;
  std::string error;
  sbc_job_stats stats{};
  double est = 0;  // estimated work, for ordering the waiting jobs
  double t_submit = 0, t_start = 0, t_done = 0;
  bool done = false;
  std::mutex mu;
  std::condition_variable cv;
  std::atomic<int> refs{2};  // the caller's handle and the server's queue entry
};

static void job_unref(sbc_job j) {
  if (j->refs.fetch_sub(1) == 1) delete j;
}

struct sbc_server_s {
  sbc_context ctx = nullptr;
  int slots = 1;
  size_t budget = 0;
  size_t in_use = 0;
  int running = 0;
  std::deque<sbc_job> pending;
  std::mutex mu;
  std::condition_variable cv;
  bool stopping = false;
  std::vector<std::thread> workers;
  std::vector<SlotResources> res;  // per slot: arena, staging, streams, events
};

static constexpr size_t kStagingBytes = (size_t)64 << 20;

static void run_job(sbc_server s, int slot, sbc_job j) {
  sbc_status rc = SBC_OK;
  std::string err;
  size_t fp = 0;
  bool reserved = false;
  try {
    const Prepared* prob = nullptr;
    Prepared plain;
    if (j->mode & SBC_COMPRESSED) {
      if (!j->g->prepared) rc = sbc_graph_preprocess(j->g, "odai", nullptr);
      prob = &j->g->prep;
    } else {
      plain_problem(j->g->g, &plain);
      prob = &plain;
    }
    if (rc == SBC_OK) {
      fp = estimate_plan_bytes(s->ctx, *prob);
      // admission: wait until the footprint fits (always admit when idle)
      {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv.wait(lk, [&] { return s->in_use + fp <= s->budget || s->running == 0; });
        s->in_use += fp;
        s->running++;
        reserved = true;
      }
      j->t_start = now_ms();
      SlotResources& r = s->res[slot];
      r.reset();
      BorrowScope borrow(&r);  // outlives the plan: its buffers are the arena's
      PlanOptions opt;
      Plan plan;
      rc = plan.build(s->ctx, *prob, j->mode, opt);
      if (rc == SBC_OK) rc = plan.execute(nullptr, nullptr);
      sbc_run_stats st{};
      if (rc == SBC_OK) rc = plan.sync(&st);
      if (rc == SBC_OK) {
        j->result.resize(plan.n);
        const size_t bytes = sizeof(double) * plan.n;
        hipError_t e;
        if (r.staging_used + bytes <= r.staging_bytes) {  // through the staging memory, on the slot's stream
          char* h = r.staging + r.staging_used;
          e = hipMemcpyAsync(h, plan.d_out.p, bytes, hipMemcpyDeviceToHost, r.own);
          if (e == hipSuccess) e = hipStreamSynchronize(r.own);
          if (e == hipSuccess) std::memcpy(j->result.data(), h, bytes);
        } else {
          e = hipMemcpy(j->result.data(), plan.d_out.p, bytes, hipMemcpyDeviceToHost);
        }
        if (e != hipSuccess) rc = hip_fail(e, "copy result");
      }
      j->stats.teps = st.teps;
      j->stats.footprint_bytes = (int64_t)r.arena_used;
    }
  } catch (const std::bad_alloc&) {
    rc = fail(SBC_E_OOM, "host allocation failed");
  } catch (...) {
    rc = fail(SBC_E_INVALID_ARG, "unexpected exception in job");
  }
  if (rc != SBC_OK) err = sbc_last_error();
  if (reserved) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->in_use -= fp;
    s->running--;
  }
  s->cv.notify_all();
  {
    std::lock_guard<std::mutex> lk(j->mu);
    j->t_done = now_ms();
    if (j->t_start == 0) j->t_start = j->t_done;
    j->stats.submit_to_start_ms = j->t_start - j->t_submit;
    j->stats.start_to_done_ms = j->t_done - j->t_start;
    j->stats.latency_ms = j->t_done - j->t_submit;
    j->status = rc;
    j->error = err;
    j->done = true;
  }
  j->cv.notify_all();
}

static void worker_loop(sbc_server s, int slot) {
  (void)hipSetDevice(s->ctx->device);
  while (true) {
    sbc_job j = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] { return s->stopping || !s->pending.empty(); });
      if (s->pending.empty()) {
        if (s->stopping) return;
        continue;
      }
      auto pick = s->pending.begin();
      const Params& pr = s->ctx->params;
      if (pr.server_order == 1 && now_ms() - (*pick)->t_submit <= (double)pr.server_max_wait_ms)
        for (auto it = s->pending.begin(); it != s->pending.end(); ++it)
          if ((*it)->est < (*pick)->est) pick = it;  // ties: the older job
      j = *pick;
      s->pending.erase(pick);
    }
    run_job(s, slot, j);
    job_unref(j);
  }
}

extern "C" {

sbc_status sbc_server_create(sbc_context ctx, int slots, size_t hbm_budget_bytes, sbc_server* out) {
  if (!ctx || !out || slots < 1 || slots > 64) return fail(SBC_E_INVALID_ARG, "bad argument");
  *out = nullptr;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  size_t freeb = 0, totalb = 0;
  (void)hipMemGetInfo(&freeb, &totalb);
  try {
    std::unique_ptr<sbc_server_s> s(new sbc_server_s());
    s->ctx = ctx;
    s->slots = slots;
    s->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(freeb * 0.8);
    s->res.resize(slots);
    for (int i = 0; i < slots; ++i) {
      if ((e = s->res[i].create(s->budget / (size_t)slots, kStagingBytes)) != hipSuccess) {
        for (auto& r : s->res) r.destroy();
        (void)hipGetLastError();
        return hip_fail(e, "server slot memory");
      }
    }
    for (int i = 0; i < slots; ++i) s->workers.emplace_back(worker_loop, s.get(), i);
    *out = s.release();
  } catch (...) {
    return fail(SBC_E_OOM, "could not start the server");
  }
  return SBC_OK;
}

sbc_status sbc_server_destroy(sbc_server s) {
  if (!s) return SBC_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv.notify_all();
  for (auto& t : s->workers) t.join();
  (void)hipSetDevice(s->ctx->device);
  for (auto& r : s->res) r.destroy();
  delete s;
  return SBC_OK;
}

sbc_status sbc_server_submit(sbc_server s, sbc_graph g, uint32_t mode, sbc_job* out) {
  if (!s || !g || !out) return fail(SBC_E_INVALID_ARG, "NULL argument");
  if (mode & ~(SBC_COMPRESSED | SBC_UNORDERED | SBC_DETERMINISTIC)) return fail(SBC_E_INVALID_ARG, "unknown mode bit");
  sbc_job j = new (std::nothrow) sbc_job_s();
  if (!j) return fail(SBC_E_OOM, "host allocation failed");
  j->g = g;
  j->mode = mode;
  j->t_submit = now_ms();
  try {
    j->est = work_estimate(g->g);
  } catch (...) {
    j->est = 0.0;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) {
      delete j;
      return fail(SBC_E_CANCELLED, "server is stopping");
    }
    s->pending.push_back(j);
  }
  s->cv.notify_all();
  *out = j;
  return SBC_OK;
}

sbc_status sbc_job_poll(sbc_job j, int* done) {
  if (!j || !done) return fail(SBC_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(j->mu);
  *done = j->done ? 1 : 0;
  return SBC_OK;
}

sbc_status sbc_job_wait(sbc_job j, double* bc_host, sbc_job_stats* st) {
  if (!j) return fail(SBC_E_INVALID_ARG, "NULL job");
  std::unique_lock<std::mutex> lk(j->mu);
  j->cv.wait(lk, [&] { return j->done; });
  if (st) *st = j->stats;
  if (j->status != SBC_OK) return fail(j->status, j->error);
  if (bc_host && !j->result.empty()) std::memcpy(bc_host, j->result.data(), sizeof(double) * j->result.size());
  return SBC_OK;
}

sbc_status sbc_job_release(sbc_job j) {
  if (j) job_unref(j);
  return SBC_OK;
}

}  // extern "C"
