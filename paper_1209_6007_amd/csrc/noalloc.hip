// sbc_piece_bc_noalloc: the computation of sbc_piece_bc (Algorithm 2 with
// identical-vertex weights on one attributed piece) for callers that cannot
// allocate device memory -- code under HIP graph capture, tight serving
// loops.  Inputs and outputs are the caller's device buffers; the traversal
// state of the 64-source batch kernel, its work items and control words live
// in `scratch`, a file-scope device array every call on a GPU shares.
//
// `scratch` is addressed from the host only through the pointer that
// hipGetSymbolAddress returns for the current device (the array's own name is
// a host-side stand-in there); it is looked up once per device, on the entry
// point's first call on that device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "runtime.hpp"
#include "shatterbc.h"

using namespace sbc;

namespace {

constexpr size_t kScratchBytes = (size_t)SBC_NOALLOC_SCRATCH_MB << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

// Control words at the start of the scratch: queue head, items done, flags.
struct NoAllocCtl {
  int32_t head, done, flags, pad;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// One piece, sources 64 at a time: item i covers sources [64i, min(n, 64i+64)).
__global__ void noalloc_setup_kernel(int32_t n, int32_t nitems, WorkItem* items, int32_t* vtx_off,
                                     int32_t* src_order, NoAllocCtl* ctl) {
  const int32_t stride = gridDim.x * blockDim.x;
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  for (int32_t i = t; i < nitems; i += stride) items[i] = {0, 64 * i, std::min(n, 64 * i + 64), KC_BATCH};
  for (int32_t v = t; v < n; v += stride) src_order[v] = v;
  if (t == 0) {
    vtx_off[0] = 0;
    vtx_off[1] = n;
    *ctl = {0, 0, 0, 0};
  }
}

// The traversal takes a piece vertex's reach as that of all its members
// together: reach x ident when both are given.  A product beyond 2^31 - 1
// (or a value below 1) is a bad item.
__global__ void noalloc_reach_kernel(int32_t n, const int32_t* reach, const int32_t* ident, int32_t* out,
                                     NoAllocCtl* ctl) {
  const int32_t stride = gridDim.x * blockDim.x;
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t r = reach[v], k = ident[v];
    if (r < 1 || k < 1 || r * k > INT32_MAX) {
      atomicOr(&ctl->flags, kFlagBadItem);
      out[v] = 1;
    } else {
      out[v] = (int32_t)(r * k);
    }
  }
}

// The run's device flags for the caller; an item that never finished counts
// as a bad item.
__global__ void noalloc_finish_kernel(NoAllocCtl* ctl, int32_t nitems, int32_t* flags_out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int32_t f = __hip_atomic_load(&ctl->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t d = __hip_atomic_load(&ctl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *flags_out = f | (d == nitems ? 0 : kFlagBadItem);
  }
}

// The scratch's device address on the current device (looked up on first use).
sbc_status scratch_of(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return fail(SBC_E_INVALID_ARG, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    }
    g_scratch[device] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch[device];
  return SBC_OK;
}

}  // namespace

extern "C" sbc_status sbc_piece_bc_noalloc(sbc_context ctx, int32_t n, int32_t arcs, const int32_t* row_ptr_dev,
                                           const int32_t* col_dev, const int32_t* reach_dev,
                                           const int32_t* ident_dev, double* bc_dev, int32_t* flags_dev,
                                           void* stream) {
  if (!ctx || !row_ptr_dev || !bc_dev || (arcs > 0 && !col_dev)) return fail(SBC_E_INVALID_ARG, "NULL argument");
  if (n < 1 || arcs < 0) return fail(SBC_E_INVALID_ARG, "need n >= 1 and arcs >= 0");
  if (n > SBC_NOALLOC_MAX_VERTICES)
    return fail(SBC_E_TOO_LARGE, "piece larger than the no-allocation scratch serves (SBC_NOALLOC_MAX_VERTICES)");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  unsigned char* base = nullptr;
  sbc_status rc = scratch_of(ctx->device, &base);
  if (rc != SBC_OK) return rc;
  hipStream_t s = (hipStream_t)stream;

  // Carve the scratch: control words, items, piece offsets, source order,
  // then as many batch-kernel slots as fit.
  const int32_t nitems = (n + 63) / 64;
  const int64_t stride = n;
  const int64_t part_cap = (int64_t)arcs / kMsSliceArcs + 2 * kMsHeavyMax;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base + off;
    off += align256(bytes);
    return p;
  };
  NoAllocCtl* ctl = reinterpret_cast<NoAllocCtl*>(take(sizeof(NoAllocCtl)));
  WorkItem* items = reinterpret_cast<WorkItem*>(take(sizeof(WorkItem) * (size_t)nitems));
  int32_t* vtx_off = reinterpret_cast<int32_t*>(take(2 * sizeof(int32_t)));
  int32_t* src_order = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)n));
  int32_t* reach_sum = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)n));
  const size_t per_slot = align256((size_t)stride * 64 * 8) * 2 + align256((size_t)stride * 64 * 4) +
                          5 * align256((size_t)stride * 8) + align256((size_t)(stride + 3) * 4) +
                          align256((size_t)part_cap * 64 * 8);
  const int64_t fit = off < kScratchBytes ? (int64_t)((kScratchBytes - off) / per_slot) : 0;
  // the batch kernel in the context's workgroup shape
  const int waves = (int)ctx->params.batch_wg_waves, eu = (int)ctx->params.batch_waves_per_eu;
  const int occ = occupancy_ms(waves, eu);
  const int64_t g = std::min<int64_t>({(int64_t)ctx->cus * std::max(occ, 1), fit, (int64_t)nitems});
  if (g < 1) return fail(SBC_E_TOO_LARGE, "piece state does not fit the no-allocation scratch");
  MsState ms{};
  ms.stride = stride;
  ms.part_cap = (int32_t)part_cap;
  ms.sg = reinterpret_cast<double*>(take(align256((size_t)stride * 64 * 8) * g));
  ms.qm = reinterpret_cast<uint64_t*>(take(align256((size_t)stride * 64 * 8) * g));
  ms.q = reinterpret_cast<int32_t*>(take(align256((size_t)stride * 64 * 4) * g));
  ms.vis = reinterpret_cast<uint64_t*>(take(align256((size_t)stride * 8) * g));
  ms.fa = reinterpret_cast<uint64_t*>(take(align256((size_t)stride * 8) * g));
  ms.fb = reinterpret_cast<uint64_t*>(take(align256((size_t)stride * 8) * g));
  ms.ba = reinterpret_cast<uint64_t*>(take(align256((size_t)stride * 8) * g));
  ms.bb = reinterpret_cast<uint64_t*>(take(align256((size_t)stride * 8) * g));
  ms.lvl = reinterpret_cast<int32_t*>(take(align256((size_t)(stride + 3) * 4) * g));
  ms.part = reinterpret_cast<double*>(take(align256((size_t)part_cap * 64 * 8) * g));
  ms.prof = nullptr;
  ms.pairs = (int32_t)ctx->params.batch_pairs;
  if (off > kScratchBytes) return fail(SBC_E_TOO_LARGE, "piece state does not fit the no-allocation scratch");
  // The slot arrays of one kind are contiguous per slot: slot b uses
  // [b*stride*64, (b+1)*stride*64) of sg, q, qm and [b*stride, ...) of the
  // masks, as the kernel indexes them; the 256-byte rounding above only pads
  // the end of each array.

  // Everything that must start at zero (or at its initial value) is written
  // by kernels on the caller's stream: the previous call's contents stay in
  // the scratch otherwise.
  (void)hipGetLastError();
  hipLaunchKernelGGL(noalloc_setup_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0, s,
                     n, nitems, items, vtx_off, src_order, ctl);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "launch setup");
  const int32_t* reach_used = reach_dev;
  if (reach_dev && ident_dev) {
    hipLaunchKernelGGL(noalloc_reach_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0,
                       s, n, reach_dev, ident_dev, reach_sum, ctl);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "launch reach");
    reach_used = reach_sum;
  }
  for (uint64_t* p : {ms.vis, ms.fa, ms.fb, ms.ba, ms.bb})
    if ((e = launch_fill_u64(p, 0, (int64_t)g * stride, s)) != hipSuccess) return hip_fail(e, "fill masks");
  if ((e = launch_fill_f64(bc_dev, 0.0, n, s)) != hipSuccess) return hip_fail(e, "fill output");
  DevPieces dp{vtx_off, row_ptr_dev, col_dev, reach_used, ident_dev, src_order, nullptr, bc_dev, 1, n, arcs, 0};
  QueueArgs qa{items, nitems, kArgMagic, &ctl->head, &ctl->flags, &ctl->done};
  e = launch_ms(dp, qa, reach_dev != nullptr, ident_dev != nullptr, waves, eu, (int)g, ms, nullptr, s);
  if (e != hipSuccess) return hip_fail(e, "launch traversal");
  if (flags_dev) {
    hipLaunchKernelGGL(noalloc_finish_kernel, dim3(1), dim3(64), 0, s, ctl, nitems, flags_dev);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "launch finish");
  }
  return SBC_OK;
}
