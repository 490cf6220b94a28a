// Host emulation of the HIP subset the library uses -- TEST INFRASTRUCTURE.
//
// Lets the library's own sources (runtime, C interface, kernels) compile with
// g++ and run on the CPU, so that indexing and synchronisation mistakes show
// up under AddressSanitizer instead of on a GPU.  Semantics:
//   * every "asynchronous" call executes at once, in host program order;
//   * a kernel launch runs its blocks one after another; each block runs
//     blockDim.x OS threads, grouped in 64-lane waves; a cooperative launch
//     runs all blocks at once (their threads together), so blocks can wait
//     for each other;
//   * __syncthreads is a barrier over the block, wave intrinsics (ballot,
//     shuffles, readlane) exchange values through a per-wave buffer with a
//     wave barrier on each side (all lanes of a wave must reach them, which the
//     kernels guarantee by calling them in wave-uniform control flow);
//   * device memory is host malloc, so out-of-bounds accesses are caught.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>
#include <utility>
#include <memory>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define SBC_KERNEL_BOUNDS(block, eu)
#define __shared__ static
#define __align__(x) alignas(x)

struct uint4 {
  unsigned x, y, z, w;
};

struct dim3 {
  unsigned x = 1, y = 1, z = 1;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

inline thread_local dim3 threadIdx(0), blockIdx(0), blockDim(1), gridDim(1);

namespace sbc_emu {

class Barrier {
 public:
  explicit Barrier(int n) : n_(n) {}
  void wait() {
    std::unique_lock<std::mutex> lk(mu_);
    const long gen = gen_;
    if (++count_ == n_) {
      count_ = 0;
      ++gen_;
      cv_.notify_all();
    } else {
      cv_.wait(lk, [&] { return gen_ != gen; });
    }
  }

 private:
  std::mutex mu_;
  std::condition_variable cv_;
  int n_;
  int count_ = 0;
  long gen_ = 0;
};

struct Wave {
  explicit Wave(int lanes) : bar(lanes), nlanes(lanes) {}
  Barrier bar;
  int nlanes;
  uint64_t slot[64];
};

struct Block {
  Barrier bar;
  std::vector<std::unique_ptr<Wave>> waves;
  unsigned char* dyn = nullptr;
  explicit Block(int threads) : bar(threads) {
    for (int w = 0; w < (threads + 63) / 64; ++w) waves.emplace_back(new Wave(std::min(64, threads - 64 * w)));
  }
};

inline thread_local Block* tl_block = nullptr;
inline std::mutex launch_mu;  // one emulated kernel at a time (static __shared__ storage is per function)

inline Wave& wave() { return *tl_block->waves[threadIdx.x / 64]; }
inline int lane() { return (int)(threadIdx.x % 64); }

template <typename T>
inline uint64_t bits(T v) {
  uint64_t b = 0;
  std::memcpy(&b, &v, sizeof(T));
  return b;
}
template <typename T>
inline T from_bits(uint64_t b) {
  T v;
  std::memcpy(&v, &b, sizeof(T));
  return v;
}

// Publish v, wait for the wave, apply f to the slots, wait again.
template <typename T, typename F>
inline T exchange(T v, F f) {
  Wave& w = wave();
  w.slot[lane()] = bits(v);
  w.bar.wait();
  T r = f(w.slot, w.nlanes);
  w.bar.wait();
  return r;
}

template <typename K>
void launch(dim3 grid, dim3 block, size_t dyn_bytes, K&& body) {
  std::lock_guard<std::mutex> lk(launch_mu);
  for (unsigned b = 0; b < grid.x; ++b) {
    Block blk((int)block.x);
    unsigned char* dynp = nullptr;
    if (dyn_bytes) {
      dynp = (unsigned char*)std::malloc(dyn_bytes);  // exact size, so overruns are caught
      std::memset(dynp, 0xC3, dyn_bytes);             // LDS starts with garbage
      blk.dyn = dynp;
    }
    std::vector<std::thread> ts;
    ts.reserve(block.x);
    for (unsigned t = 0; t < block.x; ++t)
      ts.emplace_back([&, t, b] {
        threadIdx = dim3(t);
        blockIdx = dim3(b);
        blockDim = block;
        gridDim = grid;
        tl_block = &blk;
        body();
      });
    for (auto& th : ts) th.join();
    std::free(dynp);
  }
}

// All blocks at once (cooperative launch).  Kernels launched this way keep
// their shared state in dynamic LDS (static __shared__ would be shared by all
// blocks here).
template <typename K>
void launch_all(dim3 grid, dim3 block, size_t dyn_bytes, K&& body) {
  std::lock_guard<std::mutex> lk(launch_mu);
  std::vector<std::unique_ptr<Block>> blks;
  std::vector<unsigned char*> dyns;
  for (unsigned b = 0; b < grid.x; ++b) {
    blks.emplace_back(new Block((int)block.x));
    unsigned char* dynp = nullptr;
    if (dyn_bytes) {
      dynp = (unsigned char*)std::malloc(dyn_bytes);
      std::memset(dynp, 0xC3, dyn_bytes);
    }
    blks.back()->dyn = dynp;
    dyns.push_back(dynp);
  }
  std::vector<std::thread> ts;
  ts.reserve((size_t)grid.x * block.x);
  for (unsigned b = 0; b < grid.x; ++b)
    for (unsigned t = 0; t < block.x; ++t)
      ts.emplace_back([&, t, b] {
        threadIdx = dim3(t);
        blockIdx = dim3(b);
        blockDim = block;
        gridDim = grid;
        tl_block = blks[b].get();
        body();
      });
  for (auto& th : ts) th.join();
  for (auto* d : dyns) std::free(d);
}

template <typename... A, size_t... I>
void call_with(void (*k)(A...), void** args, std::index_sequence<I...>) {
  k(*static_cast<A*>(args[I])...);
}

}  // namespace sbc_emu

#define SBC_DYNAMIC_LDS(name) unsigned char* name = sbc_emu::tl_block->dyn

inline void __syncthreads() { sbc_emu::tl_block->bar.wait(); }

#include <chrono>
inline long long wall_clock64() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
             .count() /
         10;  // 100 MHz, like the device counter
}

inline unsigned long long __ballot(int pred) {
  return sbc_emu::exchange<uint64_t>(pred ? (1ull << sbc_emu::lane()) : 0ull, [](const uint64_t* s, int n) {
    uint64_t r = 0;
    for (int i = 0; i < n; ++i) r |= s[i];
    return r;
  });
}

template <typename T>
inline T __shfl_xor(T v, int off, int width = 64) {
  (void)width;
  const int me = sbc_emu::lane();
  return sbc_emu::exchange<T>(v, [&](const uint64_t* s, int n) {
    const int src = me ^ off;
    return src < n ? sbc_emu::from_bits<T>(s[src]) : v;
  });
}

template <typename T>
inline T __shfl_up(T v, unsigned off, int width = 64) {
  (void)width;
  const int me = sbc_emu::lane();
  return sbc_emu::exchange<T>(v, [&](const uint64_t* s, int) {
    return me >= (int)off ? sbc_emu::from_bits<T>(s[me - off]) : v;
  });
}

namespace sbc_emu {
inline int readlane(int v, int k) {
  return exchange<int>(v, [&](const uint64_t* s, int n) {
    if (k < 0 || k >= n) std::abort();
    return from_bits<int>(s[k]);
  });
}
}  // namespace sbc_emu

#define __builtin_amdgcn_readlane(v, k) sbc_emu::readlane((v), (k))
#define __builtin_amdgcn_readfirstlane(v) sbc_emu::readlane((v), 0)

#define __HIP_MEMORY_SCOPE_WORKGROUP 0
#define __HIP_MEMORY_SCOPE_AGENT 0
namespace sbc_emu {
template <typename T>
inline T atomic_load(T* p) {
  T v;
  __atomic_load(p, &v, __ATOMIC_SEQ_CST);
  return v;
}
}  // namespace sbc_emu
#define __hip_atomic_load(p, order, scope) sbc_emu::atomic_load(p)
#define __hip_atomic_store(p, v, order, scope) __atomic_store_n((p), (v), __ATOMIC_SEQ_CST)
#define __hip_atomic_fetch_add(p, v, order, scope) __atomic_fetch_add((p), (v), __ATOMIC_SEQ_CST)
#define __hip_atomic_fetch_or(p, v, order, scope) __atomic_fetch_or((p), (v), __ATOMIC_SEQ_CST)
#define __builtin_amdgcn_fence(order, scope) std::atomic_thread_fence(std::memory_order_seq_cst)
#define __builtin_amdgcn_s_sleep(n) std::this_thread::yield()
// Team-kernel fences and ids: blocks 2k and 2k+1 run on XCD k mod 8 (so teams
// of one XCD and teams spread over several both occur with few blocks); lanes
// of a wave meet at a wave barrier.
#define SBC_XCD_FENCES 1
inline void xcd_release() { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline int xcc_id() { return (int)((blockIdx.x / 2) % 8); }
inline void wave_sync() { sbc_emu::wave().bar.wait(); }

inline int atomicAdd(int* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
inline int atomicCAS(int* p, int cmp, int v) {
  __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED);
  return cmp;
}
inline int atomicOr(int* p, int v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
inline unsigned long long atomicOr(unsigned long long* p, unsigned long long v) {
  return __atomic_fetch_or(p, v, __ATOMIC_RELAXED);
}
inline double atomicAdd(double* p, double v) {
  uint64_t* q = reinterpret_cast<uint64_t*>(p);
  uint64_t old = __atomic_load_n(q, __ATOMIC_RELAXED);
  while (true) {
    const double nv = sbc_emu::from_bits<double>(old) + v;
    if (__atomic_compare_exchange_n(q, &old, sbc_emu::bits(nv), false, __ATOMIC_RELAXED, __ATOMIC_RELAXED))
      return sbc_emu::from_bits<double>(old);
  }
}
using std::min;
using std::max;

// ------------------------------------------------------------ runtime API

typedef int hipError_t;
enum {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidSymbol = 13,
  hipErrorNotSupported = 801,
};
typedef struct emu_stream* hipStream_t;
typedef struct emu_event* hipEvent_t;
typedef struct emu_graph* hipGraph_t;
typedef struct emu_graph_exec* hipGraphExec_t;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipHostMallocDefault = 0 };
enum hipDeviceAttribute_t {
  hipDeviceAttributeMaxSharedMemoryPerBlock = 1,
  hipDeviceAttributeWallClockRate = 2,
  hipDeviceAttributeCooperativeLaunch = 3
};
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 1 };
enum hipStreamCaptureMode { hipStreamCaptureModeThreadLocal = 1 };

struct hipDeviceProp_t {
  char name[256] = "emulated gfx950";
  char gcnArchName[256] = "gfx950:sramecc+:xnack-";
  int multiProcessorCount = 2;
};

struct emu_stream {};
struct emu_event {
  double t_ms = 0;
};

inline const char* hipGetErrorString(hipError_t e) {
  static thread_local char buf[48];
  std::snprintf(buf, sizeof buf, "emulated HIP error %d", (int)e);
  return e == hipSuccess ? "success" : buf;
}
// As in HIP: a failing call leaves its error behind until hipGetLastError()
// reads it, and successful calls do not clear it.
inline thread_local hipError_t tl_last_error = hipSuccess;
inline hipError_t emu_fail(hipError_t e) {
  tl_last_error = e;
  return e;
}
inline hipError_t hipGetLastError() {
  const hipError_t e = tl_last_error;
  tl_last_error = hipSuccess;
  return e;
}
inline hipError_t hipGetDeviceCount(int* c) {
  *c = 1;
  return hipSuccess;
}
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  *p = hipDeviceProp_t();
  return hipSuccess;
}
// Fails like a runtime that does not know the attribute, leaving a sticky
// error: the library must neither depend on the answer nor mistake the stale
// error for a failure of a later kernel launch.
inline hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  if (a == hipDeviceAttributeWallClockRate) {
    *v = 100000;  // kHz
    return hipSuccess;
  }
  if (a == hipDeviceAttributeCooperativeLaunch) {
    *v = 1;
    return hipSuccess;
  }
  *v = 0;
  return emu_fail(hipErrorInvalidValue);
}
inline hipError_t hipMemGetInfo(size_t* f, size_t* t) {
  *f = (size_t)1 << 30;
  *t = (size_t)1 << 31;
  return hipSuccess;
}
// Device memory starts with garbage, as on the GPU: a read before the first
// write then yields a wild value instead of a convenient zero.
inline hipError_t hipMalloc(void** p, size_t b) {
  *p = std::malloc(b);
  if (*p) std::memset(*p, 0xA5, b);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
inline hipError_t hipHostMalloc(void** p, size_t b, unsigned) { return hipMalloc(p, b); }
inline hipError_t hipHostFree(void* p) { return hipFree(p); }
inline hipError_t hipMemcpy(void* d, const void* s, size_t b, hipMemcpyKind) {
  std::memcpy(d, s, b);
  return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t b, hipMemcpyKind k, hipStream_t) {
  return hipMemcpy(d, s, b, k);
}
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new emu_stream();
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new emu_event();
  return hipSuccess;
}
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
inline hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  e->t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
  return hipSuccess;
}
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = (float)(b->t_ms - a->t_ms);
  return hipSuccess;
}
inline hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t*) { return hipErrorNotSupported; }
inline hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, void*, void*, size_t) {
  return hipErrorNotSupported;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
inline hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
inline hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* nb, const void*, int, size_t) {
  *nb = 2;
  return hipSuccess;
}

// A file-scope device variable is an ordinary host object here; its "device
// address" is its host address.
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);
  return hipSuccess;
}

#define hipLaunchKernelGGL(K, G, B, S, ST, ...) sbc_emu::launch((G), (B), (S), [&] { K(__VA_ARGS__); })

template <typename... A>
inline hipError_t hipLaunchCooperativeKernel(void (*k)(A...), dim3 grid, dim3 block, void** args, unsigned dyn,
                                             hipStream_t) {
  sbc_emu::launch_all(grid, block, dyn, [&] { sbc_emu::call_with(k, args, std::index_sequence_for<A...>{}); });
  return hipSuccess;
}
