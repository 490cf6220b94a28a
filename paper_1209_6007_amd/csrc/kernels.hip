// Host launchers of the traversal kernels (device code in kernels_dev.hpp).
// SBC_EMU_FEW_VARIANTS (set only by the CPU-emulated test build) keeps the
// shapes its checks use: 4-wave batch and team workgroups, 64- and 256-thread
// per-source workgroups.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cstdint>

#include "kernels.hpp"

#ifndef SBC_DYNAMIC_LDS
#define SBC_DYNAMIC_LDS(name) extern __shared__ __align__(16) unsigned char name[]
#endif
#include "kernels_dev.hpp"

namespace sbc {

namespace {

using namespace dev;

template <typename T>
hipError_t fill(T* p, T v, int64_t count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
  (void)hipGetLastError();  // drop any stale error so the status below is this launch's own
  hipLaunchKernelGGL(fill_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, stream, p, v, count);
  return hipGetLastError();
}

template <int BLOCK, bool R, bool I, bool LDS>
hipError_t launch_wg_t(const DevPieces& P, const QueueArgs& Q, int grid, int32_t max_np, const WgState& st,
                       const DebugOut& dbg, hipStream_t stream) {
  const size_t lds = LDS ? wg_lds_bytes(max_np) : 0;
  if (LDS && lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)wg_kernel<BLOCK, R, I, LDS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return e;
    }
  }
  (void)hipGetLastError();
  hipLaunchKernelGGL((wg_kernel<BLOCK, R, I, LDS>), dim3(grid), dim3(BLOCK), lds, stream, P, Q, st, max_np, dbg);
  return hipGetLastError();
}

template <int BLOCK, bool LDS>
hipError_t launch_wg_b(const DevPieces& P, const QueueArgs& Q, bool r, bool i, int grid, int32_t max_np,
                       const WgState& st, const DebugOut& dbg, hipStream_t stream) {
  if (r && i) return launch_wg_t<BLOCK, true, true, LDS>(P, Q, grid, max_np, st, dbg, stream);
  if (r) return launch_wg_t<BLOCK, true, false, LDS>(P, Q, grid, max_np, st, dbg, stream);
  if (i) return launch_wg_t<BLOCK, false, true, LDS>(P, Q, grid, max_np, st, dbg, stream);
  return launch_wg_t<BLOCK, false, false, LDS>(P, Q, grid, max_np, st, dbg, stream);
}

template <int WAVES, bool R, bool I>
hipError_t launch_wave_t(const DevPieces& P, const QueueArgs& Q, int grid, int32_t np_max, int32_t arcs_max,
                         hipStream_t stream) {
  const size_t lds = (size_t)wave_lds_layout(np_max, arcs_max, WAVES).total;
  if (lds > kMaxLdsBytes) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)wave_kernel<WAVES, R, I>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return e;
    }
  }
  (void)hipGetLastError();
  hipLaunchKernelGGL((wave_kernel<WAVES, R, I>), dim3(grid), dim3(WAVES * 64), lds, stream, P, Q, np_max, arcs_max);
  return hipGetLastError();
}

template <int WAVES>
hipError_t launch_wave_w(const DevPieces& P, const QueueArgs& Q, bool r, bool i, int grid, int32_t np_max,
                         int32_t arcs_max, hipStream_t stream) {
  if (r && i) return launch_wave_t<WAVES, true, true>(P, Q, grid, np_max, arcs_max, stream);
  if (r) return launch_wave_t<WAVES, true, false>(P, Q, grid, np_max, arcs_max, stream);
  if (i) return launch_wave_t<WAVES, false, true>(P, Q, grid, np_max, arcs_max, stream);
  return launch_wave_t<WAVES, false, false>(P, Q, grid, np_max, arcs_max, stream);
}

template <int WAVES>
int occ_wave_w(size_t dyn) {
  int nb = 0;
  if (dyn > 64 * 1024 &&
      hipFuncSetAttribute((const void*)wave_kernel<WAVES, true, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)dyn) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)wave_kernel<WAVES, true, true>, WAVES * 64,
                                                   dyn) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

template <int WAVES, int EU>
hipError_t launch_ms_w(const DevPieces& P, const QueueArgs& Q, bool r, bool i, int grid, const MsState& st,
                       hipStream_t stream) {
  (void)hipGetLastError();
  if (r && i)
    hipLaunchKernelGGL((ms_kernel<WAVES, EU, true, true>), dim3(grid), dim3(WAVES * 64), 0, stream, P, Q, st);
  else if (r)
    hipLaunchKernelGGL((ms_kernel<WAVES, EU, true, false>), dim3(grid), dim3(WAVES * 64), 0, stream, P, Q, st);
  else if (i)
    hipLaunchKernelGGL((ms_kernel<WAVES, EU, false, true>), dim3(grid), dim3(WAVES * 64), 0, stream, P, Q, st);
  else
    hipLaunchKernelGGL((ms_kernel<WAVES, EU, false, false>), dim3(grid), dim3(WAVES * 64), 0, stream, P, Q, st);
  return hipGetLastError();
}

template <int WAVES>
hipError_t launch_ms_e(const DevPieces& P, const QueueArgs& Q, bool r, bool i, int eu, int grid, const MsState& st,
                       hipStream_t stream) {
  switch (eu) {
    case 0: return launch_ms_w<WAVES, 0>(P, Q, r, i, grid, st, stream);
    case 6: return launch_ms_w<WAVES, 6>(P, Q, r, i, grid, st, stream);
    case 8: return launch_ms_w<WAVES, 8>(P, Q, r, i, grid, st, stream);
    default: return hipErrorInvalidValue;
  }
}

// The team kernel needs all of its workgroups resident at once: a cooperative
// launch makes the runtime start the grid only when that holds (and reject a
// grid that never could).
template <int WAVES, int EU, bool R, bool I>
hipError_t launch_team_t(const DevPieces& P, const QueueArgs& Q, int grid, const MsState& st, const TeamArgs& T,
                         hipStream_t stream) {
  DevPieces p = P;
  QueueArgs q = Q;
  MsState s = st;
  TeamArgs t = T;
  void* args[] = {&p, &q, &s, &t};
  (void)hipGetLastError();
  const hipError_t e = hipLaunchCooperativeKernel(ms_team_kernel<WAVES, EU, R, I>, dim3(grid), dim3(WAVES * 64),
                                                  args, (unsigned)sizeof(TeamShared<WAVES * 64>), stream);
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

template <int WAVES, int EU>
hipError_t launch_team_w(const DevPieces& P, const QueueArgs& Q, bool r, bool i, int grid, const MsState& st,
                         const TeamArgs& T, hipStream_t stream) {
  if (r && i) return launch_team_t<WAVES, EU, true, true>(P, Q, grid, st, T, stream);
  if (r) return launch_team_t<WAVES, EU, true, false>(P, Q, grid, st, T, stream);
  if (i) return launch_team_t<WAVES, EU, false, true>(P, Q, grid, st, T, stream);
  return launch_team_t<WAVES, EU, false, false>(P, Q, grid, st, T, stream);
}

template <int WAVES, int EU>
int occ_team_w() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)ms_team_kernel<WAVES, EU, true, true>,
                                                   WAVES * 64, sizeof(TeamShared<WAVES * 64>)) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

template <int BLOCK, bool LDS>
int occ_wg_b(size_t dyn) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)wg_kernel<BLOCK, true, true, LDS>, BLOCK, dyn) !=
      hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return nb > 0 ? nb : 1;
}

template <int WAVES, int EU>
int occ_ms_w() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)ms_kernel<WAVES, EU, true, true>, WAVES * 64,
                                                   0) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return nb > 0 ? nb : 1;
}

}  // namespace

size_t wg_lds_bytes(int32_t max_np) { return (size_t)max_np * 20 + 16; }

int occupancy_wg(int block, bool lds, size_t dyn) {
  switch (block) {
    case 64: return lds ? occ_wg_b<64, true>(dyn) : occ_wg_b<64, false>(0);
    case 256: return lds ? occ_wg_b<256, true>(dyn) : occ_wg_b<256, false>(0);
#ifndef SBC_EMU_FEW_VARIANTS
    case 512: return lds ? occ_wg_b<512, true>(dyn) : occ_wg_b<512, false>(0);
    case 1024: return lds ? occ_wg_b<1024, true>(dyn) : occ_wg_b<1024, false>(0);
#endif
    default: return 1;
  }
}

int occupancy_ms(int waves, int eu) {
  const int key = waves * 100 + eu;
  switch (key) {
    case 400: return occ_ms_w<4, 0>();
    case 406: return occ_ms_w<4, 6>();
    case 408: return occ_ms_w<4, 8>();
#ifndef SBC_EMU_FEW_VARIANTS
    case 800: return occ_ms_w<8, 0>();
    case 806: return occ_ms_w<8, 6>();
    case 808: return occ_ms_w<8, 8>();
    case 1600: return occ_ms_w<16, 0>();
    case 1606: return occ_ms_w<16, 6>();
    case 1608: return occ_ms_w<16, 8>();
#endif
    default: return 1;
  }
}
hipError_t launch_wg(const DevPieces& P, const QueueArgs& Q, bool reach, bool ident, bool lds, int block, int grid,
                     int32_t max_np, const WgState& st, const DebugOut* dbg, hipStream_t stream) {
  DebugOut d{nullptr, nullptr, nullptr};
  if (dbg) d = *dbg;
  switch (block) {
    case 64:
      return lds ? launch_wg_b<64, true>(P, Q, reach, ident, grid, max_np, st, d, stream)
                 : launch_wg_b<64, false>(P, Q, reach, ident, grid, max_np, st, d, stream);
    case 256:
      return lds ? launch_wg_b<256, true>(P, Q, reach, ident, grid, max_np, st, d, stream)
                 : launch_wg_b<256, false>(P, Q, reach, ident, grid, max_np, st, d, stream);
#ifndef SBC_EMU_FEW_VARIANTS
    case 512:
      return lds ? launch_wg_b<512, true>(P, Q, reach, ident, grid, max_np, st, d, stream)
                 : launch_wg_b<512, false>(P, Q, reach, ident, grid, max_np, st, d, stream);
    case 1024:
      return lds ? launch_wg_b<1024, true>(P, Q, reach, ident, grid, max_np, st, d, stream)
                 : launch_wg_b<1024, false>(P, Q, reach, ident, grid, max_np, st, d, stream);
#endif
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_ms(const DevPieces& P, const QueueArgs& Q, bool reach, bool ident, int waves, int eu, int grid,
                     const MsState& st, hipStream_t stream) {
  switch (waves) {
    case 4: return launch_ms_e<4>(P, Q, reach, ident, eu, grid, st, stream);
#ifndef SBC_EMU_FEW_VARIANTS
    case 8: return launch_ms_e<8>(P, Q, reach, ident, eu, grid, st, stream);
    case 16: return launch_ms_e<16>(P, Q, reach, ident, eu, grid, st, stream);
#endif
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_wave(const DevPieces& P, const QueueArgs& Q, bool reach, bool ident, int waves, int grid,
                       int32_t np_max, int32_t arcs_max, hipStream_t stream) {
  switch (waves) {
    case 4: return launch_wave_w<4>(P, Q, reach, ident, grid, np_max, arcs_max, stream);
#ifndef SBC_EMU_FEW_VARIANTS
    case 8: return launch_wave_w<8>(P, Q, reach, ident, grid, np_max, arcs_max, stream);
#endif
    default: return hipErrorInvalidValue;
  }
}

int occupancy_wave(int waves, int32_t np_max, int32_t arcs_max) {
  const size_t dyn = (size_t)wave_lds_layout(np_max, arcs_max, waves).total;
  if (dyn > kMaxLdsBytes) return 0;
  switch (waves) {
    case 4: return occ_wave_w<4>(dyn);
#ifndef SBC_EMU_FEW_VARIANTS
    case 8: return occ_wave_w<8>(dyn);
#endif
    default: return 0;
  }
}

int occupancy_team(int waves, int eu) {
  switch (waves * 100 + eu) {
    case 400: return occ_team_w<4, 0>();
    case 408: return occ_team_w<4, 8>();
#ifndef SBC_EMU_FEW_VARIANTS
    case 800: return occ_team_w<8, 0>();
    case 808: return occ_team_w<8, 8>();
    case 1600: return occ_team_w<16, 0>();
    case 1608: return occ_team_w<16, 8>();
#endif
    default: return 0;
  }
}

hipError_t launch_team(const DevPieces& P, const QueueArgs& Q, bool reach, bool ident, int waves, int eu, int grid,
                       const MsState& st, const TeamArgs& T, hipStream_t stream) {
  switch (waves * 100 + eu) {
    case 400: return launch_team_w<4, 0>(P, Q, reach, ident, grid, st, T, stream);
    case 408: return launch_team_w<4, 8>(P, Q, reach, ident, grid, st, T, stream);
#ifndef SBC_EMU_FEW_VARIANTS
    case 800: return launch_team_w<8, 0>(P, Q, reach, ident, grid, st, T, stream);
    case 808: return launch_team_w<8, 8>(P, Q, reach, ident, grid, st, T, stream);
    case 1600: return launch_team_w<16, 0>(P, Q, reach, ident, grid, st, T, stream);
    case 1608: return launch_team_w<16, 8>(P, Q, reach, ident, grid, st, T, stream);
#endif
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mapback(int32_t n, int32_t nverts, int32_t nmap, const int32_t* map_off, const int32_t* map_idx,
                          const double* bcp, const double* corr, const double* bcx, double scale, double* out,
                          hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  (void)hipGetLastError();
  hipLaunchKernelGGL(mapback_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, n, nverts, nmap, map_off, map_idx,
                     bcp, corr, bcx, scale, out);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, int64_t bytes, int grid, hipStream_t stream) {
  const int64_t n = bytes / 16;
  if (n <= 0) return hipSuccess;
  (void)hipGetLastError();
  hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, stream, (const uint4*)src, (uint4*)dst, n);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t stream) {
  return fill<int32_t>(p, v, count, stream);
}
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, int64_t count, hipStream_t stream) {
  return fill<uint64_t>(p, v, count, stream);
}
hipError_t launch_fill_f64(double* p, double v, int64_t count, hipStream_t stream) {
  return fill<double>(p, v, count, stream);
}

}  // namespace sbc
