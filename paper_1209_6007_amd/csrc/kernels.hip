// Host launchers of the traversal kernels (device code in kernels_dev.hpp).
// SBC_EMU_FEW_VARIANTS (set only by the CPU-emulated test build) keeps the
// shapes its checks use: 4-wave batch, team and small-piece workgroups.
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

template <int WAVES, bool R, bool I, bool D>
hipError_t launch_wave_t(const DevPieces& P, const QueueArgs& Q, int grid, int32_t np_max, int32_t arcs_max,
                         const DumpOut& dump, hipStream_t stream) {
  const size_t lds = (size_t)wave_lds_layout(np_max, arcs_max, WAVES).total;
  if (lds > kMaxLdsBytes) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)wave_kernel<WAVES, R, I, D>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return e;
    }
  }
  (void)hipGetLastError();
  hipLaunchKernelGGL((wave_kernel<WAVES, R, I, D>), dim3(grid), dim3(WAVES * 64), lds, stream, P, Q, np_max, arcs_max,
                     dump);
  return hipGetLastError();
}

template <int WAVES, bool D>
hipError_t launch_wave_w(const DevPieces& P, const QueueArgs& Q, bool r, bool i, int grid, int32_t np_max,
                         int32_t arcs_max, const DumpOut& dump, hipStream_t stream) {
  if (r && i) return launch_wave_t<WAVES, true, true, D>(P, Q, grid, np_max, arcs_max, dump, stream);
  if (r) return launch_wave_t<WAVES, true, false, D>(P, Q, grid, np_max, arcs_max, dump, stream);
  if (i) return launch_wave_t<WAVES, false, true, D>(P, Q, grid, np_max, arcs_max, dump, stream);
  return launch_wave_t<WAVES, false, false, D>(P, Q, grid, np_max, arcs_max, dump, stream);
}

template <int WAVES>
int occ_wave_w(size_t dyn) {
  int nb = 0;
  if (dyn > 64 * 1024 &&
      hipFuncSetAttribute((const void*)wave_kernel<WAVES, true, true, false>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)wave_kernel<WAVES, true, true, false>,
                                                   WAVES * 64, dyn) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

template <int WAVES, int EU, bool D, bool C>
hipError_t launch_ms_c(const DevPieces& P, const QueueArgs& Q, bool r, bool i, int grid, const MsState& st,
                       const DumpOut& dump, hipStream_t stream) {
  (void)hipGetLastError();
  if (r && i)
    hipLaunchKernelGGL((ms_kernel<WAVES, EU, true, true, D, C>), dim3(grid), dim3(WAVES * 64), 0, stream, P, Q, st,
                       dump);
  else if (r)
    hipLaunchKernelGGL((ms_kernel<WAVES, EU, true, false, D, C>), dim3(grid), dim3(WAVES * 64), 0, stream, P, Q, st,
                       dump);
  else if (i)
    hipLaunchKernelGGL((ms_kernel<WAVES, EU, false, true, D, C>), dim3(grid), dim3(WAVES * 64), 0, stream, P, Q, st,
                       dump);
  else
    hipLaunchKernelGGL((ms_kernel<WAVES, EU, false, false, D, C>), dim3(grid), dim3(WAVES * 64), 0, stream, P, Q, st,
                       dump);
  return hipGetLastError();
}

// The compact value layout runs when the state carries its offset arrays.
template <int WAVES, int EU, bool D>
hipError_t launch_ms_w(const DevPieces& P, const QueueArgs& Q, bool r, bool i, int grid, const MsState& st,
                       const DumpOut& dump, hipStream_t stream) {
  if (st.eoff && st.ob) return launch_ms_c<WAVES, EU, D, true>(P, Q, r, i, grid, st, dump, stream);
  return launch_ms_c<WAVES, EU, D, false>(P, Q, r, i, grid, st, dump, stream);
}

// The dump variants are built at the compiler's default occupancy only.
template <int WAVES>
hipError_t launch_ms_e(const DevPieces& P, const QueueArgs& Q, bool r, bool i, int eu, int grid, const MsState& st,
                       const DumpOut* dump, hipStream_t stream) {
  if (dump) return launch_ms_w<WAVES, 0, true>(P, Q, r, i, grid, st, *dump, stream);
  const DumpOut none{};
  switch (eu) {
    case 0: return launch_ms_w<WAVES, 0, false>(P, Q, r, i, grid, st, none, stream);
    case 6: return launch_ms_w<WAVES, 6, false>(P, Q, r, i, grid, st, none, stream);
    case 8: return launch_ms_w<WAVES, 8, false>(P, Q, r, i, grid, st, none, stream);
    default: return hipErrorInvalidValue;
  }
}

// The team kernel needs all of its workgroups resident at once: a cooperative
// launch makes the runtime start the grid only when that holds (and reject a
// grid that never could).
template <int WAVES, int EU, bool R, bool I, bool D>
hipError_t launch_team_t(const DevPieces& P, const QueueArgs& Q, int grid, const MsState& st, const TeamArgs& T,
                         const DumpOut& dump, hipStream_t stream) {
  DevPieces p = P;
  QueueArgs q = Q;
  MsState s = st;
  TeamArgs t = T;
  DumpOut d = dump;
  (void)hipGetLastError();
  if (!T.cooperative) {
    // An ordinary launch of a grid the device holds at once: the kernel's
    // bounded join barrier turns a workgroup that never starts into an
    // aborted run (kFlagTeamTimeout), not a hang.
    hipLaunchKernelGGL((ms_team_kernel<WAVES, EU, R, I, D>), dim3(grid), dim3(WAVES * 64),
                       (unsigned)sizeof(TeamShared<WAVES * 64>), stream, p, q, s, t, d);
    return hipGetLastError();
  }
  void* args[] = {&p, &q, &s, &t, &d};
  const hipError_t e = hipLaunchCooperativeKernel(ms_team_kernel<WAVES, EU, R, I, D>, dim3(grid), dim3(WAVES * 64),
                                                  args, (unsigned)sizeof(TeamShared<WAVES * 64>), stream);
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

template <int WAVES, int EU, bool D>
hipError_t launch_team_w(const DevPieces& P, const QueueArgs& Q, bool r, bool i, int grid, const MsState& st,
                         const TeamArgs& T, const DumpOut& dump, hipStream_t stream) {
  if (r && i) return launch_team_t<WAVES, EU, true, true, D>(P, Q, grid, st, T, dump, stream);
  if (r) return launch_team_t<WAVES, EU, true, false, D>(P, Q, grid, st, T, dump, stream);
  if (i) return launch_team_t<WAVES, EU, false, true, D>(P, Q, grid, st, T, dump, stream);
  return launch_team_t<WAVES, EU, false, false, D>(P, Q, grid, st, T, dump, stream);
}

template <int WAVES, int EU, bool D>
int occ_team_w() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)ms_team_kernel<WAVES, EU, true, true, D>,
                                                   WAVES * 64, sizeof(TeamShared<WAVES * 64>)) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

template <int WAVES, int EU>
int occ_ms_w() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)ms_kernel<WAVES, EU, true, true, false>, WAVES * 64,
                                                   0) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return nb > 0 ? nb : 1;
}

}  // namespace

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
hipError_t launch_ms(const DevPieces& P, const QueueArgs& Q, bool reach, bool ident, int waves, int eu, int grid,
                     const MsState& st, const DumpOut* dump, hipStream_t stream) {
  switch (waves) {
    case 4: return launch_ms_e<4>(P, Q, reach, ident, eu, grid, st, dump, stream);
#ifndef SBC_EMU_FEW_VARIANTS
    case 8: return launch_ms_e<8>(P, Q, reach, ident, eu, grid, st, dump, stream);
    case 16: return launch_ms_e<16>(P, Q, reach, ident, eu, grid, st, dump, stream);
#endif
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_wave(const DevPieces& P, const QueueArgs& Q, bool reach, bool ident, int waves, int grid,
                       int32_t np_max, int32_t arcs_max, const DumpOut* dump, hipStream_t stream) {
  const DumpOut none{};
  switch (waves) {
    case 4:
      return dump ? launch_wave_w<4, true>(P, Q, reach, ident, grid, np_max, arcs_max, *dump, stream)
                  : launch_wave_w<4, false>(P, Q, reach, ident, grid, np_max, arcs_max, none, stream);
#ifndef SBC_EMU_FEW_VARIANTS
    case 8:
      return dump ? launch_wave_w<8, true>(P, Q, reach, ident, grid, np_max, arcs_max, *dump, stream)
                  : launch_wave_w<8, false>(P, Q, reach, ident, grid, np_max, arcs_max, none, stream);
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

int occupancy_team(int waves, int eu, bool dump) {
  if (dump) {
    switch (waves) {
      case 4: return occ_team_w<4, 0, true>();
#ifndef SBC_EMU_FEW_VARIANTS
      case 8: return occ_team_w<8, 0, true>();
      case 16: return occ_team_w<16, 0, true>();
#endif
      default: return 0;
    }
  }
  switch (waves * 100 + eu) {
    case 400: return occ_team_w<4, 0, false>();
    case 408: return occ_team_w<4, 8, false>();
#ifndef SBC_EMU_FEW_VARIANTS
    case 800: return occ_team_w<8, 0, false>();
    case 808: return occ_team_w<8, 8, false>();
    case 1600: return occ_team_w<16, 0, false>();
    case 1608: return occ_team_w<16, 8, false>();
#endif
    default: return 0;
  }
}

hipError_t launch_team(const DevPieces& P, const QueueArgs& Q, bool reach, bool ident, int waves, int eu, int grid,
                       const MsState& st, const TeamArgs& T, const DumpOut* dump, hipStream_t stream) {
  const DumpOut none{};
  if (dump) {  // the dump variants: compiler-default occupancy only (the host sizes the grid for it)
    switch (waves) {
      case 4: return launch_team_w<4, 0, true>(P, Q, reach, ident, grid, st, T, *dump, stream);
#ifndef SBC_EMU_FEW_VARIANTS
      case 8: return launch_team_w<8, 0, true>(P, Q, reach, ident, grid, st, T, *dump, stream);
      case 16: return launch_team_w<16, 0, true>(P, Q, reach, ident, grid, st, T, *dump, stream);
#endif
      default: return hipErrorInvalidValue;
    }
  }
  switch (waves * 100 + eu) {
    case 400: return launch_team_w<4, 0, false>(P, Q, reach, ident, grid, st, T, none, stream);
    case 408: return launch_team_w<4, 8, false>(P, Q, reach, ident, grid, st, T, none, stream);
#ifndef SBC_EMU_FEW_VARIANTS
    case 800: return launch_team_w<8, 0, false>(P, Q, reach, ident, grid, st, T, none, stream);
    case 808: return launch_team_w<8, 8, false>(P, Q, reach, ident, grid, st, T, none, stream);
    case 1600: return launch_team_w<16, 0, false>(P, Q, reach, ident, grid, st, T, none, stream);
    case 1608: return launch_team_w<16, 8, false>(P, Q, reach, ident, grid, st, T, none, stream);
#endif
    default: return hipErrorInvalidValue;
  }
}

namespace {
template <int WAVES>
hipError_t launch_far_w(const DevPieces& P, const QueueArgs& Q, bool reach, int grid, const FarState& st,
                        int64_t* out, hipStream_t stream) {
  (void)hipGetLastError();
  if (reach)
    hipLaunchKernelGGL((far_kernel<WAVES, true>), dim3(grid), dim3(WAVES * 64), 0, stream, P, Q, st, out);
  else
    hipLaunchKernelGGL((far_kernel<WAVES, false>), dim3(grid), dim3(WAVES * 64), 0, stream, P, Q, st, out);
  return hipGetLastError();
}
template <int WAVES>
int occ_far_w() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)far_kernel<WAVES, true>, WAVES * 64, 0) !=
      hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}
}  // namespace

hipError_t launch_far(const DevPieces& P, const QueueArgs& Q, bool reach, int waves, int grid, const FarState& st,
                      int64_t* out, hipStream_t stream) {
  switch (waves) {
    case 4: return launch_far_w<4>(P, Q, reach, grid, st, out, stream);
#ifndef SBC_EMU_FEW_VARIANTS
    case 8: return launch_far_w<8>(P, Q, reach, grid, st, out, stream);
    case 16: return launch_far_w<16>(P, Q, reach, grid, st, out, stream);
#endif
    default: return hipErrorInvalidValue;
  }
}

int occupancy_far(int waves) {
  switch (waves) {
    case 4: return occ_far_w<4>();
#ifndef SBC_EMU_FEW_VARIANTS
    case 8: return occ_far_w<8>();
    case 16: return occ_far_w<16>();
#endif
    default: return 0;
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

hipError_t launch_det_reduce(int32_t nverts, int32_t npieces, const int32_t* vtx_off, const int64_t* area_base,
                             const int32_t* piece_items, const double* item_out, double* bcp, hipStream_t stream) {
  if (nverts <= 0) return hipSuccess;
  (void)hipGetLastError();
  hipLaunchKernelGGL(det_reduce_kernel, dim3((nverts + 255) / 256), dim3(256), 0, stream, nverts, npieces, vtx_off,
                     area_base, piece_items, item_out, bcp);
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
