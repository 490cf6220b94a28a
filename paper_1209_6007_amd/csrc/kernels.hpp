// Device kernels of the traversal (Algorithm 2 with identical-vertex weights)
// and their host-side launchers.  All launchers are asynchronous on `stream`.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernel_types.hpp"

namespace sbc {

// Launchers.  `dump`, when not null, runs the kernel's verification variant,
// which also writes every source's levels, path counts and dependencies there.
hipError_t launch_ms(const DevPieces& P, const QueueArgs& Q, bool reach, bool ident, int waves, int eu, int grid,
                     const MsState& st, const DumpOut* dump, hipStream_t stream);
// Team kernel (a cooperative launch of `grid` workgroups in T.nteams teams);
// waves in {4, 8, 16}, eu in {0, 8} (0 for the dump variant).
hipError_t launch_team(const DevPieces& P, const QueueArgs& Q, bool reach, bool ident, int waves, int eu, int grid,
                       const MsState& st, const TeamArgs& T, const DumpOut* dump, hipStream_t stream);
// Small-piece kernel: one source per wavefront, pieces of at most np_max
// vertices and arcs_max arcs in LDS; waves in {4, 8}.
hipError_t launch_wave(const DevPieces& P, const QueueArgs& Q, bool reach, bool ident, int waves, int grid,
                       int32_t np_max, int32_t arcs_max, const DumpOut* dump, hipStream_t stream);
hipError_t launch_mapback(int32_t n, int32_t nverts, int32_t nmap, const int32_t* map_off, const int32_t* map_idx,
                          const double* bcp, const double* corr, const double* bcx, double scale, double* out,
                          hipStream_t stream);
// Deterministic runs: bcp[x] = sum over x's piece's items, in item order, of
// the item areas (see QueueArgs::item_base).
hipError_t launch_det_reduce(int32_t nverts, int32_t npieces, const int32_t* vtx_off, const int64_t* area_base,
                             const int32_t* piece_items, const double* item_out, double* bcp, hipStream_t stream);
// Farness kernel: per-source sums of reach x distance within each piece,
// sources 64 per item (the item's s0..s1-1 are piece-local ids); waves in
// {4, 8, 16}.
hipError_t launch_far(const DevPieces& P, const QueueArgs& Q, bool reach, int waves, int grid, const FarState& st,
                      int64_t* out, hipStream_t stream);
int occupancy_far(int waves);
hipError_t launch_copy(const void* src, void* dst, int64_t bytes, int grid, hipStream_t stream);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t stream);
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, int64_t count, hipStream_t stream);
hipError_t launch_fill_f64(double* p, double v, int64_t count, hipStream_t stream);

// Resident workgroups per compute unit (from the HIP occupancy calculator).
int occupancy_ms(int waves, int eu);
// 0 when the configuration is not built or cannot be resident.
int occupancy_team(int waves, int eu, bool dump);
int occupancy_wave(int waves, int32_t np_max, int32_t arcs_max);

// Largest LDS allocation a block may use on this device.
constexpr size_t kMaxLdsBytes = 160 * 1024;

}  // namespace sbc
