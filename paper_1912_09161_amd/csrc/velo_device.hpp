// velo_device.hpp -- device-side constants and helpers shared by the HIP
// kernels of libvelo (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/velo.h"

namespace velo {

constexpr int kLayers = 26;
constexpr int kPix = 1536;
constexpr int kWave = 64;

// Plane positions: -280 mm + 1030 mm * l / 25, evaluated in double and
// rounded once to binary32 (constant-folded at compile time).
#define VELO_Z(l) ((float)(-280.0 + 1030.0 * (double)(l) / 25.0))
__constant__ const float kLayerZ[kLayers] = {
    VELO_Z(0),  VELO_Z(1),  VELO_Z(2),  VELO_Z(3),  VELO_Z(4),  VELO_Z(5),  VELO_Z(6),
    VELO_Z(7),  VELO_Z(8),  VELO_Z(9),  VELO_Z(10), VELO_Z(11), VELO_Z(12), VELO_Z(13),
    VELO_Z(14), VELO_Z(15), VELO_Z(16), VELO_Z(17), VELO_Z(18), VELO_Z(19), VELO_Z(20),
    VELO_Z(21), VELO_Z(22), VELO_Z(23), VELO_Z(24), VELO_Z(25)};
#undef VELO_Z

// raw word fields
__device__ __forceinline__ uint32_t w_col(uint32_t w) { return w & 0x7FFu; }
__device__ __forceinline__ uint32_t w_row(uint32_t w) { return (w >> 11) & 0x7FFu; }
__device__ __forceinline__ uint32_t w_layer(uint32_t w) { return (w >> 22) & 31u; }
__device__ __forceinline__ uint32_t w_charge(uint32_t w) { return (w >> 27) & 15u; }

// inactive pixel: centre radius < 5.1 mm, in exact integer form
// Track slots of an event with ne raw words: every track holds at least three
// distinct hits and an event has at most ne hits, so a count above ne / 3
// cannot come from the track finding and is clamped (the event's slots end
// there; no slot of another event is touched).
__device__ __forceinline__ uint32_t event_tracks(uint32_t n_tracks, uint32_t ne) {
  return n_tracks < ne / 3 ? n_tracks : ne / 3;
}

__device__ __forceinline__ bool in_hole(uint32_t col, uint32_t row) {
  int dc = 2 * (int)col - 1535, dr = 2 * (int)row - 1535;
  return dc * dc + dr * dr <= 34393;
}

// exclusive prefix count of `pred` over the 64 lanes of the calling wave;
// *total receives the wave's count
__device__ __forceinline__ uint32_t wave_prefix(bool pred, uint32_t* total) {
  uint64_t m = __ballot(pred);
  *total = (uint32_t)__popcll(m);
  uint32_t lo = __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u);
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), lo);
}

// Workgroup barrier.  LDS_ONLY: orders LDS accesses only, so outstanding
// global stores (results nobody in the workgroup reads back) do not delay it.
template <bool LDS_ONLY>
__device__ __forceinline__ void wg_barrier() {
  if constexpr (LDS_ONLY) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  } else {
    __syncthreads();
  }
}

// Inclusive scan of v over the 64 lanes of the calling wave without LDS
// round trips: Hillis-Steele steps inside each 16-lane row by DPP row shifts
// (1, 2, 4, 8; lanes shifted in from outside the row read 0), then the row
// totals carried across rows by the row_bcast:15 (rows 1, 3) and
// row_bcast:31 (rows 2, 3) broadcasts.  Every lane of the wave must be
// active (all callers are in wave-uniform control flow).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  uint32_t x = v;
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);   // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);   // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true);   // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true);   // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}

// Workgroup exclusive scan of one value per thread; NT threads, `tmp` holds
// NT/64 + 1 uint32 of LDS.  Returns the exclusive prefix; *total = sum.
template <int NT, bool LDS_ONLY = false>
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const uint32_t x = wave_incl_scan(v);
  if constexpr (NW == 1) {
    *total = __builtin_amdgcn_readlane(x, kWave - 1);
    return x - v;
  } else {
    if (lane == kWave - 1) tmp[wid] = x;
    wg_barrier<LDS_ONLY>();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      uint32_t t = tmp[w];
      if (w < wid) base += t;
      tot += t;
    }
    wg_barrier<LDS_ONLY>();
    *total = tot;
    return base + x - v;
  }
}

// Workgroup exclusive scan with a single barrier: `tmp` (NT/64 words of LDS)
// must not be reused by the next scan, so callers alternate two buffers (the
// barrier of the next scan orders the reads of this one before any reuse).
template <int NT, bool LDS_ONLY = false>
__device__ __forceinline__ uint32_t block_scan1(uint32_t v, uint32_t* tmp, uint32_t* total) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const uint32_t x = wave_incl_scan(v);
  if constexpr (NW == 1) {
    *total = __builtin_amdgcn_readlane(x, kWave - 1);
    return x - v;
  } else {
    if (lane == kWave - 1) tmp[wid] = x;
    wg_barrier<LDS_ONLY>();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      uint32_t t = tmp[w];
      if (w < wid) base += t;
      tot += t;
    }
    *total = tot;
    return base + x - v;
  }
}

}  // namespace velo
