// azimuth.hpp -- azimuth bucket tables of the hits of one (event, plane)
// (paper Sec. 2.3.1: hits of every plane kept in azimuth order for fast
// look-up), built by the track-finding stage from the hits.
#pragma once

#include "velo_device.hpp"

namespace velo {

constexpr uint32_t kNB = 256;  // azimuth buckets per plane

// Upper bound of the pseudo-angle's derivative with respect to the azimuth:
// an azimuth window of half width d lies inside the pseudo-angle window of
// half width kPaSlope * d.
constexpr float kPaSlope = 0.6502f;

// Monotone pseudo-angle of (x, y) in [0, 4]: in every octant, with u the
// ratio of the smaller to the larger of |x| and |y|, g(u) = 0.64 u /
// (1 + 0.28 u^2) (a rational approximation of 2 atan(u) / pi, g(1) = 1/2).
// Its derivative with respect to the azimuth lies in [0.5625, 0.6502] (2/pi is
// 0.6366), so buckets of equal pseudo-angle width cover nearly equal azimuth
// ranges and windows stay close to the exact azimuth windows.
__device__ __forceinline__ float pangle(float x, float y) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mn = fminf(ax, ay), mx = fmaxf(ax, ay);
  // hardware reciprocals (about 1 ulp): bucket assignment and window centres use
  // this same function, and every window carries a margin far above its error
  const float u = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
  const float g = (0.64f * u) * __builtin_amdgcn_rcpf(1.0f + (0.28f * u) * u);
  const float r = ay <= ax ? g : 1.0f - g;  // from the x axis towards the y axis
  if (y >= 0.0f) return x >= 0.0f ? r : 2.0f - r;
  return x < 0.0f ? 2.0f + r : 4.0f - r;
}

__device__ __forceinline__ uint32_t bucket_of(float pa, uint32_t nb) {
  int b = (int)(pa * (float)nb * 0.25f);
  return b < 0 ? 0u : (b >= (int)nb ? nb - 1 : (uint32_t)b);
}

// Destination of the tables (the track-finding workspace, at the hits' slots):
// at every bucket position the hit's local index and coordinates, and per
// (event, plane) the kNB + 1 bucket starts.
struct AzOut {
  uint32_t* order;
  float* xs;
  float* ys;
  uint32_t* bst;
};

// Counting sort of the n hits at slots [base, base + n) into kNB buckets with
// NT lanes; `cnt` holds kNB words of LDS, `tmp` NT/64 + 1 words.
template <int NT>
__device__ void azimuth_tables(const float* __restrict__ X, const float* __restrict__ Y,
                               uint64_t base, uint32_t n, uint64_t seg, uint32_t* cnt, uint32_t* tmp,
                               const AzOut& az) {
  uint32_t* bs = az.bst + seg * (kNB + 1);
  for (uint32_t b = threadIdx.x; b < kNB; b += NT) cnt[b] = 0;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += NT)
    atomicAdd(cnt + bucket_of(pangle(X[base + i], Y[base + i]), kNB), 1u);
  __syncthreads();
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < kNB; b0 += NT) {
    const uint32_t b = b0 + threadIdx.x;
    const uint32_t c = b < kNB ? cnt[b] : 0u;
    uint32_t tot;
    const uint32_t ex = block_scan<NT>(c, tmp, &tot);
    if (b < kNB) { bs[b] = carry + ex; cnt[b] = carry + ex; }
    carry += tot;
  }
  if (threadIdx.x == 0) bs[kNB] = carry;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += NT) {
    const float x = X[base + i], y = Y[base + i];
    const uint64_t p = base + atomicAdd(cnt + bucket_of(pangle(x, y), kNB), 1u);
    az.order[p] = i;
    az.xs[p] = x;
    az.ys[p] = y;
  }
}

}  // namespace velo
