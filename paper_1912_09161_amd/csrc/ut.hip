// ut.hip -- Velo-to-UT search windows (paper Sec. 2.3.2).
//
// The upstream tracker (UT) is read as four planes of silicon strips
// (outer two vertical, inner two tilted by +5 and -5 degrees); its hits are
// single strips, decoded into regions and sorted so that the hits near an
// extrapolated Velo track are found at once, and every Velo track is
// extrapolated to the UT with the largest bending a particle of at least
// p_min can take.  The model (plane positions, strips, sensor rows, raw
// word, single transverse kick) is the one stated in include/velo.h.
//
// One 256-lane workgroup per event:
//   1. the event's words (at most kUtMaxHits) are loaded into LDS and
//      checked (offsets rule from k_offsets, count, bad words);
//   2. a bitonic sort in LDS orders them by the 19-bit word, i.e. by plane,
//      sensor row, strip: each region (plane, sensor row) becomes a run
//      sorted along u; equal neighbours flag a duplicate;
//   3. region starts are read off the sorted run;
//   4. one lane per accepted track: the straight line from the beamline
//      state to each plane, the sensor rows it may cross, and in each such
//      region two binary searches for the first hit with u >= up - w and the
//      first with u > up + w (u grows with the strip number, so this is the
//      run of hits inside the window, found without scanning it).
#include "velo_device.hpp"

namespace velo {

constexpr uint32_t kUtMaxHits = 8192;
constexpr uint32_t kUtSectors = 14;
constexpr uint32_t kUtRegions = 4 * kUtSectors;
constexpr int kUtThreads = 256;

__constant__ const float kUtZ[4] = {2327.5f, 2372.5f, 2597.5f, 2642.5f};
__constant__ const float kUtC[4] = {1.0f, 0.9961947f, 0.9961947f, 1.0f};
__constant__ const float kUtS[4] = {0.0f, 0.08715574f, -0.08715574f, 0.0f};

// u of a strip's centre, exact in binary32
__device__ __forceinline__ float ut_u(uint32_t strip) { return ((float)strip + 0.5f) * 0.1875f - 768.0f; }
__device__ __forceinline__ uint32_t ut_region(uint32_t w) { return (w >> 17) * kUtSectors + ((w >> 13) & 15u); }

struct UtConst {
  float p_min, kick, z_kick, tol_u, tol_y;
};

struct UtState {
  const float *x, *y, *z, *tx, *ty;
  const uint8_t* accepted;
};

// first h in [lo, hi) with pred(h) true, pred monotone (false ... true)
template <class F>
__device__ __forceinline__ uint32_t lower_bound(uint32_t lo, uint32_t hi, F pred) {
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (pred(mid)) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// status[e] holds the offsets check (k_offsets on the UT offsets) on entry.
__global__ __launch_bounds__(kUtThreads) void k_ut(const uint32_t* __restrict__ words,
                                                   const uint64_t* __restrict__ ut_off,
                                                   const uint64_t* __restrict__ offsets, uint64_t n_pixels,
                                                   const uint32_t* __restrict__ n_tracks, UtState S,
                                                   UtConst C, uint32_t* __restrict__ sorted,
                                                   uint32_t* __restrict__ region,
                                                   uint32_t* __restrict__ status,
                                                   uint32_t* __restrict__ win) {
  __shared__ uint32_t sw[kUtMaxHits];
  __shared__ uint32_t sreg[kUtRegions + 1];
  __shared__ uint32_t sflag;
  const uint32_t e = blockIdx.x, tid = threadIdx.x;
  uint32_t st = status[e];
  const uint64_t ub = ut_off[e];
  uint32_t n = 0;
  if (st == 0) {
    const uint64_t nn = ut_off[e + 1] - ub;
    if (nn > kUtMaxHits) st = VELO_EV_UT_OVERFLOW;
    else n = (uint32_t)nn;
  }
  if (tid == 0) sflag = 0;
  __syncthreads();
  // 1. load and check
  uint32_t P = 1;
  if (st == 0) {
    while (P < n) P <<= 1;
    uint32_t bad = 0;
    for (uint32_t i = tid; i < P; i += kUtThreads) {
      uint32_t w = 0xFFFFFFFFu;  // padding sorts last
      if (i < n) {
        w = words[ub + i];
        if ((w >> 19) != 0u || ((w >> 13) & 15u) >= kUtSectors) bad = 1;
      }
      sw[i] = w;
    }
    if (bad) atomicOr(&sflag, VELO_EV_BAD_WORD);
  }
  __syncthreads();
  st |= sflag;
  // 2. bitonic sort of sw[0, P)
  if (st == 0 && n > 1) {
    for (uint32_t k = 2; k <= P; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        for (uint32_t t = tid; t < (P >> 1); t += kUtThreads) {
          const uint32_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
          const uint32_t a = sw[i], c = sw[i + j];
          const bool up = (i & k) == 0;
          if ((a > c) == up) {
            sw[i] = c;
            sw[i + j] = a;
          }
        }
        __syncthreads();
      }
    }
    uint32_t dup = 0;
    for (uint32_t i = tid + 1; i < n; i += kUtThreads) dup |= sw[i] == sw[i - 1];
    if (dup) atomicOr(&sflag, VELO_EV_DUPLICATE);
    __syncthreads();
    st |= sflag;
  }
  // 3. region starts: region r begins at the first word whose region is >= r
  if (st == 0) {
    for (uint32_t i = tid; i < n; i += kUtThreads) {
      const uint32_t r = ut_region(sw[i]);
      const int rp = i ? (int)ut_region(sw[i - 1]) : -1;
      for (int q = rp + 1; q <= (int)r; ++q) sreg[q] = i;
    }
    if (tid == 0) {
      const uint32_t rl = n ? ut_region(sw[n - 1]) : 0u;
      for (uint32_t q = n ? rl + 1 : 0u; q <= kUtRegions; ++q) sreg[q] = n;
    }
    for (uint32_t i = tid; i < n; i += kUtThreads) sorted[ub + i] = sw[i];
  } else {
    for (uint32_t q = tid; q <= kUtRegions; q += kUtThreads) sreg[q] = 0;
  }
  __syncthreads();
  for (uint32_t q = tid; q <= kUtRegions; q += kUtThreads) region[(uint64_t)(kUtRegions + 1) * e + q] = sreg[q];
  if (tid == 0) status[e] = st;
  // 4. windows of the event's track slots
  const uint64_t b = offsets[e], end = offsets[e + 1];
  const uint32_t cap = (end >= b && end <= n_pixels) ? (uint32_t)((end - b) / 3) : 0u;
  const uint32_t nt = n_tracks[e] < cap ? n_tracks[e] : cap;
  const float dtx = C.kick / C.p_min;
  for (uint32_t t = tid; t < nt; t += kUtThreads) {
    const uint64_t s = b / 3 + t;
    uint32_t o[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (st == 0 && S.accepted[s]) {
      const float x = S.x[s], y = S.y[s], z = S.z[s], tx = S.tx[s], ty = S.ty[s];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float w = (dtx * (kUtZ[k] - C.z_kick)) * kUtC[k] + C.tol_u;
        const float dz = kUtZ[k] - z;
        const float xp = x + tx * dz;
        const float yp = y + ty * dz;
        const float up = xp * kUtC[k] + yp * kUtS[k];
        const float lo = up - w, hi = up + w;
        int i = 0;
        for (uint32_t j = 0; j < kUtSectors && i < 2; ++j) {
          const float ylo = -700.0f + 100.0f * (float)j, yhi = ylo + 100.0f;
          if (!(yp + C.tol_y >= ylo && yp - C.tol_y < yhi)) continue;
          const uint32_t r = (uint32_t)k * kUtSectors + j;
          const uint32_t r0 = sreg[r], r1 = sreg[r + 1];
          const uint32_t a = lower_bound(r0, r1, [&](uint32_t h) { return ut_u(sw[h] & 8191u) >= lo; });
          const uint32_t c = lower_bound(r0, r1, [&](uint32_t h) { return !(ut_u(sw[h] & 8191u) <= hi); });
          const uint32_t count = c > a ? c - a : 0u;
          o[2 * k + i] = count ? (a | count << 16) : 0u;
          ++i;
        }
      }
    }
    uint4* dst = reinterpret_cast<uint4*>(win + 8 * s);
    dst[0] = make_uint4(o[0], o[1], o[2], o[3]);
    dst[1] = make_uint4(o[4], o[5], o[6], o[7]);
  }
}

hipError_t launch_ut(const uint32_t* words, const uint64_t* ut_off, uint32_t n_events, uint64_t n_ut,
                     const uint64_t* offsets, uint64_t n_pixels, const velo_tracks* t,
                     const velo_states* s, const velo_ut_params* p, const velo_ut_out* out,
                     hipStream_t stream) {
  hipLaunchKernelGGL(k_offsets, dim3(1), dim3(kOffThreads), 0, stream, ut_off, n_events, n_ut, out->status);
  const UtState S{s->x, s->y, s->z, s->tx, s->ty, s->accepted};
  const UtConst C{p->p_min_mev, p->kick_mev, p->z_kick, p->tol_u, p->tol_y};
  hipLaunchKernelGGL(k_ut, dim3(n_events), dim3(kUtThreads), 0, stream, words, ut_off, offsets, n_pixels,
                     t->n_tracks, S, C, out->sorted, out->region, out->status, out->win);
  return hipGetLastError();
}

}  // namespace velo
