// pv.hip -- primary-vertex finding on the fitted Velo tracks (paper Sec.
// 2.3.1, last paragraph: PV candidates are clusters in a histogram of the
// tracks' points of closest approach to the beamline; every track is
// assigned to every candidate with a weight, so all candidates are fitted
// in parallel instead of one after another).
//
// One workgroup per event, everything in LDS:
//   admission   accepted tracks whose slope is not along the beam and whose
//               beamline-z variance (tx^2 var_x + ty^2 var_y) / t^4 is at most
//               max_var, inside the histogram range; compacted in slot order
//               by a workgroup prefix scan (at most kPvTracks per event)
//   histogram   integer counts with LDS atomics: 2 in the track's bin, 1 in
//               each neighbour (sums of integers do not depend on order)
//   candidates  one lane per bin: count >= seed_min, strictly above the nms
//               bins before, at least the nms bins after; compacted in bin
//               order (at most VELO_MAX_PVS)
//   fit         n_iter rounds: lanes over tracks form each track's share
//               denominator sum_u r_u over the candidates (Tukey weights
//               r = (1 - chi2/cut)^2); then one lane per candidate sums
//               w / var and w z / var over the tracks in slot order, w =
//               r (r / share); new positions replace the old ones together
//   output      weights at the final positions give var = 1 / sum(w / var)
//               and the weight sum; candidates with weight sum >= min_weight
//               are the event's PVs, in candidate order.
// Every float expression is the same sequence of binary32 operations as the
// method's definition (sums in the stated order, no contraction), so the
// results are reproducible bit for bit.
#include "velo_device.hpp"

namespace velo {

constexpr int kPvThreads = 256;
constexpr uint32_t kPvTracks = 2048;  // admitted tracks of one event held in LDS
constexpr int kPvBins = 1024;         // histogram bins held in LDS (n_bins <= this)

struct PvConst {
  float z0, bin_w, zhi, max_var, chi2_cut, min_weight;
  int32_t n_bins, seed_min, nms, n_iter;
};

__device__ __forceinline__ float pv_tukey(float z, float var, float zv, float cut) {
  const float d = z - zv;
  const float c = (d * d) / var;
  if (!(c < cut)) return 0.0f;
  const float q = 1.0f - c / cut;
  return q * q;
}

struct PvLds {
  float tz[kPvTracks], tv[kPvTracks], share[kPvTracks];
  uint32_t hist[kPvBins];
  float cz[VELO_MAX_PVS], nz[VELO_MAX_PVS], cvar[VELO_MAX_PVS], cw[VELO_MAX_PVS];
  uint32_t scan[2][kPvThreads / kWave];
};

__global__ __launch_bounds__(kPvThreads) void k_find_pvs(
    const uint64_t* __restrict__ offsets, uint64_t n_pixels, const uint32_t* __restrict__ n_tracks,
    const float* __restrict__ sz, const float* __restrict__ stx, const float* __restrict__ sty,
    const float* __restrict__ cov_x, const float* __restrict__ cov_y,
    const uint8_t* __restrict__ accepted, PvConst P, velo_pvs o) {
  __shared__ PvLds L;
  const uint32_t e = blockIdx.x, tid = threadIdx.x;
  const uint64_t b = offsets[e], end = offsets[e + 1];
  const uint32_t nt = (b <= end && end <= n_pixels) ? event_tracks(n_tracks[e], (uint32_t)(end - b)) : 0u;
  const uint64_t base = b / 3;

  // admission, compacted in slot order
  uint32_t n = 0;
  int buf = 0;
  for (uint32_t t0 = 0; t0 < nt; t0 += kPvThreads, buf ^= 1) {
    const uint32_t t = t0 + tid;
    bool adm = false;
    float z = 0.0f, var = 0.0f;
    if (t < nt) {
      const uint64_t s = base + t;
      if (accepted[s]) {
        const float tx = stx[s], ty = sty[s];
        const float t2 = tx * tx + ty * ty;
        if (t2 >= 1e-6f) {
          var = (tx * tx * cov_x[3 * s] + ty * ty * cov_y[3 * s]) / (t2 * t2);
          z = sz[s];
          adm = var <= P.max_var && var > 0.0f && z >= P.z0 && z < P.zhi;
        }
      }
    }
    uint32_t tot;
    const uint32_t pos = n + block_scan1<kPvThreads, true>(adm ? 1u : 0u, L.scan[buf], &tot);
    if (adm && pos < kPvTracks) {
      L.tz[pos] = z;
      L.tv[pos] = var;
    }
    n += tot;
  }
  if (n > kPvTracks) {  // more admitted tracks than the tables hold: no PVs
    if (tid == 0) {
      o.n_pv[e] = 0;
      o.status[e] = VELO_EV_PV_OVERFLOW;
    }
    for (uint32_t k = tid; k < VELO_MAX_PVS; k += kPvThreads) {
      const uint64_t j = (uint64_t)e * VELO_MAX_PVS + k;
      o.z[j] = 0.0f;
      o.var[j] = 0.0f;
      o.weight[j] = 0.0f;
    }
    return;
  }

  // histogram
  for (int k = tid; k < P.n_bins; k += kPvThreads) L.hist[k] = 0;
  __syncthreads();
  for (uint32_t i = tid; i < n; i += kPvThreads) {
    const int32_t bin = (int32_t)floorf((L.tz[i] - P.z0) / P.bin_w);
    if (bin < 0 || bin >= P.n_bins) continue;
    atomicAdd(&L.hist[bin], 2u);
    if (bin > 0) atomicAdd(&L.hist[bin - 1], 1u);
    if (bin + 1 < P.n_bins) atomicAdd(&L.hist[bin + 1], 1u);
  }
  __syncthreads();

  // candidates in bin order
  uint32_t nc = 0;
  bool ovf = false;
  for (int b0 = 0; b0 < P.n_bins; b0 += kPvThreads, buf ^= 1) {
    const int bin = b0 + (int)tid;
    bool cand = false;
    if (bin < P.n_bins) {
      const uint32_t h = L.hist[bin];
      cand = h >= (uint32_t)P.seed_min;
      for (int c = bin - P.nms; c < bin && cand; ++c)
        if (c >= 0 && !(h > L.hist[c])) cand = false;
      for (int c = bin + 1; c <= bin + P.nms && cand; ++c)
        if (c < P.n_bins && !(h >= L.hist[c])) cand = false;
    }
    uint32_t tot;
    const uint32_t pos = nc + block_scan1<kPvThreads, true>(cand ? 1u : 0u, L.scan[buf], &tot);
    if (cand && pos < VELO_MAX_PVS) L.cz[pos] = P.z0 + ((float)bin + 0.5f) * P.bin_w;
    nc += tot;
  }
  if (nc > VELO_MAX_PVS) {
    ovf = true;
    nc = VELO_MAX_PVS;
  }
  __syncthreads();

  // fit rounds; the last pass evaluates the weights at the final positions
  for (int it = 0; it <= P.n_iter; ++it) {
    for (uint32_t i = tid; i < n; i += kPvThreads) {
      const float zi = L.tz[i], vi = L.tv[i];
      float s = 0.0f;
      for (uint32_t v = 0; v < nc; ++v) s = s + pv_tukey(zi, vi, L.cz[v], P.chi2_cut);
      L.share[i] = s;
    }
    __syncthreads();
    for (uint32_t v = tid; v < nc; v += kPvThreads) {
      const float zv = L.cz[v];
      float sa = 0.0f, saz = 0.0f, sw = 0.0f;
      for (uint32_t i = 0; i < n; ++i) {
        const float zi = L.tz[i], vi = L.tv[i];
        const float r = pv_tukey(zi, vi, zv, P.chi2_cut);
        if (!(r > 0.0f)) continue;
        const float w = r * (r / L.share[i]);
        const float a = w / vi;
        sa = sa + a;
        saz = saz + a * zi;
        sw = sw + w;
      }
      if (it < P.n_iter) {
        L.nz[v] = sa > 0.0f ? saz / sa : zv;
      } else {
        L.cvar[v] = sa > 0.0f ? 1.0f / sa : 0.0f;
        L.cw[v] = sw;
      }
    }
    __syncthreads();
    if (it < P.n_iter) {
      for (uint32_t v = tid; v < nc; v += kPvThreads) L.cz[v] = L.nz[v];
      __syncthreads();
    }
  }

  // PVs in candidate order (one wave: VELO_MAX_PVS == 64 candidates)
  static_assert(VELO_MAX_PVS == kWave, "one wave compacts the candidates");
  if (tid < kWave) {
    const bool keep = tid < nc && L.cw[tid] >= P.min_weight;
    uint32_t tot;
    const uint32_t pos = wave_prefix(keep, &tot);
    const uint64_t row = (uint64_t)e * VELO_MAX_PVS;
    if (keep) {
      o.z[row + pos] = L.cz[tid];
      o.var[row + pos] = L.cvar[tid];
      o.weight[row + pos] = L.cw[tid];
    }
    if (tid >= tot) {
      o.z[row + tid] = 0.0f;
      o.var[row + tid] = 0.0f;
      o.weight[row + tid] = 0.0f;
    }
    if (tid == 0) {
      o.n_pv[e] = tot;
      o.status[e] = ovf ? VELO_EV_PV_OVERFLOW : 0u;
    }
  }
}

PvConst make_pv_const(const velo_pv_params* p) {
  PvConst c;
  c.z0 = p->z0;
  c.bin_w = p->bin_w;
  c.n_bins = p->n_bins;
  c.zhi = p->z0 + p->bin_w * (float)p->n_bins;
  c.max_var = p->max_var;
  c.seed_min = p->seed_min;
  c.nms = p->nms;
  c.chi2_cut = p->chi2_cut;
  c.n_iter = p->n_iter;
  c.min_weight = p->min_weight;
  return c;
}

hipError_t launch_find_pvs(const velo_tracks* t, const velo_states* s, const uint64_t* offsets,
                           uint32_t n_events, uint64_t n_pixels, const velo_pv_params* p,
                           const velo_pvs* o, hipStream_t stream) {
  hipLaunchKernelGGL(k_find_pvs, dim3(n_events), dim3(kPvThreads), 0, stream, offsets, n_pixels,
                     t->n_tracks, s->z, s->tx, s->ty, s->cov_x, s->cov_y, s->accepted,
                     make_pv_const(p), *o);
  return hipGetLastError();
}

}  // namespace velo
