// fit.hip -- VELO track fit (paper Sec. 2.3.1, third and fourth paragraphs):
// a simple Kalman filter per projection with x and y independent, process
// noise from multiple scattering for a constant transverse momentum pt0,
// then the transport to the point of closest approach to the beamline.
//
// One lane per track, hits in decreasing z (the order in which track finding
// stores them); both projections advance in the same loop.  The arithmetic is the
// binary32 sequence below in this order (no contraction):
//   init at hit 1 from hits 0, 1:  u = m1, t = (m1-m0)/d, d = z1-z0,
//        C00 = s2, C01 = s2/d, C11 = (2 s2)/(d d)
//   per hit i >= 2:  C11 += dl*ms2 (dl = planes crossed), u += t*dz,
//        C00 += 2 dz C01 + dz dz C11, C01 += dz C11, r = m - u, S = C00 + s2,
//        K0 = C00/S, K1 = C01/S, u += K0 r, t += K1 r, C11 -= K1 C01,
//        C01 -= K0 C01, C00 -= K0 C00, chi2 += (r r)/S
//   ms2 = (184.96 X/X0 / pt0^2) t2/(1+t2), t2 = squared slope of hits 0, 1
//        (13.6 MeV Highland constant, p = pt0 sqrt(1+t2)/sqrt(t2))
//   beamline: dzb = -(x tx + y ty)/(tx tx + ty ty) (0 if the slope is below
//        1e-6), one plane of slope noise, then transport by dzb.
// With a measured momentum p per track (Sec. 2.3.5: the Velo segment fitted
// with the momentum of the whole track) ms2 = 184.96 X/X0 / p^2, and the
// transport to the beamline point stops at every plane between it and the
// last hit, adding ms2 to the slope variance at each; a p that is not a
// positive finite number falls back to the constant-pt0 fit.
#include "velo_device.hpp"
#include "mlp.hip"

namespace velo {

struct FitConst {
  float sig2;  // sigma_meas^2
  float kms;   // 184.96 * x_over_x0 / pt0^2
  float k184;  // 184.96 * x_over_x0
  float qc3, qc4;
};

struct Kf1 {
  float u, t, c00, c01, c11, chi2;
};

__device__ __forceinline__ void kf_step(Kf1& s, float m, float dz, float dl, float ms2, float sig2) {
  s.c11 = s.c11 + dl * ms2;
  s.u = s.u + s.t * dz;
  s.c00 = s.c00 + 2.0f * dz * s.c01 + dz * dz * s.c11;
  s.c01 = s.c01 + dz * s.c11;
  const float r = m - s.u;
  const float S = s.c00 + sig2;
  const float k0 = s.c00 / S;
  const float k1 = s.c01 / S;
  s.u = s.u + k0 * r;
  s.t = s.t + k1 * r;
  s.c11 = s.c11 - k1 * s.c01;
  s.c01 = s.c01 - k0 * s.c01;
  s.c00 = s.c00 - k0 * s.c00;
  s.chi2 = s.chi2 + (r * r) / S;
}

__device__ __forceinline__ void kf_transport(Kf1& s, float dz) {
  s.u = s.u + s.t * dz;
  s.c00 = s.c00 + 2.0f * dz * s.c01 + dz * dz * s.c11;
  s.c01 = s.c01 + dz * s.c11;
}

constexpr int kFitThreads = 256;

struct FitOut {
  float x, y, z, tx, ty, cx[3], cy[3], chi2;
  int ndof, n, lf, ll;  // hits, first and last plane
};

// Fit the track in `slot` (hits in decreasing z).  Returns false for a
// malformed track.  All hit indices, then all coordinates are loaded before
// the filter runs, so a track costs two memory round trips.  MOM: p_mev is
// the track's measured momentum (see the file header).
template <bool MOM = false>
__device__ __forceinline__ bool fit_track(const float* __restrict__ X, const float* __restrict__ Y,
                                          const uint32_t* __restrict__ key, uint64_t b, uint32_t ne,
                                          const uint8_t* __restrict__ nhits,
                                          const uint32_t* __restrict__ hit_idx, uint64_t slot,
                                          const FitConst& P, FitOut& o, float p_mev = 0.0f) {
  const int n = nhits[slot];
  if (n < 3 || n > kLayers) return false;
  const uint32_t* hi = hit_idx + 26ull * slot;
  uint32_t idx[kLayers];
#pragma unroll
  for (int j = 0; j < kLayers; ++j) idx[j] = j < n ? hi[j] : 0u;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < kLayers; ++j) ok &= idx[j] < ne;
  if (!ok) return false;
  float xs[kLayers], ys[kLayers];
  uint32_t ls[kLayers];
#pragma unroll
  for (int j = 0; j < kLayers; ++j) {
    if (j < n) {
      xs[j] = X[b + idx[j]];
      ys[j] = Y[b + idx[j]];
      const uint32_t lj = key[b + idx[j]] >> 22;
      ls[j] = lj < 26u ? lj : 25u;
    } else {
      xs[j] = 0.0f;
      ys[j] = 0.0f;
      ls[j] = 0u;
    }
  }
  const float z0 = kLayerZ[ls[0]], z1 = kLayerZ[ls[1]];
  const float d = z1 - z0;
  const float tx0 = (xs[1] - xs[0]) / d;
  const float ty0 = (ys[1] - ys[0]) / d;
  const float t2 = tx0 * tx0 + ty0 * ty0;
  bool thru = false;  // transport through the planes below the last hit
  float ms2;
  if constexpr (MOM) {
    thru = p_mev > 0.0f && p_mev <= 3.0e38f;
    ms2 = thru ? P.k184 / (p_mev * p_mev) : (P.kms * t2) / (1.0f + t2);
  } else {
    ms2 = (P.kms * t2) / (1.0f + t2);
  }
  const float s2 = P.sig2;
  Kf1 sx{xs[1], tx0, s2, s2 / d, (2.0f * s2) / (d * d), 0.0f};
  Kf1 sy{ys[1], ty0, s2, s2 / d, (2.0f * s2) / (d * d), 0.0f};
  float zp = z1;
  uint32_t lp = ls[1];
#pragma unroll
  for (int j = 2; j < kLayers; ++j) {
    if (j < n) {
      const float zj = kLayerZ[ls[j]];
      const float dz = zj - zp;
      const float dl = (float)((int)lp - (int)ls[j]);
      kf_step(sx, xs[j], dz, dl, ms2, s2);
      kf_step(sy, ys[j], dz, dl, ms2, s2);
      zp = zj;
      lp = ls[j];
    }
  }
  const float num = sx.u * sx.t + sy.u * sy.t;
  const float den = sx.t * sx.t + sy.t * sy.t;
  const float dzb = den < 1e-12f ? 0.0f : -(num / den);
  sx.c11 = sx.c11 + ms2;
  sy.c11 = sy.c11 + ms2;
  if (MOM && thru) {
    // plane by plane towards the beamline point, slope noise at each plane
    const float zb = zp + dzb;
    float zc = zp;
    for (int l = (int)lp - 1; l >= 0; --l) {
      const float zl = kLayerZ[l];
      if (!(zl > zb)) break;
      kf_transport(sx, zl - zc);
      kf_transport(sy, zl - zc);
      sx.c11 = sx.c11 + ms2;
      sy.c11 = sy.c11 + ms2;
      zc = zl;
    }
    kf_transport(sx, zb - zc);
    kf_transport(sy, zb - zc);
  } else {
    kf_transport(sx, dzb);
    kf_transport(sy, dzb);
  }
  o.x = sx.u; o.y = sy.u; o.z = zp + dzb; o.tx = sx.t; o.ty = sy.t;
  o.cx[0] = sx.c00; o.cx[1] = sx.c01; o.cx[2] = sx.c11;
  o.cy[0] = sy.c00; o.cy[1] = sy.c01; o.cy[2] = sy.c11;
  o.chi2 = sx.chi2 + sy.chi2;
  o.ndof = 2 * n - 4;
  o.n = n;
  o.lf = (int)ls[0];
  o.ll = (int)lp;
  return true;
}

__device__ __forceinline__ void store_state(const velo_states& o, uint64_t slot, const FitOut& f) {
  o.x[slot] = f.x;
  o.y[slot] = f.y;
  o.z[slot] = f.z;
  o.tx[slot] = f.tx;
  o.ty[slot] = f.ty;
  o.cov_x[3 * slot] = f.cx[0];
  o.cov_x[3 * slot + 1] = f.cx[1];
  o.cov_x[3 * slot + 2] = f.cx[2];
  o.cov_y[3 * slot] = f.cy[0];
  o.cov_y[3 * slot + 1] = f.cy[1];
  o.cov_y[3 * slot + 2] = f.cy[2];
  o.chi2[slot] = f.chi2;
  o.ndof[slot] = f.ndof;
}

// Plain form: one lane per track, plain chi2/hit-count cut.
template <int NT>
__global__ __launch_bounds__(NT) void k_fit(const float* __restrict__ X,
                                                     const float* __restrict__ Y,
                                                     const uint32_t* __restrict__ key,
                                                     const uint64_t* __restrict__ offsets,
                                                     uint64_t n_pixels,
                                                     const uint32_t* __restrict__ n_tracks,
                                                     const uint8_t* __restrict__ nhits,
                                                     const uint32_t* __restrict__ hit_idx,
                                                     FitConst P, velo_states o) {
  const uint32_t e = blockIdx.x;
  const uint64_t b = offsets[e], end = offsets[e + 1];
  if (end < b || end > n_pixels) return;
  const uint32_t ne = (uint32_t)(end - b);
  const uint64_t base = b / 3;
  const uint32_t nt = event_tracks(n_tracks[e], ne);
  for (uint32_t t = threadIdx.x; t < nt; t += NT) {
    const uint64_t slot = base + t;
    FitOut f;
    if (!fit_track(X, Y, key, b, ne, nhits, hit_idx, slot, P, f)) continue;
    store_state(o, slot, f);
    const float r = f.chi2 / (float)f.ndof;
    o.accepted[slot] = (uint8_t)(f.n >= 4 ? (r <= P.qc4) : (r <= P.qc3));
    if (o.score) o.score[slot] = r;
  }
}

// The fit with a measured momentum per track slot (p_mev[slot], MeV), plain
// chi2/hit-count cut.
template <int NT>
__global__ __launch_bounds__(NT) void k_fit_momentum(const float* __restrict__ X,
                                                     const float* __restrict__ Y,
                                                     const uint32_t* __restrict__ key,
                                                     const uint64_t* __restrict__ offsets,
                                                     uint64_t n_pixels,
                                                     const uint32_t* __restrict__ n_tracks,
                                                     const uint8_t* __restrict__ nhits,
                                                     const uint32_t* __restrict__ hit_idx,
                                                     const float* __restrict__ p_mev, FitConst P,
                                                     velo_states o) {
  const uint32_t e = blockIdx.x;
  const uint64_t b = offsets[e], end = offsets[e + 1];
  if (end < b || end > n_pixels) return;
  const uint32_t ne = (uint32_t)(end - b);
  const uint64_t base = b / 3;
  const uint32_t nt = event_tracks(n_tracks[e], ne);
  for (uint32_t t = threadIdx.x; t < nt; t += NT) {
    const uint64_t slot = base + t;
    FitOut f;
    if (!fit_track<true>(X, Y, key, b, ne, nhits, hit_idx, slot, P, f, p_mev[slot])) continue;
    store_state(o, slot, f);
    const float r = f.chi2 / (float)f.ndof;
    o.accepted[slot] = (uint8_t)(f.n >= 4 ? (r <= P.qc4) : (r <= P.qc3));
    if (o.score) o.score[slot] = r;
  }
}

// Learned form: the fit, the features and the BF16 MFMA classifier in one
// pass; every wave handles 64 consecutive tracks (all lanes take part in the
// matrix instructions), accepted = logit >= threshold.
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_fit_mlp(const float* __restrict__ X,
                                                         const float* __restrict__ Y,
                                                         const uint32_t* __restrict__ key,
                                                         const uint64_t* __restrict__ offsets,
                                                         uint64_t n_pixels,
                                                         const uint32_t* __restrict__ n_tracks,
                                                         const uint8_t* __restrict__ nhits,
                                                         const uint32_t* __restrict__ hit_idx,
                                                         FitConst P, const float* __restrict__ mp,
                                                         const float* __restrict__ mmean,
                                                         const float* __restrict__ mstd,
                                                         float threshold, velo_states o) {
  __shared__ MlpLds L;
  mlp_load(L, mp, mmean, mstd, NT);
  __syncthreads();
  const uint32_t e = blockIdx.x;
  const uint64_t b = offsets[e], end = offsets[e + 1];
  if (end < b || end > n_pixels) return;
  const uint32_t ne = (uint32_t)(end - b);
  const uint64_t base = b / 3;
  const uint32_t nt = event_tracks(n_tracks[e], ne);
  for (uint32_t t0 = 0; t0 < nt; t0 += NT) {
    const uint32_t t = t0 + threadIdx.x;
    const uint64_t slot = base + t;
    FitOut f;
    const bool ok = t < nt && fit_track(X, Y, key, b, ne, nhits, hit_idx, slot, P, f);
    float feat[kNF];
    if (ok) track_features(f.chi2, f.ndof, f.n, f.lf, f.ll, f.tx, f.ty, feat);
    else
      for (int k = 0; k < kNF; ++k) feat[k] = L.mean[k];
    // the whole wave runs the classifier (uniform per wave: t0 is uniform)
    const bool wave_live = __any(ok);
    float z = 0.0f;
    if (wave_live) z = mlp_wave_logit(L, feat);
    if (ok) {
      store_state(o, slot, f);
      o.accepted[slot] = (uint8_t)(z >= threshold);
      o.score[slot] = z;
    }
  }
}

FitConst make_fit_const(const velo_params* p) {
  FitConst c;
  c.sig2 = p->sigma_meas * p->sigma_meas;
  c.kms = (184.96f * p->x_over_x0) / (p->pt0_mev * p->pt0_mev);
  c.k184 = 184.96f * p->x_over_x0;
  c.qc3 = p->qc3;
  c.qc4 = p->qc4;
  return c;
}

template <int NT>
static void fit_kernels(const velo_hits* h, const velo_tracks* t, const uint64_t* offsets,
                        uint32_t n_events, uint64_t n_pixels, const FitConst& c, const velo_mlp* m,
                        const velo_states* o, hipStream_t s) {
  if (m)
    hipLaunchKernelGGL(k_fit_mlp<NT>, dim3(n_events), dim3(NT), 0, s, h->x, h->y, h->key, offsets,
                       n_pixels, t->n_tracks, t->nhits, t->hit_idx, c, m->params, m->mean, m->std,
                       m->threshold, *o);
  else
    hipLaunchKernelGGL(k_fit<NT>, dim3(n_events), dim3(NT), 0, s, h->x, h->y, h->key, offsets,
                       n_pixels, t->n_tracks, t->nhits, t->hit_idx, c, *o);
}

// threads: 64, 128 or 256 lanes per event (the batched form's autotuner picks it)
// ev (may be null): events recorded just before and after the fit kernel
hipError_t launch_fit_cfg(const velo_hits* h, const velo_tracks* t, const uint64_t* offsets,
                          uint32_t n_events, uint64_t n_pixels, const velo_params* p,
                          const velo_mlp* m, const velo_states* o, hipStream_t s, int threads,
                          const hipEvent_t* ev = nullptr) {
  const FitConst c = make_fit_const(p);
  if (ev && ev[0]) (void)hipEventRecord(ev[0], s);
  if (threads == 64) fit_kernels<64>(h, t, offsets, n_events, n_pixels, c, m, o, s);
  else if (threads == 256) fit_kernels<256>(h, t, offsets, n_events, n_pixels, c, m, o, s);
  else fit_kernels<kFitThreads>(h, t, offsets, n_events, n_pixels, c, m, o, s);
  if (ev && ev[1]) (void)hipEventRecord(ev[1], s);
  return hipGetLastError();
}

hipError_t launch_fit(const velo_hits* h, const velo_tracks* t, const uint64_t* offsets,
                      uint32_t n_events, uint64_t n_pixels, const velo_params* p,
                      const velo_states* o, hipStream_t s) {
  return launch_fit_cfg(h, t, offsets, n_events, n_pixels, p, nullptr, o, s, kFitThreads);
}

hipError_t launch_fit_mlp(const velo_hits* h, const velo_tracks* t, const uint64_t* offsets,
                          uint32_t n_events, uint64_t n_pixels, const velo_params* p,
                          const velo_mlp* m, const velo_states* o, hipStream_t s) {
  return launch_fit_cfg(h, t, offsets, n_events, n_pixels, p, m, o, s, kFitThreads);
}

hipError_t launch_fit_momentum(const velo_hits* h, const velo_tracks* t, const uint64_t* offsets,
                               uint32_t n_events, uint64_t n_pixels, const velo_params* p,
                               const float* p_mev, const velo_states* o, hipStream_t s) {
  const FitConst c = make_fit_const(p);
  hipLaunchKernelGGL(k_fit_momentum<kFitThreads>, dim3(n_events), dim3(kFitThreads), 0, s, h->x, h->y,
                     h->key, offsets, n_pixels, t->n_tracks, t->nhits, t->hit_idx, p_mev, c, *o);
  return hipGetLastError();
}

}  // namespace velo
