// mlp.hip -- learned track-quality classifier: features after the fit, FP32
// training kernels (forward, backward, Adam) and BF16 MFMA inference fused
// into the fit.
//
// Not part of the paper; it replaces the plain chi2/hit-count cut after the
// simple Kalman fit of Sec. 2.3.1 (the plain cut stays available as
// velo_fit).  Features of a track (binary32): chi2/ndof, hits n, missed
// planes (l_first - l_last + 1) - n, tx, ty, eta = asinh(1/sqrt(tx^2+ty^2)),
// z of the first and of the last hit plane; standardised with the training
// mean and standard deviation.  Network 8 -> 32 (relu) -> 32 (relu) -> 1,
// 1377 parameters stored flat: W1[32][8], b1[32], W2[32][32], b2[32],
// w3[32], b3.  Loss: mean binary cross-entropy with logits.
//
// Training (FP32): one lane per sample computes the forward and backward
// pass and leaves its activations in LDS; the workgroup then sums every
// parameter's gradient over its samples in a fixed order, and a second
// kernel sums the workgroups in a fixed order, so gradients are
// deterministic.  Inference: bfloat16 weights and activations (round to
// nearest even) into v_mfma_f32_16x16x32_bf16, FP32 accumulation, 64 tracks
// per wave.
#include "velo_device.hpp"

namespace velo {

constexpr int kNF = 8, kNH = 32, kNP = 1377;
constexpr int kOW1 = 0, kOB1 = 256, kOW2 = 288, kOB2 = 1312, kOW3 = 1344, kOB3 = 1376;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void track_features(float chi2, int ndof, int n, int lf, int ll, float tx,
                                               float ty, float* f) {
  f[0] = chi2 / (float)ndof;
  f[1] = (float)n;
  f[2] = (float)((lf - ll + 1) - n);
  f[3] = tx;
  f[4] = ty;
  float t2 = tx * tx + ty * ty;
  if (t2 < 1e-12f) t2 = 1e-12f;
  f[5] = asinhf(1.0f / sqrtf(t2));
  f[6] = kLayerZ[lf];
  f[7] = kLayerZ[ll];
}

// ---------------------------------------------------------------------------
// features of every track slot

__global__ __launch_bounds__(128) void k_features(const uint32_t* __restrict__ key,
                                                  const uint64_t* __restrict__ offsets,
                                                  uint64_t n_pixels,
                                                  const uint32_t* __restrict__ n_tracks,
                                                  const uint8_t* __restrict__ nhits,
                                                  const uint32_t* __restrict__ hit_idx,
                                                  velo_states s, float* __restrict__ feat) {
  const uint32_t e = blockIdx.x;
  const uint64_t b = offsets[e], end = offsets[e + 1];
  if (end < b || end > n_pixels) return;
  const uint32_t ne = (uint32_t)(end - b);
  const uint64_t base = b / 3;
  const uint32_t nt = event_tracks(n_tracks[e], ne);
  for (uint32_t t = threadIdx.x; t < nt; t += 128) {
    const uint64_t slot = base + t;
    const int n = nhits[slot];
    if (n < 3 || n > kLayers) continue;
    const uint32_t i0 = hit_idx[26ull * slot], i1 = hit_idx[26ull * slot + n - 1];
    if (i0 >= ne || i1 >= ne) continue;
    const uint32_t lf = key[b + i0] >> 22, ll = key[b + i1] >> 22;
    float f[kNF];
    track_features(s.chi2[slot], s.ndof[slot], n, lf < 26u ? lf : 25u, ll < 26u ? ll : 25u,
                   s.tx[slot], s.ty[slot], f);
#pragma unroll
    for (int k = 0; k < kNF; ++k) feat[8 * slot + k] = f[k];
  }
}

// ---------------------------------------------------------------------------
// mean and standard deviation of n feature rows (double partial sums per
// workgroup, then a fixed-order final sum)

constexpr int kStatThreads = 256;

__global__ __launch_bounds__(kStatThreads) void k_stat_partial(const float* __restrict__ f, uint64_t n,
                                                               double* __restrict__ part) {
  __shared__ double acc[kStatThreads][2 * kNF + 1];
  double s[2 * kNF];
  for (int k = 0; k < 2 * kNF; ++k) s[k] = 0.0;
  for (uint64_t i = (uint64_t)blockIdx.x * kStatThreads + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kStatThreads) {
#pragma unroll
    for (int k = 0; k < kNF; ++k) {
      const double v = f[8 * i + k];
      s[k] += v;
      s[kNF + k] += v * v;
    }
  }
  for (int k = 0; k < 2 * kNF; ++k) acc[threadIdx.x][k] = s[k];
  __syncthreads();
  if (threadIdx.x < 2 * kNF) {
    double t = 0.0;
    for (int j = 0; j < kStatThreads; ++j) t += acc[j][threadIdx.x];
    part[(size_t)blockIdx.x * 2 * kNF + threadIdx.x] = t;
  }
}

__global__ void k_stat_final(const double* __restrict__ part, int blocks, uint64_t n,
                             float* __restrict__ mean, float* __restrict__ stdv) {
  const int k = threadIdx.x;
  if (k >= kNF) return;
  double s = 0.0, q = 0.0;
  for (int b = 0; b < blocks; ++b) {
    s += part[(size_t)b * 2 * kNF + k];
    q += part[(size_t)b * 2 * kNF + kNF + k];
  }
  const double m = n ? s / (double)n : 0.0;
  double var = n ? q / (double)n - m * m : 0.0;
  if (var < 1e-12) var = 1e-12;
  mean[k] = (float)m;
  stdv[k] = (float)sqrt(var);
}

// ---------------------------------------------------------------------------
// FP32 training: gradient of the mean loss over n samples

constexpr int kTS = 128;        // samples per workgroup
constexpr int kTThreads = 256;  // lanes per workgroup (the first kTS own a sample)
constexpr int kNPart = kNP + 1; // gradient + loss

__global__ __launch_bounds__(kTThreads) void k_mlp_grad(const float* __restrict__ P,
                                                        const float* __restrict__ mean,
                                                        const float* __restrict__ stdv,
                                                        const float* __restrict__ feat,
                                                        const float* __restrict__ label,
                                                        const uint32_t* __restrict__ idx, uint32_t n,
                                                        float* __restrict__ part) {
  __shared__ float w[kNP];
  __shared__ float sx[kTS][kNF + 1];
  __shared__ float sh1[kTS][kNH + 1], sh2[kTS][kNH + 1], sdh1[kTS][kNH + 1];
  __shared__ float sdz[kTS], sloss[kTS];
  for (int p = threadIdx.x; p < kNP; p += kTThreads) w[p] = P[p];
  __syncthreads();
  const uint32_t s = threadIdx.x;
  if (s < (uint32_t)kTS) {
    // the lane's own activation rows live in LDS (keeps register pressure low)
    const uint32_t i = blockIdx.x * kTS + s;
    float dz = 0.0f, loss = 0.0f;
    if (i < n) {
      const uint32_t j = idx ? idx[i] : i;
      const float y = label[j];
      float x[kNF];
#pragma unroll
      for (int k = 0; k < kNF; ++k) {
        x[k] = (feat[8ull * j + k] - mean[k]) / stdv[k];
        sx[s][k] = x[k];
      }
      for (int u = 0; u < kNH; ++u) {
        float a = w[kOB1 + u];
#pragma unroll
        for (int k = 0; k < kNF; ++k) a += w[kOW1 + kNF * u + k] * x[k];
        sh1[s][u] = a > 0.0f ? a : 0.0f;
      }
      float z = w[kOB3];
      for (int u = 0; u < kNH; ++u) {
        float a = w[kOB2 + u];
        for (int k = 0; k < kNH; ++k) a += w[kOW2 + kNH * u + k] * sh1[s][k];
        const float h = a > 0.0f ? a : 0.0f;
        sh2[s][u] = h;
        z += w[kOW3 + u] * h;
      }
      loss = (z > 0.0f ? z : 0.0f) - z * y + log1pf(expf(-fabsf(z)));
      dz = (1.0f / (1.0f + expf(-z)) - y) / (float)n;
      for (int k = 0; k < kNH; ++k) {
        float a = 0.0f;
        for (int u = 0; u < kNH; ++u) a += w[kOW2 + kNH * u + k] * (sh2[s][u] > 0.0f ? dz * w[kOW3 + u] : 0.0f);
        sdh1[s][k] = sh1[s][k] > 0.0f ? a : 0.0f;
      }
    } else {
      for (int k = 0; k < kNF; ++k) sx[s][k] = 0.0f;
      for (int u = 0; u < kNH; ++u) { sh1[s][u] = 0.0f; sh2[s][u] = 0.0f; sdh1[s][u] = 0.0f; }
    }
    sdz[s] = dz;
    sloss[s] = loss;
  }
  __syncthreads();
  float* out = part + (size_t)blockIdx.x * kNPart;
  for (int p = threadIdx.x; p < kNPart; p += kTThreads) {
    float acc = 0.0f;
    if (p < kOB1) {
      const int u = p / kNF, k = p % kNF;
      for (int q = 0; q < kTS; ++q) acc += sdh1[q][u] * sx[q][k];
    } else if (p < kOW2) {
      const int u = p - kOB1;
      for (int q = 0; q < kTS; ++q) acc += sdh1[q][u];
    } else if (p < kOB2) {
      const int u = (p - kOW2) / kNH, k = (p - kOW2) % kNH;
      const float w3u = w[kOW3 + u];
      for (int q = 0; q < kTS; ++q) acc += (sh2[q][u] > 0.0f ? sdz[q] * w3u : 0.0f) * sh1[q][k];
    } else if (p < kOW3) {
      const int u = p - kOB2;
      const float w3u = w[kOW3 + u];
      for (int q = 0; q < kTS; ++q) acc += sh2[q][u] > 0.0f ? sdz[q] * w3u : 0.0f;
    } else if (p < kOB3) {
      const int u = p - kOW3;
      for (int q = 0; q < kTS; ++q) acc += sdz[q] * sh2[q][u];
    } else if (p == kOB3) {
      for (int q = 0; q < kTS; ++q) acc += sdz[q];
    } else {
      for (int q = 0; q < kTS; ++q) acc += sloss[q];
    }
    out[p] = acc;
  }
}

__global__ void k_mlp_grad_sum(const float* __restrict__ part, int blocks, uint32_t n,
                               float* __restrict__ grad, float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNPart) return;
  float acc = 0.0f;
  for (int b = 0; b < blocks; ++b) acc += part[(size_t)b * kNPart + p];
  if (p < kNP) grad[p] = acc;
  else if (loss) *loss = n ? acc / (float)n : 0.0f;
}

__global__ void k_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNP) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.0f - b1) * gp;
  const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  P[p] = P[p] - lr * (mp * c1) / (sqrtf(vp * c2) + eps);
}

// ---------------------------------------------------------------------------
// BF16 MFMA inference of 64 samples per wave

struct MlpLds {       // per workgroup
  __bf16 w1[kNH][kNF];
  __bf16 w2[kNH][kNH];
  __bf16 w3[kNH];
  float b1[kNH], b2[kNH], b3, mean[kNF], sd[kNF];
};

__device__ __forceinline__ void mlp_load(MlpLds& L, const float* __restrict__ P,
                                         const float* __restrict__ mean,
                                         const float* __restrict__ stdv, int nthreads) {
  for (int p = threadIdx.x; p < kNH * kNF; p += nthreads) L.w1[p / kNF][p % kNF] = (__bf16)P[kOW1 + p];
  for (int p = threadIdx.x; p < kNH * kNH; p += nthreads) L.w2[p / kNH][p % kNH] = (__bf16)P[kOW2 + p];
  for (int p = threadIdx.x; p < kNH; p += nthreads) {
    L.w3[p] = (__bf16)P[kOW3 + p];
    L.b1[p] = P[kOB1 + p];
    L.b2[p] = P[kOB2 + p];
  }
  if (threadIdx.x == 0) L.b3 = P[kOB3];
  for (int k = threadIdx.x; k < kNF; k += nthreads) { L.mean[k] = mean[k]; L.sd[k] = stdv[k]; }
}

// Logit of the calling lane's sample (raw features f); every lane of the wave
// must call it (invalid lanes pass any finite values).  The wave's 64
// samples are the columns of the activation matrices and stay in registers.
// v_mfma_f32_16x16x32_bf16 computes D = A B where lane l = 16 g + r supplies
// A[r][8g+i] and B[8g+i][r] (i < 8) and receives D[4g+i][r] (i < 4); rows of
// A and D are units, columns of B and D samples.
//   Layer 1, sample block m (samples 16m..16m+15), unit block n: B[8g+i][r]
//   = feature i of the lane's own sample 16g+r, A[r][8g+i] = W1[16n+r][i] for
//   g == m and 0 otherwise, so only block m's K-slots contribute:
//   D[4g+i][r] = unit 16n+4g+i of sample 16m+r.
//   After both unit blocks, lane (g, r) holds for every block m the units
//   4g..4g+3 and 16+4g..16+4g+3 of sample 16m+r: the 8 K-slots it supplies
//   to layer 2 when the columns of W2 are taken in that same order.
//   Layer 3: w3 times the lane's 8 units, summed over the four lanes of the
//   sample's column (r, 16+r, 32+r, 48+r) by two exchanges, after which
//   lane 16g+r holds the logit of its own sample (block m = g).
__device__ __forceinline__ float mlp_wave_logit(const MlpLds& L, const float* f) {
  // compiler barrier: the weight loads below stay here instead of being
  // hoisted out of the caller's loop, where they would hold registers
  // through the whole fit
  __asm__ volatile("" ::: "memory");
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  bf16x8 xv;
#pragma unroll
  for (int k = 0; k < kNF; ++k) xv[k] = (__bf16)((f[k] - L.mean[k]) / L.sd[k]);
  const bf16x8 zero8 = {};
  const bf16x8 w1a = *reinterpret_cast<const bf16x8*>(&L.w1[r][0]);
  const bf16x8 w1b = *reinterpret_cast<const bf16x8*>(&L.w1[16 + r][0]);
  bf16x8 w2a, w2b;  // rows r and 16 + r of W2, columns 4g..4g+3 and 16+4g..16+4g+3
  float b1v[8], b2v[8], w3v[8];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    w2a[i] = L.w2[r][4 * g + i];
    w2a[4 + i] = L.w2[r][16 + 4 * g + i];
    w2b[i] = L.w2[16 + r][4 * g + i];
    w2b[4 + i] = L.w2[16 + r][16 + 4 * g + i];
    b1v[i] = L.b1[4 * g + i];
    b1v[4 + i] = L.b1[16 + 4 * g + i];
    b2v[i] = L.b2[4 * g + i];
    b2v[4 + i] = L.b2[16 + 4 * g + i];
    w3v[i] = (float)L.w3[4 * g + i];
    w3v[4 + i] = (float)L.w3[16 + 4 * g + i];
  }
  const floatx4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f};
  bf16x8 h1[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const floatx4 d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(g == m ? w1a : zero8, xv, acc0, 0, 0, 0);
    const floatx4 d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(g == m ? w1b : zero8, xv, acc0, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float u0 = d0[i] + b1v[i], u1 = d1[i] + b1v[4 + i];
      h1[m][i] = (__bf16)(u0 > 0.0f ? u0 : 0.0f);
      h1[m][4 + i] = (__bf16)(u1 > 0.0f ? u1 : 0.0f);
    }
  }
  float p[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const floatx4 d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2a, h1[m], acc0, 0, 0, 0);
    const floatx4 d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2b, h1[m], acc0, 0, 0, 0);
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float u0 = d0[i] + b2v[i];
      s = s + w3v[i] * (float)(__bf16)(u0 > 0.0f ? u0 : 0.0f);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float u1 = d1[i] + b2v[4 + i];
      s = s + w3v[4 + i] * (float)(__bf16)(u1 > 0.0f ? u1 : 0.0f);
    }
    p[m] = s;
  }
  // lanes 32 apart: keep the two blocks whose bit 1 is g's, add the partner's
  const bool hi = (g >> 1) != 0;
  float k0 = hi ? p[2] : p[0], k1 = hi ? p[3] : p[1];
  const float s0 = hi ? p[0] : p[2], s1 = hi ? p[1] : p[3];
  k0 = k0 + __shfl_xor(s0, 32, 64);
  k1 = k1 + __shfl_xor(s1, 32, 64);
  // lanes 16 apart: keep the block whose bit 0 is g's
  const bool lo = (g & 1) != 0;
  float z = lo ? k1 : k0;
  z = z + __shfl_xor(lo ? k0 : k1, 16, 64);
  return z + L.b3;
}

constexpr int kInferThreads = 256;

__global__ __launch_bounds__(kInferThreads) void k_mlp_infer(const float* __restrict__ P,
                                                             const float* __restrict__ mean,
                                                             const float* __restrict__ stdv,
                                                             const float* __restrict__ feat,
                                                             uint32_t n, float* __restrict__ logit) {
  __shared__ MlpLds L;
  mlp_load(L, P, mean, stdv, kInferThreads);
  __syncthreads();
  for (uint64_t b0 = (uint64_t)blockIdx.x * kInferThreads; b0 < n; b0 += (uint64_t)gridDim.x * kInferThreads) {
    const uint64_t i = b0 + threadIdx.x;
    float f[kNF];
#pragma unroll
    for (int k = 0; k < kNF; ++k) f[k] = i < n ? feat[8 * i + k] : L.mean[k];
    const float z = mlp_wave_logit(L, f);
    if (i < n) logit[i] = z;
  }
}

// ---------------------------------------------------------------------------

size_t mlp_workspace_bytes(uint32_t n) {
  const size_t blocks = (n + kTS - 1) / kTS;
  const size_t a = blocks * kNPart * sizeof(float);
  const size_t b = 1024 * 2 * kNF * sizeof(double);
  return (a > b ? a : b) + 256;
}

hipError_t launch_features(const velo_hits* h, const velo_tracks* t, const velo_states* s,
                           const uint64_t* offsets, uint32_t n_events, uint64_t n_pixels,
                           float* feat, hipStream_t st) {
  hipLaunchKernelGGL(k_features, dim3(n_events), dim3(128), 0, st, h->key, offsets, n_pixels,
                     t->n_tracks, t->nhits, t->hit_idx, *s, feat);
  return hipGetLastError();
}

hipError_t launch_feature_stats(const float* feat, uint64_t n, float* mean, float* stdv, void* ws,
                                hipStream_t st) {
  const int blocks = (int)((n + kStatThreads - 1) / kStatThreads < 1024 ? (n + kStatThreads - 1) / kStatThreads : 1024);
  const int nb = blocks > 0 ? blocks : 1;
  hipLaunchKernelGGL(k_stat_partial, dim3(nb), dim3(kStatThreads), 0, st, feat, n, (double*)ws);
  hipLaunchKernelGGL(k_stat_final, dim3(1), dim3(64), 0, st, (const double*)ws, nb, n, mean, stdv);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* P, const float* mean, const float* stdv, const float* feat,
                           const float* label, const uint32_t* idx, uint32_t n, float* grad,
                           float* loss, void* ws, hipStream_t st) {
  const int blocks = (int)((n + kTS - 1) / kTS);
  const int nb = blocks > 0 ? blocks : 1;
  hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(kTThreads), 0, st, P, mean, stdv, feat, label, idx, n,
                     (float*)ws);
  hipLaunchKernelGGL(k_mlp_grad_sum, dim3((kNPart + 255) / 256), dim3(256), 0, st, (const float*)ws, nb,
                     n, grad, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* P, float* m, float* v, const float* g, uint32_t step, float lr,
                       hipStream_t st) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - pow(b1, (double)step)));
  const float c2 = (float)(1.0 / (1.0 - pow(b2, (double)step)));
  hipLaunchKernelGGL(k_adam, dim3((kNP + 255) / 256), dim3(256), 0, st, P, m, v, g, lr, (float)b1,
                     (float)b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_infer(const float* P, const float* mean, const float* stdv, const float* feat,
                            uint32_t n, float* logit, hipStream_t st) {
  uint32_t blocks = (n + kInferThreads - 1) / kInferThreads;
  if (blocks > 2048) blocks = 2048;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_mlp_infer, dim3(blocks), dim3(kInferThreads), 0, st, P, mean, stdv, feat, n, logit);
  return hipGetLastError();
}

}  // namespace velo
