// cluster.hip -- decoding and clustering of raw VELO pixel words
// (paper Sec. 2.3.1, first paragraph: connected-component labelling of the
// fired pixels of each plane, processed independently per small region;
// here a region is one (event, plane) segment of the raw buffer).
//
// Pipeline (all on one stream, no host round trip):
//   k_clear     status[e] = 0, work-list counter = 0
//   k_validate  one thread per word: bad word / hole / plane-order flags and
//               the plane boundaries (layer_start) of every event
//   k_small     one 64-lane workgroup per (event, plane) segment of at most
//               kSmallCap words: LDS sort by address, 8-neighbour union-find
//               (hook to the smaller index), integer charge sums, ordered
//               emission by wave ballot/prefix; larger segments are appended
//               to a work list
//   k_mid       persistent 256-lane workgroups over the work list: the same
//               algorithm in LDS up to kMidCap words, else in the caller's
//               workspace at the segment's own word positions
//   k_finalize  one thread per event: per-event status, hit counts, zeroed
//               outputs for flagged events
#include "velo_device.hpp"

namespace velo {

constexpr uint32_t kSmallCap = 512;   // words per segment handled by one wave
constexpr uint32_t kMidCap = 2048;    // words per segment handled in LDS by 256 lanes
constexpr int kMidThreads = 256;
constexpr uint32_t kDupBit = 0x80000000u;

struct HitsOut {
  float* x;
  float* y;
  uint32_t* key;
  uint32_t* aux;
};

// Loads of shared scratch (LDS or global workspace) that other lanes of the
// workgroup update with atomics.
__device__ __forceinline__ uint32_t ld(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Ascending bitonic sort network (flip form: every comparator puts the
// smaller value at the lower index), over the virtual power-of-two extension
// of a[0..n); entries >= n act as +infinity and are never touched.
template <int NT>
__device__ void sort_u32(uint32_t* a, uint32_t n) {
  uint32_t P = 1;
  while (P < n) P <<= 1;
  const uint32_t half = P >> 1;
  for (uint32_t k = 2; k <= P; k <<= 1) {
    const uint32_t lh = __builtin_ctz(k >> 1);
    for (uint32_t t = threadIdx.x; t < half; t += NT) {
      uint32_t i = ((t >> lh) << (lh + 1)) | (t & ((k >> 1) - 1));
      uint32_t j = i ^ (k - 1);
      if (j < n) {
        uint32_t x = ld(a + i), y = ld(a + j);
        if (x > y) { a[i] = y; a[j] = x; }
      }
    }
    __syncthreads();
    for (uint32_t d = k >> 2; d > 0; d >>= 1) {
      const uint32_t ld2 = __builtin_ctz(d);
      for (uint32_t t = threadIdx.x; t < half; t += NT) {
        uint32_t i = ((t >> ld2) << (ld2 + 1)) | (t & (d - 1));
        uint32_t j = i + d;
        if (j < n) {
          uint32_t x = ld(a + i), y = ld(a + j);
          if (x > y) { a[i] = y; a[j] = x; }
        }
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ uint32_t uf_find(uint32_t* par, uint32_t x) {
  uint32_t p = ld(par + x);
  while (p != x) {
    x = p;
    p = ld(par + x);
  }
  return x;
}

// Join the trees of a and b, hooking the larger root under the smaller one,
// so that every tree's root is its smallest index.
__device__ __forceinline__ void uf_unite(uint32_t* par, uint32_t a, uint32_t b) {
  while (true) {
    a = uf_find(par, a);
    b = uf_find(par, b);
    if (a == b) return;
    if (a > b) { uint32_t t = a; a = b; b = t; }
    uint32_t old = atomicMin(par + b, a);
    if (old == b) return;
    b = old;
  }
}

// first index j in [lo, hi) with (srt[j] >> 4) >= addr, else hi
__device__ __forceinline__ uint32_t lower_bound_addr(const uint32_t* srt, uint32_t lo, uint32_t hi,
                                                     uint32_t addr) {
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if ((ld(srt + mid) >> 4) < addr) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Cluster the n words of one (event, plane) segment with NT lanes.
// Scratch arrays (n entries each): srt, par, qs, ns, scs, srs; tmp holds
// NT/64+1 words and flag one word, both in LDS.  Writes hits at
// out_base + rank (rank = position among the segment's clusters by key).
// Returns the number of clusters, or kDupBit if two words share an address.
template <int NT>
__device__ uint32_t cluster_segment(const uint32_t* __restrict__ w, uint32_t n, uint32_t layer,
                                    uint32_t* srt, uint32_t* par, uint32_t* qs, uint32_t* ns,
                                    uint32_t* scs, uint32_t* srs, uint32_t* tmp, uint32_t* flag,
                                    HitsOut o, uint64_t out_base) {
  const uint32_t tid = threadIdx.x;
  // sort value: 22-bit in-plane address (row << 11 | col) then charge
  for (uint32_t i = tid; i < n; i += NT) {
    uint32_t v = w[i];
    srt[i] = ((w_row(v) << 11 | w_col(v)) << 4) | w_charge(v);
  }
  if (tid == 0) *flag = 0;
  __syncthreads();
  sort_u32<NT>(srt, n);
  bool dup = false;
  for (uint32_t i = tid; i < n; i += NT) {
    uint32_t a = ld(srt + i) >> 4;
    if (i > 0 && (ld(srt + i - 1) >> 4) == a) dup = true;
    par[i] = i;
    qs[i] = 0;
    ns[i] = 0;
    scs[i] = 0;
    srs[i] = 0;
  }
  if (dup) atomicOr(flag, 1u);
  __syncthreads();
  if (ld(flag)) return kDupBit;

  // edges to the forward neighbours (r, c+1), (r+1, c-1..c+1)
  for (uint32_t i = tid; i < n; i += NT) {
    uint32_t a = ld(srt + i) >> 4;
    uint32_t r = a >> 11, c = a & 0x7FFu;
    if (i + 1 < n && (ld(srt + i + 1) >> 4) == a + 1) uf_unite(par, i, i + 1);
    if (r + 1 < (uint32_t)kPix) {
      uint32_t lo = ((r + 1) << 11) | (c ? c - 1 : 0u);
      uint32_t hi = ((r + 1) << 11) | (c + 1 < (uint32_t)kPix ? c + 1 : c);
      for (uint32_t j = lower_bound_addr(srt, i + 1, n, lo); j < n && (ld(srt + j) >> 4) <= hi; ++j)
        uf_unite(par, i, j);
    }
  }
  __syncthreads();
  // flatten and accumulate integer sums at the roots
  for (uint32_t i = tid; i < n; i += NT) {
    uint32_t r = uf_find(par, i);
    uint32_t v = ld(srt + i);
    uint32_t q = v & 15u, a = v >> 4;
    atomicAdd(qs + r, q);
    atomicAdd(ns + r, 1u);
    atomicAdd(scs + r, q * (a & 0x7FFu));
    atomicAdd(srs + r, q * (a >> 11));
    if (r != i) par[i] = r;
  }
  __syncthreads();
  // roots in index (= address) order, compacted by a workgroup prefix count
  uint32_t carry = 0;
  for (uint32_t b = 0; b < n; b += NT) {
    uint32_t i = b + tid;
    bool root = i < n && ld(par + i) == i;
    uint32_t tot;
    uint32_t rank = block_scan<NT>(root ? 1u : 0u, tmp, &tot);
    if (root) {
      uint64_t slot = out_base + carry + rank;
      uint32_t Q = ld(qs + i), N = ld(ns + i), SC = ld(scs + i), SR = ld(srs + i);
      o.x[slot] = ((float)SC / (float)Q - 767.5f) * 0.055f;
      o.y[slot] = ((float)SR / (float)Q - 767.5f) * 0.055f;
      o.key[slot] = (layer << 22) | (ld(srt + i) >> 4);
      o.aux[slot] = ((N < 65535u ? N : 65535u) << 16) | (Q < 65535u ? Q : 65535u);
    }
    carry += tot;
  }
  return carry;
}

// ---------------------------------------------------------------------------

__global__ void k_clear(uint32_t* __restrict__ status, uint32_t n_events, uint32_t* __restrict__ counter) {
  uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n_events) status[e] = 0;
  if (e == 0) *counter = 0;
}

// largest e in [lo, hi] with offsets[e] <= i (offsets[lo] <= i assumed)
__device__ __forceinline__ uint32_t event_of(const uint64_t* __restrict__ offsets, uint32_t lo,
                                             uint32_t hi, uint64_t i) {
  while (lo < hi) {
    uint32_t mid = lo + ((hi - lo + 1) >> 1);
    if (offsets[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

constexpr uint32_t kValWords = 16;  // words per thread of k_validate

__global__ __launch_bounds__(256) void k_validate(const uint32_t* __restrict__ px,
                                                  const uint64_t* __restrict__ offsets,
                                                  uint32_t n_events, uint64_t n_pixels,
                                                  uint32_t* __restrict__ status,
                                                  uint32_t* __restrict__ layer_start) {
  __shared__ uint32_t ev_range[2];
  const uint64_t span = 256ull * kValWords;
  const uint64_t i0 = (uint64_t)blockIdx.x * span;
  if (threadIdx.x < 2) {
    const uint64_t last = i0 + span - 1 < n_pixels ? i0 + span - 1 : n_pixels - 1;
    const uint64_t probe = threadIdx.x == 0 ? i0 : last;
    uint32_t e = 0;
    if (offsets[0] <= probe) e = event_of(offsets, 0, n_events - 1, probe);
    ev_range[threadIdx.x] = e;
  }
  __syncthreads();
  uint32_t lo = ev_range[0], hi = ev_range[1];
  if (hi < lo) hi = lo;  // offsets not monotone: the event is flagged by k_finalize
#pragma unroll 4
  for (uint32_t k = 0; k < kValWords; ++k) {
    const uint64_t i = i0 + threadIdx.x + 256ull * k;
    if (i >= n_pixels || offsets[0] > i) continue;
    const uint32_t e = event_of(offsets, lo, hi, i);
    const uint64_t b = offsets[e], end = offsets[e + 1];
    if (!(b <= i && i < end) || end > n_pixels) continue;
    const uint32_t w = px[i];
    const uint32_t p = (uint32_t)(i - b), n = (uint32_t)(end - b);
    const uint32_t col = w_col(w), row = w_row(w), lay = w_layer(w), q = w_charge(w);
    uint32_t flags = 0;
    const bool valid = !(w >> 31) && lay < (uint32_t)kLayers && row < (uint32_t)kPix &&
                       col < (uint32_t)kPix && q >= 1u;
    if (!valid) flags |= VELO_EV_BAD_WORD;
    else if (in_hole(col, row)) flags |= VELO_EV_HOLE;
    const uint32_t lc = lay < 26u ? lay : 26u;
    int lp = -1;
    if (p > 0) {
      const uint32_t wp = w_layer(px[i - 1]);
      if (lay < wp) flags |= VELO_EV_LAYER_ORDER;
      lp = (int)(wp < 26u ? wp : 26u);
    }
    if (flags) atomicOr(status + e, flags);
    uint32_t* ls = layer_start + 27ull * e;
    for (int l = lp + 1; l <= (int)lc; ++l) ls[l] = p;
    if (p == n - 1)
      for (int l = (int)lc + 1; l <= 26; ++l) ls[l] = n;
  }
}

// offsets of event e are usable (monotone and inside the buffer)
__device__ __forceinline__ bool event_ok(const uint64_t* __restrict__ offsets, uint32_t e,
                                         uint64_t n_pixels) {
  uint64_t a = offsets[e], b = offsets[e + 1];
  return a <= b && b <= n_pixels;
}

struct SmallArgs {
  const uint32_t* px;
  const uint64_t* offsets;
  uint64_t n_pixels;
  const uint32_t* status;
  const uint32_t* layer_start;
  uint32_t* layer_nhits;
  HitsOut o;
  uint32_t* mid_count;
  uint32_t* mid_list;
};

struct SmallLds {
  uint32_t srt[kSmallCap], par[kSmallCap], qs[kSmallCap], ns[kSmallCap], scs[kSmallCap],
      srs[kSmallCap];
  uint32_t tmp[2], flag;
};

// One (event, plane) segment with one wave; segments above kSmallCap words
// are appended to the large-segment list.
__device__ __forceinline__ void small_segment(const SmallArgs& a, SmallLds& S, uint32_t seg) {
  const uint32_t e = seg / kLayers, l = seg % kLayers;
  if (a.status[e] != 0 || !event_ok(a.offsets, e, a.n_pixels)) return;
  const uint64_t b = a.offsets[e];
  const uint64_t ne = a.offsets[e + 1] - b;
  if (ne == 0) return;  // empty event: k_finalize writes its outputs
  const uint32_t s0 = a.layer_start[27ull * e + l], s1 = a.layer_start[27ull * e + l + 1];
  if (s0 > s1 || s1 > ne) return;  // cannot happen for a validated event
  const uint32_t n = s1 - s0;
  if (n > kSmallCap) {
    if (threadIdx.x == 0) a.mid_list[atomicAdd(a.mid_count, 1u)] = seg;
    return;
  }
  uint32_t cnt = 0;
  if (n > 0)
    cnt = cluster_segment<64>(a.px + b + s0, n, l, S.srt, S.par, S.qs, S.ns, S.scs, S.srs, S.tmp,
                              &S.flag, a.o, b + s0);
  if (threadIdx.x == 0) a.layer_nhits[seg] = cnt;
}

// plain form: one workgroup per segment
__global__ __launch_bounds__(64) void k_small(SmallArgs a) {
  __shared__ SmallLds S;
  small_segment(a, S, blockIdx.x);
}

// Pop the next work item of a persistent workgroup from a device counter.
__device__ __forceinline__ uint32_t pop_item(uint32_t* counter, uint32_t* slot) {
  if (threadIdx.x == 0) *slot = atomicAdd(counter, 1u);
  __syncthreads();
  const uint32_t it = *slot;
  __syncthreads();
  return it;
}

// batched form: persistent workgroups steal segments in descending-size order
__global__ __launch_bounds__(64) void k_small_ws(SmallArgs a, const uint32_t* __restrict__ order,
                                                 uint32_t total, uint32_t* __restrict__ counter) {
  __shared__ SmallLds S;
  __shared__ uint32_t item;
  for (uint32_t it = pop_item(counter, &item); it < total; it = pop_item(counter, &item)) {
    small_segment(a, S, order[it]);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kMidThreads) void k_mid(const uint32_t* __restrict__ px,
                                                     const uint64_t* __restrict__ offsets,
                                                     const uint32_t* __restrict__ layer_start,
                                                     uint32_t* __restrict__ layer_nhits, HitsOut o,
                                                     const uint32_t* __restrict__ mid_count,
                                                     const uint32_t* __restrict__ mid_list,
                                                     uint32_t* __restrict__ ws, uint64_t n_pixels,
                                                     uint32_t* __restrict__ steal) {
  __shared__ uint32_t srt[kMidCap], par[kMidCap], qs[kMidCap], ns[kMidCap], scs[kMidCap],
      srs[kMidCap];
  __shared__ uint32_t tmp[kMidThreads / kWave + 1], flag, item;
  const uint32_t count = *mid_count;
  // static round robin, or work stealing from a counter when `steal` is given
  for (uint32_t it = steal ? pop_item(steal, &item) : blockIdx.x; it < count;
       it = steal ? pop_item(steal, &item) : it + gridDim.x) {
    const uint32_t seg = mid_list[it];
    const uint32_t e = seg / kLayers, l = seg % kLayers;
    const uint64_t b = offsets[e];
    const uint32_t s0 = layer_start[27ull * e + l], s1 = layer_start[27ull * e + l + 1];
    const uint32_t n = s1 - s0;
    uint32_t cnt;
    if (n <= kMidCap) {
      cnt = cluster_segment<kMidThreads>(px + b + s0, n, l, srt, par, qs, ns, scs, srs, tmp, &flag,
                                         o, b + s0);
    } else {
      // scratch in the workspace at the segment's own word positions
      const uint64_t p0 = b + s0;
      cnt = cluster_segment<kMidThreads>(px + p0, n, l, ws + p0, ws + n_pixels + p0,
                                         ws + 2 * n_pixels + p0, ws + 3 * n_pixels + p0,
                                         ws + 4 * n_pixels + p0, ws + 5 * n_pixels + p0, tmp, &flag,
                                         o, p0);
    }
    if (threadIdx.x == 0) layer_nhits[seg] = cnt;
    __syncthreads();
  }
}

__global__ void k_finalize(const uint64_t* __restrict__ offsets, uint32_t n_events,
                           uint64_t n_pixels, uint32_t* __restrict__ status,
                           uint32_t* __restrict__ layer_start, uint32_t* __restrict__ layer_nhits,
                           uint32_t* __restrict__ n_hits) {
  uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_events) return;
  uint32_t st = status[e];
  const bool ok = event_ok(offsets, e, n_pixels);
  if (!ok) st = VELO_EV_BAD_OFFSETS;
  const bool empty = ok && offsets[e + 1] == offsets[e];
  uint32_t total = 0;
  if (st == 0 && !empty) {
    for (int l = 0; l < kLayers; ++l) {
      uint32_t c = layer_nhits[26ull * e + l];
      if (c & kDupBit) st |= VELO_EV_DUPLICATE;
      total += c & ~kDupBit;
    }
  }
  if (st != 0 || empty) {
    for (int l = 0; l < 27; ++l) layer_start[27ull * e + l] = 0;
    for (int l = 0; l < kLayers; ++l) layer_nhits[26ull * e + l] = 0;
    total = 0;
  }
  status[e] = st;
  n_hits[e] = total;
}

// ---------------------------------------------------------------------------

// Launch shape of the clustering stage (the batched form's autotuner picks it).
struct ClusterCfg {
  uint32_t small_grid;        // 0: one workgroup per segment; else persistent work stealing
  uint32_t mid_grid;          // workgroups of the large-segment kernel
  const uint32_t* seg_order;  // descending-size order of the segments (work stealing)
  uint32_t* counters;         // [2] zeroed work-stealing counters (work stealing)
};

size_t cluster_workspace_bytes(uint64_t n_pixels, uint32_t n_events) {
  auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
  return up(4) + up(4ull * kLayers * n_events) + up(6ull * 4 * n_pixels);
}

hipError_t launch_cluster_cfg(const uint32_t* px, const uint64_t* offsets, uint32_t n_events,
                              uint64_t n_pixels, const velo_hits* h, void* ws, hipStream_t s,
                              const ClusterCfg& cfg, bool validated = false) {
  auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
  char* base = (char*)ws;
  uint32_t* mid_count = (uint32_t*)base;
  uint32_t* mid_list = (uint32_t*)(base + up(4));
  uint32_t* scratch = (uint32_t*)(base + up(4) + up(4ull * kLayers * n_events));
  HitsOut o{h->x, h->y, h->key, h->aux};
  if (!validated) {
    hipLaunchKernelGGL(k_clear, dim3((n_events + 255) / 256), dim3(256), 0, s, h->status, n_events,
                       mid_count);
    if (n_pixels > 0)
      hipLaunchKernelGGL(k_validate, dim3((unsigned)((n_pixels + 256 * kValWords - 1) / (256 * kValWords))),
                         dim3(256), 0, s, px, offsets, n_events, n_pixels, h->status, h->layer_start);
  }
  SmallArgs a{px, offsets, n_pixels, h->status, h->layer_start, h->layer_nhits, o, mid_count, mid_list};
  if (cfg.small_grid == 0)
    hipLaunchKernelGGL(k_small, dim3(n_events * kLayers), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(k_small_ws, dim3(cfg.small_grid), dim3(64), 0, s, a, cfg.seg_order,
                       n_events * kLayers, cfg.counters);
  hipLaunchKernelGGL(k_mid, dim3(cfg.mid_grid), dim3(kMidThreads), 0, s, px, offsets, h->layer_start,
                     h->layer_nhits, o, mid_count, mid_list, scratch, n_pixels,
                     cfg.small_grid ? cfg.counters + 1 : (uint32_t*)nullptr);
  hipLaunchKernelGGL(k_finalize, dim3((n_events + 255) / 256), dim3(256), 0, s, offsets, n_events,
                     n_pixels, h->status, h->layer_start, h->layer_nhits, h->n_hits);
  return hipGetLastError();
}

hipError_t launch_cluster(const uint32_t* px, const uint64_t* offsets, uint32_t n_events,
                          uint64_t n_pixels, const velo_hits* h, void* ws, hipStream_t s) {
  return launch_cluster_cfg(px, offsets, n_events, n_pixels, h, ws, s, ClusterCfg{0, 512, nullptr, nullptr});
}

}  // namespace velo
