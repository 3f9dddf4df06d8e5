// cluster.hip -- decoding and clustering of raw VELO pixel words
// (paper Sec. 2.3.1, first paragraph: connected-component labelling of the
// fired pixels of each plane, processed independently per small region;
// here a region is one (event, plane) segment of the raw buffer).
//
// Pipeline (all on one stream, no host round trip):
//   k_offsets   one workgroup: events whose offsets are unusable (decreasing,
//               beyond the buffer, or overlapping an earlier event's words)
//   k_validate  one workgroup per event: bad word / hole / plane-order flags
//               and the plane boundaries (layer_start) of the event; clears
//               the large-segment work list
//   k_small     one 64-lane workgroup per (event, plane) segment of at most
//               kSmallCap words: LDS counting sort by address (row buckets,
//               then rank inside the row), 8-neighbour union-find (roots =
//               smallest addresses), integer charge sums, ordered emission by
//               a prefix count; larger segments are appended to a work list
//   k_mid       persistent 512-lane workgroups over the work list: the same
//               algorithm in LDS up to kMidCap words, else in the caller's
//               workspace at the segment's own word positions
//   k_finalize  one thread per event: per-event status, hit counts, zeroed
//               outputs for flagged events
#include "velo_device.hpp"

namespace velo {

constexpr uint32_t kSmallCap = 448;   // words per segment handled by one wave
constexpr uint32_t kMidCap = 2048;    // words per segment handled in LDS by one workgroup
static_assert(kMidCap >= (uint32_t)kPix, "the workspace row table lives at the segment's own positions");
constexpr int kMidThreads = 512;
static_assert(kSmallCap % 64 == 0 && kMidCap % kMidThreads == 0, "register staging of the words");
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

// Union-find over address-ordered positions: the root of a tree is its
// smallest position, i.e. its pixel of smallest address.
__device__ __forceinline__ uint32_t uf_find(uint32_t* par, uint32_t x) {
  uint32_t p = ld(par + x);
  while (p != x) {
    x = p;
    p = ld(par + x);
  }
  return x;
}

// Join the trees of a and b by hooking the larger root under the smaller.
__device__ __forceinline__ void uf_unite(uint32_t* par, uint32_t a, uint32_t b) {
  while (true) {
    a = uf_find(par, a);
    b = uf_find(par, b);
    if (a == b) return;
    if (a > b) { uint32_t t = a; a = b; b = t; }
    const uint32_t old = atomicMin(par + b, a);
    if (old == b) return;
    b = old;
  }
}

// Per-row table of one segment.  PACKED (LDS tiers, n <= 65535): two rows
// per word, 16 bits each; otherwise one word per row.  add() returns the
// row's previous value.
template <bool PACKED>
struct RowTab {
  uint32_t* w;
  static constexpr uint32_t kWords = PACKED ? kPix / 2 : kPix;
  __device__ __forceinline__ uint32_t add(uint32_t r) const {
    if constexpr (PACKED) {
      const uint32_t sh = (r & 1u) << 4;
      return (atomicAdd(w + (r >> 1), 1u << sh) >> sh) & 0xFFFFu;
    } else {
      return atomicAdd(w + r, 1u);
    }
  }
  __device__ __forceinline__ uint32_t get(uint32_t r) const {
    if constexpr (PACKED) return (ld(w + (r >> 1)) >> ((r & 1u) << 4)) & 0xFFFFu;
    else return ld(w + r);
  }
};

// Scratch of one segment of n words (LDS, or the caller's workspace at the
// segment's own word positions).  PACKED: Q and N share one word (Q in the
// high half; n <= 2048 keeps Q below 2^16).
template <bool PACKED>
struct SegScratch {
  uint32_t* rows;  // RowTab words: row counts, then row starts, then row ends
  uint32_t* srt;   // [n] address << 4 | charge, in address order
  uint32_t* par;   // [n] bucket-order staging, then union-find parents
  uint32_t* qs;    // [n] per root: Q << 16 | N (PACKED) or Q
  uint32_t* ns;    // [n] per root: N (unused when PACKED)
  uint64_t* scr;   // [n] per root: charge-weighted row sum << 32 | column sum (may share
                   // the row table's space: cleared after the row table's last use)
  uint32_t* tmp;   // NT/64 + 1 words of LDS (scans)
  uint32_t* flag;  // one word of LDS
};

// Cluster the n words of one (event, plane) segment with NT lanes; writes the
// hits at out_base + rank (rank = position of the cluster's key among the
// segment's keys).  Returns the number of clusters, or kDupBit if two words
// share an address.
//
// The pixels are sorted by address with two counting passes: by row into
// row buckets, then each pixel's rank among the smaller columns of its row
// bucket.  In address order the same-row neighbour is the next position and
// the next-row neighbours are a short run of the next row's bucket; the
// union-find roots are the smallest positions (= addresses), so the roots in
// position order are the clusters in key order and their ranks are a prefix
// count.
//
// MAXW > 0: n <= MAXW * NT, the words are loaded once into registers (all
// loads in flight together); MAXW == 0: any n, the words are read twice.
template <int NT, bool PACKED, uint32_t MAXW>
__device__ uint32_t cluster_segment(const uint32_t* __restrict__ w, uint32_t n, uint32_t layer,
                                    const SegScratch<PACKED>& S, HitsOut o, uint64_t out_base) {
  constexpr uint32_t WPL = (RowTab<PACKED>::kWords + NT - 1) / NT;  // row words per lane
  // the lanes' words tile the row table in 16-byte pieces: they are cleared,
  // read and written as such (the table is 16-byte aligned)
  constexpr bool VEC = NT * WPL == RowTab<PACKED>::kWords && WPL % 4 == 0;
  const uint32_t tid = threadIdx.x;
  const RowTab<PACKED> rt{S.rows};
  constexpr uint32_t RW = MAXW > 0 ? MAXW : 1;
  uint32_t wr[RW];
  if constexpr (MAXW > 0) {
#pragma unroll
    for (uint32_t k = 0; k < MAXW; ++k) {
      const uint32_t i = tid + k * NT;
      wr[k] = i < n ? w[i] : 0u;
    }
  }
  if constexpr (VEC) {
#pragma unroll
    for (uint32_t k = 0; k < WPL; k += 4)
      *reinterpret_cast<uint4*>(S.rows + tid * WPL + k) = make_uint4(0u, 0u, 0u, 0u);
  } else {
    for (uint32_t i = tid; i < RowTab<PACKED>::kWords; i += NT) S.rows[i] = 0;
  }
  if (tid == 0) *S.flag = 0;
  __syncthreads();
  if constexpr (MAXW > 0) {
#pragma unroll
    for (uint32_t k = 0; k < MAXW; ++k)
      if (tid + k * NT < n) rt.add(w_row(wr[k]));
  } else {
    for (uint32_t i = tid; i < n; i += NT) rt.add(w_row(w[i]));
  }
  __syncthreads();
  {  // row starts: exclusive prefix over rows, WPL consecutive words per lane
    const uint32_t w0 = tid * WPL;
    uint32_t c[WPL], sum = 0;
    if constexpr (VEC) {
#pragma unroll
      for (uint32_t k = 0; k < WPL; k += 4) {
        const uint4 v = *reinterpret_cast<const uint4*>(S.rows + w0 + k);
        c[k] = v.x; c[k + 1] = v.y; c[k + 2] = v.z; c[k + 3] = v.w;
      }
    } else {
#pragma unroll
      for (uint32_t k = 0; k < WPL; ++k) c[k] = w0 + k < RowTab<PACKED>::kWords ? ld(S.rows + w0 + k) : 0u;
    }
#pragma unroll
    for (uint32_t k = 0; k < WPL; ++k) sum += PACKED ? (c[k] & 0xFFFFu) + (c[k] >> 16) : c[k];
    uint32_t tot;
    uint32_t run = block_scan<NT>(sum, S.tmp, &tot);
    uint32_t o[WPL];
#pragma unroll
    for (uint32_t k = 0; k < WPL; ++k) {
      if constexpr (PACKED) {
        const uint32_t lo = run, hi = run + (c[k] & 0xFFFFu);
        o[k] = lo | (hi << 16);
        run = hi + (c[k] >> 16);
      } else {
        o[k] = run;
        run += c[k];
      }
    }
    if constexpr (VEC) {
#pragma unroll
      for (uint32_t k = 0; k < WPL; k += 4)
        *reinterpret_cast<uint4*>(S.rows + w0 + k) = make_uint4(o[k], o[k + 1], o[k + 2], o[k + 3]);
    } else {
#pragma unroll
      for (uint32_t k = 0; k < WPL; ++k)
        if (w0 + k < RowTab<PACKED>::kWords) S.rows[w0 + k] = o[k];
    }
  }
  __syncthreads();
  // row buckets (staged in par); afterwards the table holds the row ends
  auto stage = [&](uint32_t v) {
    S.par[rt.add(w_row(v))] = ((w_row(v) << 11 | w_col(v)) << 4) | w_charge(v);
  };
  if constexpr (MAXW > 0) {
#pragma unroll
    for (uint32_t k = 0; k < MAXW; ++k)
      if (tid + k * NT < n) stage(wr[k]);
  } else {
    for (uint32_t i = tid; i < n; i += NT) stage(w[i]);
  }
  __syncthreads();
  // address order: row start + smaller columns in the row; equal columns are
  // repeated addresses
  bool dup = false;
  for (uint32_t p = tid; p < n; p += NT) {
    const uint32_t v = ld(S.par + p);
    const uint32_t r = (v >> 15) & 0x7FFu, c = (v >> 4) & 0x7FFu;
    const uint32_t b0 = r ? rt.get(r - 1) : 0u, b1 = rt.get(r);
    uint32_t k = b0;
    for (uint32_t q = b0; q < b1; ++q) {
      const uint32_t cq = (ld(S.par + q) >> 4) & 0x7FFu;
      k += cq < c;
      dup |= q != p && cq == c;
    }
    S.srt[k] = v;
  }
  if (dup) atomicOr(S.flag, 1u);
  __syncthreads();
  if (ld(S.flag)) return kDupBit;
  for (uint32_t p = tid; p < n; p += NT) {
    S.par[p] = p;
    S.qs[p] = 0;
    if constexpr (!PACKED) S.ns[p] = 0;
  }
  __syncthreads();
  // edges to (r, c+1) and (r+1, c-1..c+1)
  for (uint32_t p = tid; p < n; p += NT) {
    const uint32_t a = ld(S.srt + p) >> 4;
    const uint32_t r = a >> 11, c = a & 0x7FFu;
    if (p + 1 < n && (ld(S.srt + p + 1) >> 4) == a + 1) uf_unite(S.par, p, p + 1);
    if (r + 1 < (uint32_t)kPix) {
      const uint32_t e1 = rt.get(r + 1);
      for (uint32_t q = rt.get(r); q < e1; ++q) {
        const uint32_t cq = (ld(S.srt + q) >> 4) & 0x7FFu;
        if (cq > c + 1) break;
        if (cq + 1 >= c) uf_unite(S.par, p, q);
      }
    }
  }
  __syncthreads();
  // the row table is dead from here on (the sums may share its space)
  for (uint32_t p = tid; p < n; p += NT) S.scr[p] = 0;
  __syncthreads();
  // integer sums at the roots
  for (uint32_t p = tid; p < n; p += NT) {
    const uint32_t r = uf_find(S.par, p);
    const uint32_t v = ld(S.srt + p);
    const uint32_t q = v & 15u, a = v >> 4;
    if constexpr (PACKED) {
      atomicAdd(S.qs + r, (q << 16) | 1u);
    } else {
      atomicAdd(S.qs + r, q);
      atomicAdd(S.ns + r, 1u);
    }
    atomicAdd((unsigned long long*)(S.scr + r),
              ((unsigned long long)(q * (a >> 11)) << 32) | (unsigned long long)(q * (a & 0x7FFu)));
    if (r != p) S.par[p] = r;
  }
  __syncthreads();
  // roots in position order = clusters in key order
  uint32_t carry = 0;
  for (uint32_t b = 0; b < n; b += NT) {
    const uint32_t p = b + tid;
    const bool root = p < n && ld(S.par + p) == p;
    uint32_t tot;
    const uint32_t rank = block_scan<NT>(root ? 1u : 0u, S.tmp, &tot);
    if (root) {
      const uint64_t slot = out_base + carry + rank;
      const uint32_t qv = ld(S.qs + p);
      const uint32_t Q = PACKED ? qv >> 16 : qv, N = PACKED ? qv & 0xFFFFu : ld(S.ns + p);
      const uint64_t sr = S.scr[p];
      const uint32_t SC = (uint32_t)sr, SR = (uint32_t)(sr >> 32);
      o.x[slot] = ((float)SC / (float)Q - 767.5f) * 0.055f;
      o.y[slot] = ((float)SR / (float)Q - 767.5f) * 0.055f;
      o.key[slot] = (layer << 22) | (ld(S.srt + p) >> 4);
      o.aux[slot] = ((N < 65535u ? N : 65535u) << 16) | (Q < 65535u ? Q : 65535u);
    }
    carry += tot;
  }
  return carry;
}

// ---------------------------------------------------------------------------

constexpr int kValThreads = 256;
constexpr uint32_t kValUnroll = 8;  // words in flight per lane

// Flags of the n words of one event (OR-ed into *flags, in LDS) and its plane
// boundaries ls[0..26]; kValThreads lanes, kValUnroll words in flight per lane.
__device__ __forceinline__ void validate_words(const uint32_t* __restrict__ w, uint32_t n,
                                               uint32_t* __restrict__ ls, uint32_t* flags_out) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  uint32_t flags = 0;
  for (uint32_t i0 = 0; i0 < n; i0 += kValThreads * kValUnroll) {
    uint32_t v[kValUnroll];
#pragma unroll
    for (uint32_t u = 0; u < kValUnroll; ++u) {
      const uint32_t i = i0 + u * kValThreads + threadIdx.x;
      v[u] = i < n ? w[i] : 0u;
    }
#pragma unroll
    for (uint32_t u = 0; u < kValUnroll; ++u) {
      const uint32_t i = i0 + u * kValThreads + threadIdx.x;
      uint32_t prev = __shfl_up(v[u], 1, kWave);  // word i - 1 (lane 0 loads it)
      if (lane == 0 && i > 0 && i < n) prev = w[i - 1];
      if (i >= n) continue;
      const uint32_t x = v[u];
      const uint32_t col = w_col(x), row = w_row(x), lay = w_layer(x), q = w_charge(x);
      const bool valid = !(x >> 31) && lay < (uint32_t)kLayers && row < (uint32_t)kPix &&
                         col < (uint32_t)kPix && q >= 1u;
      if (!valid) flags |= VELO_EV_BAD_WORD;
      else if (in_hole(col, row)) flags |= VELO_EV_HOLE;
      const uint32_t lc = lay < 26u ? lay : 26u;
      int lp = -1;
      if (i > 0) {
        const uint32_t wp = w_layer(prev);
        if (lay < wp) flags |= VELO_EV_LAYER_ORDER;
        lp = (int)(wp < 26u ? wp : 26u);
      }
      for (int l = lp + 1; l <= (int)lc; ++l) ls[l] = i;
      if (i == n - 1)
        for (int l = (int)lc + 1; l <= 26; ++l) ls[l] = n;
    }
  }
  if (flags) atomicOr(flags_out, flags);
}

// Usable offsets: event e owns words [offsets[e], offsets[e+1]) only if
// offsets[e] <= offsets[e+1] <= n_pixels and no earlier offset exceeds
// offsets[e] (offsets[e] is the running maximum of offsets[0..e]); then the
// word ranges of usable events are disjoint.  One 256-lane workgroup walks
// the offsets in tiles of 256 events, carrying the running maximum from tile
// to tile, and writes status[e] = 0 or VELO_EV_BAD_OFFSETS.  (A small
// workgroup finds a place on a GPU busy with other streams' work sooner.)
constexpr int kOffThreads = 256;
__global__ __launch_bounds__(kOffThreads) void k_offsets(const uint64_t* __restrict__ offsets,
                                                         uint32_t n_events, uint64_t n_pixels,
                                                         uint32_t* __restrict__ status) {
  __shared__ uint64_t wmax[2][kOffThreads / kWave];
  const uint32_t lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  uint64_t carry = 0;  // largest offset before the tile
  int buf = 0;
  for (uint32_t t0 = 0; t0 < n_events; t0 += kOffThreads, buf ^= 1) {
    const uint32_t e = t0 + threadIdx.x;
    const bool in = e < n_events;
    const uint64_t a = in ? offsets[e] : 0, b = in ? offsets[e + 1] : 0;
    uint64_t x = a;  // inclusive running maximum over the wave
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const uint64_t y = __shfl_up(x, d, kWave);
      if ((int)lane >= d) x = x > y ? x : y;
    }
    if (lane == kWave - 1) wmax[buf][wid] = x;
    __syncthreads();  // (the other buffer serves the next tile)
    uint64_t before = carry, tile = carry;
    for (uint32_t w = 0; w < kOffThreads / kWave; ++w) {
      const uint64_t v = wmax[buf][w];
      if (w < wid) before = before > v ? before : v;
      tile = tile > v ? tile : v;
    }
    const uint64_t left = __shfl_up(x, 1, kWave);  // lanes before this one
    if (lane > 0) before = before > left ? before : left;
    if (in) status[e] = (a > b || b > n_pixels || a < before) ? VELO_EV_BAD_OFFSETS : 0u;
    carry = tile;
  }
}

// One workgroup per event: flags of every word (status[e], written whole)
// and the plane boundaries of the event (layer_start[27e + l] = index of the
// first word of plane >= l); workgroup 0 also clears the large-segment list.
// Runs after k_offsets: an event it flagged is left as it is, and usable
// events never share a word, so one event's words cannot disturb another.
__global__ __launch_bounds__(kValThreads) void k_validate(const uint32_t* __restrict__ px,
                                                          const uint64_t* __restrict__ offsets,
                                                          uint64_t n_pixels,
                                                          uint32_t* __restrict__ status,
                                                          uint32_t* __restrict__ layer_start,
                                                          uint32_t* __restrict__ mid_count) {
  __shared__ uint32_t s_flags;
  const uint32_t e = blockIdx.x;
  const uint32_t st0 = status[e];
  if (threadIdx.x == 0) {
    s_flags = 0;
    if (e == 0) *mid_count = 0;
  }
  __syncthreads();
  const uint64_t b = offsets[e], end = offsets[e + 1];
  if (st0 == 0 && b <= end && end <= n_pixels)
    validate_words(px + b, (uint32_t)(end - b), layer_start + 27ull * e, &s_flags);
  __syncthreads();
  if (threadIdx.x == 0) status[e] = s_flags | st0;
}

// offsets check, then word validation (both orders of events are free)
inline void launch_validate(const uint32_t* px, const uint64_t* offsets, uint32_t n_events,
                            uint64_t n_pixels, uint32_t* status, uint32_t* layer_start,
                            uint32_t* mid_count, hipStream_t s) {
  hipLaunchKernelGGL(k_offsets, dim3(1), dim3(kOffThreads), 0, s, offsets, n_events, n_pixels, status);
  hipLaunchKernelGGL(k_validate, dim3(n_events), dim3(kValThreads), 0, s, px, offsets, n_pixels,
                     status, layer_start, mid_count);
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
  // the row table and the cluster sums are never live together
  union alignas(16) {
    uint32_t rows[kPix / 2];
    uint64_t scr[kSmallCap];
  } rs;
  uint32_t srt[kSmallCap], par[kSmallCap], qs[kSmallCap];
  uint32_t tmp[2], flag;
  __device__ SegScratch<true> scratch() {
    return SegScratch<true>{rs.rows, srt, par, qs, nullptr, rs.scr, tmp, &flag};
  }
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
    cnt = cluster_segment<64, true, kSmallCap / 64>(a.px + b + s0, n, l, S.scratch(), a.o, b + s0);
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
                                                     uint32_t* __restrict__ ws,
                                                     uint64_t* __restrict__ ws64, uint64_t n_pixels,
                                                     uint32_t* __restrict__ steal) {
  __shared__ uint64_t scr[kMidCap];  // its first kPix / 2 words also hold the row table
  __shared__ uint32_t srt[kMidCap], par[kMidCap], qs[kMidCap];
  uint32_t* rows = reinterpret_cast<uint32_t*>(scr);
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
      const SegScratch<true> S{rows, srt, par, qs, nullptr, scr, tmp, &flag};
      cnt = cluster_segment<kMidThreads, true, kMidCap / kMidThreads>(px + b + s0, n, l, S, o, b + s0);
    } else {
      // scratch in the workspace at the segment's own word positions (n > kPix,
      // so the row table fits there too)
      const uint64_t p0 = b + s0;
      const SegScratch<false> S{ws + p0, ws + n_pixels + p0, ws + 2 * n_pixels + p0,
                                ws + 3 * n_pixels + p0, ws + 4 * n_pixels + p0,
                                ws64 + p0, tmp, &flag};
      cnt = cluster_segment<kMidThreads, false, 0>(px + p0, n, l, S, o, p0);
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
  uint32_t st = status[e];  // VELO_EV_BAD_OFFSETS from k_offsets stands alone
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
  return up(4) + up(4ull * kLayers * n_events) + up(5ull * 4 * n_pixels) + up(8ull * n_pixels);
}

// ev (may be null): events recorded just before and after the per-segment kernel
hipError_t launch_cluster_cfg(const uint32_t* px, const uint64_t* offsets, uint32_t n_events,
                              uint64_t n_pixels, const velo_hits* h, void* ws, hipStream_t s,
                              const ClusterCfg& cfg, bool validated = false,
                              const hipEvent_t* ev = nullptr) {
  auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
  char* base = (char*)ws;
  uint32_t* mid_count = (uint32_t*)base;
  uint32_t* mid_list = (uint32_t*)(base + up(4));
  uint32_t* scratch = (uint32_t*)(base + up(4) + up(4ull * kLayers * n_events));
  uint64_t* scratch64 = (uint64_t*)((char*)scratch + up(5ull * 4 * n_pixels));
  HitsOut o{h->x, h->y, h->key, h->aux};
  if (!validated)
    launch_validate(px, offsets, n_events, n_pixels, h->status, h->layer_start, mid_count, s);
  SmallArgs a{px, offsets, n_pixels, h->status, h->layer_start, h->layer_nhits, o, mid_count, mid_list};
  if (ev && ev[0]) (void)hipEventRecord(ev[0], s);
  if (cfg.small_grid == 0)
    hipLaunchKernelGGL(k_small, dim3(n_events * kLayers), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(k_small_ws, dim3(cfg.small_grid), dim3(64), 0, s, a, cfg.seg_order,
                       n_events * kLayers, cfg.counters);
  if (ev && ev[1]) (void)hipEventRecord(ev[1], s);
  hipLaunchKernelGGL(k_mid, dim3(cfg.mid_grid), dim3(kMidThreads), 0, s, px, offsets, h->layer_start,
                     h->layer_nhits, o, mid_count, mid_list, scratch, scratch64, n_pixels,
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
