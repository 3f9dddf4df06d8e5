// find.hip -- VELO track finding by triplet seeding and forwarding
// (paper Sec. 2.3.1, second paragraph: seeds of three hits on consecutive
// planes, extended to the other planes along straight lines; hits of every
// plane kept in azimuth order for fast look-up).
//
// One workgroup per event walks the planes from z = +750 mm down; the three
// planes in use (l+2, l+1, l) are staged in a ring of LDS tables indexed by
// bucket position: the hits of a plane are read in key order and counting-
// sorted into kNB azimuth buckets of a monotone pseudo-angle of (x, y) while
// they are staged (coordinates, the hit's index in key order, bucket starts;
// used flags).  A window scan thus reads the coordinates of consecutive
// positions directly.  Candidate windows in
// pseudo-angle are derived conservatively from the exact cuts, so they only
// accelerate; every decision uses the exact binary32 cut expressions.
//
// Conflicts are resolved exactly like the sequential greedy rule (ascending
// priority, a candidate wins iff none of its hits / its track is taken):
// rounds in which every live candidate that has the smallest priority at all
// of its hits (and, for extensions, at its track) is accepted reproduce the
// lexicographically-first maximal independent set / matching (Blelloch,
// Fineman and Shun, SPAA 2012).
//
// Tracks are numbered at creation (decreasing first-hit key), so their output
// slots, hit lists and counts are written directly; no atomics decide an
// output position.
//
// Four tiers share one implementation: a 256-lane workgroup per event with
// small LDS tables, persistent 512- and 1024-lane workgroups with middle and
// large LDS tables, and 256 lanes that first write the event's bucket tables
// to the workspace and then read them in place, with per-event scratch in the
// caller's workspace at the event's own hit / track positions.  An event whose tables outgrow its tier is re-run from scratch by
// the next tier.
#include "azimuth.hpp"

namespace velo {

constexpr uint32_t kNone = 0xFFFFFFFFu;

struct FindConst {
  float max_t, sin2, s_seed, s_fwd;
  int max_skip;
  float win_doublet;  // pseudo-angle half width of the seed doublet search
  float rho_seed, rho_fwd;  // upper bounds of sqrt(s_seed), sqrt(s_fwd)
};


// One plane, indexed by bucket position p.  The hit's local index (rank of
// its key in the plane, the order of its event-relative slot) is kr[p].  The
// LDS tiers (64-bit round winners) interleave x and y, so that one 8-byte
// LDS access reads both; the workspace tier reads two arrays.
template <typename IDX, typename SLOT>
struct LayerTab {
  static constexpr uint32_t XS = sizeof(SLOT) == 8 ? 2u : 1u;
  const float* hx;        // x at position p: hx[XS * p]
  const float* hy;        // y at position p: hy[XS * p] (hx + 1 when interleaved)
  const IDX* kr;          // local index of the hit at each position
  uint8_t* used;
  SLOT* best;             // round winner at the hit (see Cands)
  const IDX* bstart;      // [kNB + 1] first position of every bucket
  __device__ __forceinline__ float2 xy(uint32_t p) const {
    if constexpr (XS == 2) return reinterpret_cast<const float2*>(hx)[p];
    else return make_float2(hx[p], hy[p]);
  }
};

template <typename SLOT, typename K>
struct TrackTab {
  K* slot;          // output slot, counted from the event's first track slot
  K* key0;          // first hit: plane << KSH | local index (orders like its key)
  float4* st;       // last hit (x, y) and slope through the last two hits (z: tx, w: ty),
                    // one 16-byte access
  uint8_t* la;      // plane of the last hit
  uint8_t* n;       // hits so far
  uint8_t* skip;    // planes missed in a row
  SLOT* tbest;      // per round: winner at the track
  uint32_t* tmatch; // position of the hit taken at this plane
};

// Candidates.  Extension: track a, hit b; seed: h0 a, h1 b, h2 c (bucket
// positions).  Priority: extension (s, first-hit key of the track, hit key),
// seed (s, key of h1, key of h0, key of h2); s >= 0, so its float bits order
// like s.
//   LDS tiers (local indices < 1024): the priority packed in 64 bits, unique
//   per candidate; a resource's round winner is the atomic minimum of the
//   priorities proposed to it.  Positions packed 10 bits each in `pos`, bit 31
//   marks an accepted seed.
//   Workspace tier (keys of any width): {s, a, b, c}; the winner slot holds a
//   candidate index, updated by a CAS loop with a comparator.
struct Cand {
  float s;
  uint32_t a, b, c;
};
template <bool RING> struct CandSlot { using T = uint32_t; static constexpr uint32_t kFree = 0xFFFFFFFFu; };
template <> struct CandSlot<true> { using T = uint64_t; static constexpr uint64_t kFree = ~0ull; };
constexpr uint32_t kPosBits = 10, kPosMask = (1u << kPosBits) - 1u, kAccepted = 1u << 31;

// seed doublet: h0 | h1 << 16 (bucket positions); its slopes are recomputed
// from the hits, by the same expressions, when the third hit is searched
using Dbl = uint32_t;

struct EventIO {
  const float* X;          // coordinates of the event's hits in bucket order (workspace tier)
  const float* Y;          // (absolute base applied)
  const float* HX;         // coordinates of the event's hits in key order (the LDS tiers
  const float* HY;         // sort them into the ring themselves)
  const uint32_t* lstart;  // [27]
  const uint32_t* lnh;     // [26]
  const uint32_t* order;   // local index at every bucket position (at the hits' slots)
  const uint32_t* bst;     // [26 * (kNB + 1)] bucket starts of every plane
  uint8_t* nhits;          // track outputs (absolute slots)
  uint32_t* hit_idx;
  uint64_t slot_base;
};

// Tables of one event.  RING (LDS tiers): the three planes in use are copied
// into a ring of tables stored back to back (stride capL), addressed
// arithmetically so that the pointers stay in registers.  !RING (workspace
// tier): coordinates and bucket tables are read in place, used / best live
// in scratch at the plane's own event-relative slots.
template <typename IDX, bool RING>
struct FindMem {
  using SLOT = typename CandSlot<RING>::T;
  static constexpr uint32_t KSH = RING ? kPosBits : 22;  // key0 = plane << KSH | local index
  float* hx;         // LDS tiers: x and y interleaved (hy = hx + 1)
  float* hy;
  IDX* kr;
  uint8_t* used;
  SLOT* best;
  IDX* bstart;       // [3 * (kNB + 1)]
  TrackTab<SLOT, IDX> T;
  Cand* cand;        // workspace tier
  uint64_t* cprio;   // LDS tiers
  uint32_t* cpos;
  // seed doublet search (LDS tiers): per middle hit the two bucket ranges of
  // its window on plane l+2 (start | length << 16) and the prefix of their
  // lengths; passing doublets
  uint32_t* w0;
  uint32_t* w1;
  uint32_t* wp;   // [capL + 1]
  uint32_t* own;  // [NT] middle hit holding a lane's first pair (one-pass prefix)
  // forward search (LDS tiers): the same for every active track on the next plane
  uint32_t* tw0;
  uint32_t* tw1;
  uint32_t* twp;  // [capT + 1]
  uint32_t* twown;  // [NT] track holding a lane's first pair (one-pass prefix)
  Dbl* dbl;       // [capD]
  uint32_t* cnt;  // [kNB / 2] bucket counters of the plane being staged, 16 bits each (LDS tiers)
  uint32_t capL, capT, capC, capD;
  __device__ __forceinline__ LayerTab<IDX, SLOT> layer(const EventIO& io, int l) const {
    if constexpr (RING) {
      const uint32_t r = (uint32_t)l % 3u, o = r * capL;
      return LayerTab<IDX, SLOT>{hx + 2 * o, hy + 2 * o, kr + o, used + o, best + o, bstart + r * (kNB + 1)};
    } else {
      const uint32_t o = io.lstart[l];
      return LayerTab<IDX, SLOT>{io.X + o, io.Y + o, io.order + o, used + o, best + o,
                           io.bst + (uint32_t)l * (kNB + 1)};
    }
  }
};

// Bucket ranges covering the pseudo-angle window [c - d, c + d] (wrapping).
struct Ranges { uint32_t b0, b1, b2, b3; };  // [b0,b1] and [b2,b3], b2 > b3 if unused
__device__ __forceinline__ Ranges window(float c, float d, uint32_t nb) {
  Ranges r;
  if (d >= 2.0f) { r.b0 = 0; r.b1 = nb - 1; r.b2 = 1; r.b3 = 0; return r; }
  float lo = c - d, hi = c + d;
  if (lo < 0.0f) {
    r.b0 = 0; r.b1 = bucket_of(hi, nb); r.b2 = bucket_of(lo + 4.0f, nb); r.b3 = nb - 1;
  } else if (hi >= 4.0f) {
    r.b0 = bucket_of(lo, nb); r.b1 = nb - 1; r.b2 = 0; r.b3 = bucket_of(hi - 4.0f, nb);
    // express the second range with b2 <= b3
  } else {
    r.b0 = bucket_of(lo, nb); r.b1 = bucket_of(hi, nb); r.b2 = 1; r.b3 = 0;
  }
  if (r.b2 <= r.b3 && r.b0 <= r.b3 && r.b2 <= r.b1) {  // overlapping: merge into one range
    r.b0 = r.b0 < r.b2 ? r.b0 : r.b2;
    r.b1 = r.b1 > r.b3 ? r.b1 : r.b3;
    r.b2 = 1; r.b3 = 0;
  }
  return r;
}

// pseudo-angle half width for hits within rho of the point (x, y) at radius
// R: the azimuth moves by at most asin(rho / R) <= rho / sqrt(R^2 - rho^2),
// the pseudo-angle by at most kPaSlope times that; hardware reciprocal square
// root (about 1 ulp) under a 0.1 % + 1e-3 margin
__device__ __forceinline__ float point_window(float x, float y, float rho) {
  const float R2 = x * x + y * y, rho2 = rho * rho;
  if (R2 <= 2.25f * rho2) return 4.0f;  // R <= 1.5 rho: whole plane
  return (kPaSlope * rho) * __builtin_amdgcn_rsqf(R2 - rho2) * 1.001f + 1e-3f;
}

template <typename F>
__device__ __forceinline__ void cas_min(uint32_t* slot, uint32_t k, F less) {
  uint32_t cur = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  while (cur == kNone || less(k, cur)) {
    uint32_t prev = atomicCAS(slot, cur, k);
    if (prev == cur) return;
    cur = prev;
  }
}

__device__ __forceinline__ uint32_t lda(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// shared scalars of one event
struct FindScal {
  uint32_t ncf;      // extension candidates found this step (may exceed capC)
  uint32_t ncs;      // seed candidates found this step (may exceed capC)
  uint32_t nd;       // seed doublets found this step (may exceed capD)
  uint32_t item;     // work item popped by a persistent workgroup
  uint32_t flag[2];  // any live candidate left (alternating by round)
  uint32_t n_act;    // active tracks
  uint32_t n_created;
  uint32_t fail;     // 0 ok, 1 escalate, 2 overflow
  uint32_t tmp[2][16];  // scan scratch, two alternating buffers of NT/64 words
  uint32_t lstart[27], lnh[26];  // plane tables of the event
  float z[kLayers];              // plane positions
};

// Staging of plane l into the ring (LDS tiers).  The plane's hits are read
// in key order at the start of step l+1 (issue: coordinates into registers,
// so the global-memory latency overlaps the step) and counting-sorted into
// the slot late in that step, once the seeds no longer read the slot's
// previous plane (l+3):
//   count   every hit takes its rank inside its azimuth bucket from a packed
//           16-bit LDS counter (the order inside a bucket is irrelevant:
//           every use scans whole buckets);
//   starts  a scan of the bucket counts (by the first wave alone) gives the
//           slot's bucket starts; the counters are cleared for the next plane;
//   place   coordinates and local index (the hit's rank in key order) at
//           bucket start + rank.
// A barrier must separate count from starts and starts from place; the
// caller's next barrier publishes the slot.  The used flags and round
// winners of a plane are cleared at the start of its own step.
// Hits per lane staged by the LDS tiers (their plane capacity is at most
// kPrefetch * NT; unused register slots would only raise register pressure).
template <int NT> constexpr int kPrefetch = NT >= 1024 ? 1 : (NT >= 256 ? 2 : 3);
// Candidates per lane in the LDS tiers' conflict rounds (their candidate
// capacity is at most kCandPerLane * NT): each lane keeps its candidates'
// positions and priorities in registers for all rounds.
template <int NT> constexpr int kCandPerLane = NT >= 256 ? 2 : 3;

template <int NT, typename IDX, bool RING>
struct PlanePrefetch {
  static constexpr int PF = RING ? kPrefetch<NT> : 1;  // hits per lane
  float x[PF], y[PF];
  uint32_t br[PF];  // bucket | rank << 16
  uint32_t n = 0;
  __device__ __forceinline__ void issue(const EventIO& io, int l, uint32_t capL) {
    if constexpr (RING) {
      n = io.lnh[l];
      const uint32_t base = io.lstart[l];
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const uint32_t i = threadIdx.x + k * NT;
        if (i < n && i < capL) { x[k] = io.HX[base + i]; y[k] = io.HY[base + i]; }
      }
    }
  }
  template <typename MEM>
  __device__ __forceinline__ void count(const MEM& M) {
    if constexpr (RING) {
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const uint32_t i = threadIdx.x + k * NT;
        if (i < n) {
          const uint32_t b = bucket_of(pangle(x[k], y[k]), kNB), sh = (b & 1u) << 4;
          const uint32_t old = atomicAdd(M.cnt + (b >> 1), 1u << sh);
          br[k] = b | (((old >> sh) & 0xFFFFu) << 16);
        }
      }
    }
  }
  // The first wave alone scans the bucket counts (four buckets per lane, a
  // DPP wave scan), so no extra workgroup barrier is needed: the caller's
  // next barrier publishes the starts.  Each lane reads its two counter words
  // before it clears them (a wave's LDS operations complete in order).
  template <typename MEM>
  __device__ __forceinline__ void starts(const EventIO& io, int l, const MEM& M) {
    static_assert(kNB == 4 * kWave, "four buckets per lane of one wave");
    if constexpr (RING) {
      if (threadIdx.x >= (uint32_t)kWave) return;
      IDX* bsd = const_cast<IDX*>(M.layer(io, l).bstart);
      const uint32_t lane = threadIdx.x;
      const uint32_t w0 = M.cnt[2 * lane], w1 = M.cnt[2 * lane + 1];
      const uint32_t c0 = w0 & 0xFFFFu, c1 = w0 >> 16, c2 = w1 & 0xFFFFu, c3 = w1 >> 16;
      const uint32_t sum = c0 + c1 + c2 + c3;
      const uint32_t incl = wave_incl_scan(sum);
      const uint32_t run = incl - sum;
      bsd[4 * lane] = (IDX)run;
      bsd[4 * lane + 1] = (IDX)(run + c0);
      bsd[4 * lane + 2] = (IDX)(run + c0 + c1);
      bsd[4 * lane + 3] = (IDX)(run + c0 + c1 + c2);
      if (lane == kWave - 1) bsd[kNB] = (IDX)incl;
      M.cnt[2 * lane] = 0;
      M.cnt[2 * lane + 1] = 0;
    }
  }
  template <typename MEM>
  __device__ __forceinline__ void place(const EventIO& io, int l, const MEM& M) {
    if constexpr (RING) {
      const auto t = M.layer(io, l);
      float2* hxy = reinterpret_cast<float2*>(const_cast<float*>(t.hx));
      IDX* kr = const_cast<IDX*>(t.kr);
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const uint32_t i = threadIdx.x + k * NT;
        if (i < n) {
          const uint32_t p = (uint32_t)t.bstart[br[k] & 0xFFFFu] + (br[k] >> 16);
          hxy[p] = make_float2(x[k], y[k]);
          kr[p] = (IDX)i;
        }
      }
    }
  }
};

// Visit positions [p, e) four at a time: the coordinates of a group are
// loaded together (clamped to e - 1), so their LDS latencies overlap.
template <typename LT, typename F>
__device__ __forceinline__ void scan_range(const LT& t, uint32_t p, uint32_t e, F f) {
  for (; p < e; p += 4) {
    float x[4], y[4];
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      const uint32_t q = p + j < e ? p + j : e - 1;
      const float2 v = t.xy(q);
      x[j] = v.x;
      y[j] = v.y;
    }
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j)
      if (p + j < e) f(p + j, x[j], y[j]);
  }
}

template <typename LT, typename F>
__device__ __forceinline__ void scan_window(const LT& t, Ranges r, F f) {
  scan_range(t, t.bstart[r.b0], t.bstart[r.b1 + 1], f);
  if (r.b2 <= r.b3) scan_range(t, t.bstart[r.b2], t.bstart[r.b3 + 1], f);
}

// Conflict rounds of a greedy rule over nc candidates (Blelloch-Fineman-Shun):
// every live candidate proposes itself at each of its resources (CAS-min by
// priority); a candidate that holds all of its resources wins and takes them;
// repeat while a live candidate is left.  Three barriers per round: the
// winners' slots are cleared in the same phase that looks for live
// candidates, and the flag alternates between two words so it is cleared a
// round ahead.  Invariant: every best/tbest slot is kNone before and after,
// and both flags are 0.  Every candidate is live in the first round, so
// propose(true) skips the test; a candidate that holds all of its resources
// is live (a dead one proposed nothing this round, and priorities are
// unique), so acceptance needs no test either.
template <bool RING, typename PROPOSE, typename ACCEPT, typename CLEAR>
__device__ __forceinline__ void greedy_rounds(uint32_t nc, FindScal& sc, PROPOSE propose,
                                              ACCEPT accept, CLEAR clear_and_live) {
  const uint32_t tid = threadIdx.x;
  for (uint32_t round = 0; round <= nc; ++round) {
    propose(round == 0);
    wg_barrier<RING>();
    accept();
    wg_barrier<RING>();
    const bool live = clear_and_live();
    if (live) sc.flag[round & 1] = 1;
    if (tid == 0) sc.flag[(round + 1) & 1] = 0;
    wg_barrier<RING>();
    if (!sc.flag[round & 1]) break;
  }
}

// Returns 0 when done, 1 when the event needs a larger tier, 2 on overflow.
template <int NT, typename IDX, bool RING>
__device__ __forceinline__ uint32_t find_event(const EventIO& io, const FindConst& P,
                                               const FindMem<IDX, RING>& M, FindScal& sc) {
  const uint32_t tid = threadIdx.x;
  const float* zt = sc.z;
  for (int l = 0; l < kLayers; ++l)
    if (io.lnh[l] > M.capL) return 1u;
  if (tid == 0) {
    sc.n_act = 0; sc.n_created = 0; sc.fail = 0; sc.ncf = 0; sc.flag[0] = 0; sc.flag[1] = 0;
  }
  uint32_t sbuf = 0;  // alternating scan buffer
  auto scan = [&](uint32_t v, uint32_t* tot) {
    sbuf ^= 1u;
    return block_scan1<NT, RING>(v, sc.tmp[sbuf], tot);
  };
  PlanePrefetch<NT, IDX, RING> pf;
  if constexpr (RING) {
    for (uint32_t w = tid; w < kNB / 2; w += NT) M.cnt[w] = 0;
    pf.issue(io, kLayers - 1, M.capL);
    wg_barrier<RING>();
    pf.count(M);
    wg_barrier<RING>();
    pf.starts(io, kLayers - 1, M);
    wg_barrier<RING>();
    pf.place(io, kLayers - 1, M);
  }
  wg_barrier<RING>();
  const auto A = M.T;
  using SLOT = typename CandSlot<RING>::T;
  constexpr SLOT kFree = CandSlot<RING>::kFree;
  // a resource proposes / holds candidate k
  // The candidates of the conflict rounds, visited by each lane: in the LDS
  // tiers the lane's own (k = tid + j NT) with their positions and priorities
  // loaded once into registers (cpos_r, cprio_r); in the workspace tier every
  // NT-th candidate, read from the table.
  constexpr int KPL = RING ? kCandPerLane<NT> : 1;
  uint32_t cpos_r[KPL];
  uint64_t cprio_r[KPL];
  auto load_cands = [&](uint32_t nc) {
    if constexpr (RING) {
#pragma unroll
      for (int j = 0; j < KPL; ++j) {
        const uint32_t k = tid + (uint32_t)j * NT;
        if (k < nc) { cpos_r[j] = M.cpos[k]; cprio_r[j] = M.cprio[k]; }
      }
    }
  };
  auto for_cands = [&](uint32_t nc, auto f) {
    if constexpr (RING) {
#pragma unroll
      for (int j = 0; j < KPL; ++j) {
        const uint32_t k = tid + (uint32_t)j * NT;
        if (k < nc) f(k, j);
      }
    } else {
      for (uint32_t k = tid; k < nc; k += NT) f(k, 0);
    }
  };
  // a resource holds candidate k (the lane's j-th)
  auto holds = [&](SLOT* slot, uint32_t k, int j) {
    if constexpr (RING) return __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == cprio_r[j];
    else return lda(slot) == k;
  };
  for (int l = kLayers - 1; l >= 0; --l) {
    if (l > 0) pf.issue(io, l - 1, M.capL);
    const auto T0 = M.layer(io, l);
    const uint32_t base0 = io.lstart[l];
    const float zl = zt[l];
    const uint32_t n_act = sc.n_act;
    // plane l enters its step: no hit used, no round winner
    for (uint32_t i = tid; i < io.lnh[l]; i += NT) { T0.used[i] = 0; T0.best[i] = CandSlot<RING>::kFree; }

    // ---- 1. extend active tracks into plane l ----
    // (the seed counters were last read a step ago, several barriers back)
    if (tid == 0) { sc.ncs = 0; sc.nd = 0; }
    // extrapolation of track t to plane l
    auto extrap = [&](uint32_t t, float& xp, float& yp) {
      const float d = zl - zt[A.la[t]];
      const float4 v = A.st[t];
      xp = v.x + v.z * d;
      yp = v.y + v.w * d;
    };
    auto add_ext = [&](uint32_t t, uint32_t key0, uint32_t h, float s) {
      uint32_t k = atomicAdd(&sc.ncf, 1u);
      if (k < M.capC) {
        if constexpr (RING) {
          M.cprio[k] = ((uint64_t)__float_as_uint(s) << 32) | ((uint64_t)key0 << kPosBits) |
                       (uint64_t)T0.kr[h];
          M.cpos[k] = t | (h << kPosBits);
        } else {
          M.cand[k] = Cand{s, t, h, 0u};
        }
      }
    };
    if (n_act > 0) {
      // Big events (the middle and large tiers) have long windows of uneven length:
      // there the (track, hit) pairs are balanced over the lanes; small events
      // scan each track's window in its own lane.
      if constexpr (RING && NT >= 512) {
        // (a) window of every active track, prefix of the window sizes
        uint32_t carry = 0;
        for (uint32_t b0 = 0; b0 < n_act; b0 += NT) {
          const uint32_t t = b0 + tid;
          uint32_t cnt = 0;
          if (t < n_act) {
            A.tmatch[t] = kNone;
            A.tbest[t] = kFree;
            float xp, yp;
            extrap(t, xp, yp);
            const Ranges r = window(pangle(xp, yp), point_window(xp, yp, P.rho_fwd), kNB);
            const uint32_t s0 = T0.bstart[r.b0], l0 = T0.bstart[r.b1 + 1] - s0;
            uint32_t s1 = 0, l1 = 0;
            if (r.b2 <= r.b3) { s1 = T0.bstart[r.b2]; l1 = T0.bstart[r.b3 + 1] - s1; }
            M.tw0[t] = s0 | (l0 << 16);
            M.tw1[t] = s1 | (l1 << 16);
            cnt = l0 + l1;
          }
          uint32_t tot;
          const uint32_t ex = scan(cnt, &tot);
          if (t < n_act) M.twp[t] = carry + ex;
          if (n_act <= NT && cnt > 0) {
            // one pass: the track whose pairs contain a lane's first pair
            const uint32_t per = (tot + NT - 1) / NT;
            for (uint32_t L = (ex + per - 1) / per; L * per < ex + cnt; ++L) M.twown[L] = t;
          }
          carry += tot;
        }
        if (tid == 0) M.twp[n_act] = carry;
        wg_barrier<RING>();
        // (b) all (track, hit) pairs, split evenly over the lanes in contiguous
        // chunks; four pairs of one track per step, their loads issued together
        const uint32_t total = carry, per = (total + NT - 1) / NT;
        uint32_t j = tid * per;
        const uint32_t jend = j + per < total ? j + per : total;
        if (j < jend) {
          uint32_t lo = 0, hi = n_act - 1;
          if (n_act <= NT) {
            lo = M.twown[tid];
          } else {
            while (lo < hi) {
              const uint32_t mid = (lo + hi + 1) >> 1;
              if (M.twp[mid] <= j) lo = mid; else hi = mid - 1;
            }
          }
          for (uint32_t t = lo; j < jend; ++t) {
            const uint32_t wb = M.twp[t], we = M.twp[t + 1];
            if (we <= j) continue;
            const uint32_t w0 = M.tw0[t], w1 = M.tw1[t], l0 = w0 >> 16, key0 = A.key0[t];
            float xp, yp;
            extrap(t, xp, yp);
            const uint32_t stop = we < jend ? we : jend;
            for (uint32_t g = j; g < stop; g += 4) {
              uint32_t ph[4];
              float xh[4], yh[4];
  #pragma unroll
              for (uint32_t q = 0; q < 4; ++q) {
                const uint32_t k = (g + q < stop ? g + q : stop - 1) - wb;
                ph[q] = k < l0 ? (w0 & 0xFFFFu) + k : (w1 & 0xFFFFu) + (k - l0);
                const float2 v = T0.xy(ph[q]);
                xh[q] = v.x;
                yh[q] = v.y;
              }
  #pragma unroll
              for (uint32_t q = 0; q < 4; ++q) {
                if (g + q >= stop) continue;
                const float dx = xh[q] - xp, dy = yh[q] - yp;
                const float s = dx * dx + dy * dy;
                if (s <= P.s_fwd) add_ext(t, key0, ph[q], s);
              }
            }
            j = stop;
          }
        }
      } else {
        for (uint32_t t = tid; t < n_act; t += NT) {
          A.tmatch[t] = kNone;
          A.tbest[t] = kFree;
          const uint32_t key0 = A.key0[t];
          float xp, yp;
          extrap(t, xp, yp);
          Ranges r = window(pangle(xp, yp), point_window(xp, yp, P.rho_fwd), kNB);
          scan_window(T0, r, [&](uint32_t h, float xh, float yh) {
            const float dx = xh - xp, dy = yh - yp;
            const float s = dx * dx + dy * dy;
            if (s <= P.s_fwd) add_ext(t, key0, h, s);
          });
        }
      }
      wg_barrier<RING>();
      {
        const uint32_t nc = sc.ncf;
        if (nc > VELO_MAX_CANDIDATES) return 2u;
        if (nc > M.capC) return 1u;
        if (nc > 0) {
          // greedy matching by (s, first-hit key of the track, hit key)
          auto less_hit = [&](uint32_t i, uint32_t j) {
            const Cand ci = M.cand[i], cj = M.cand[j];
            if (ci.s != cj.s) return ci.s < cj.s;
            return A.key0[ci.a] < A.key0[cj.a];
          };
          auto less_trk = [&](uint32_t i, uint32_t j) {
            const Cand ci = M.cand[i], cj = M.cand[j];
            if (ci.s != cj.s) return ci.s < cj.s;
            return T0.kr[ci.b] < T0.kr[cj.b];
          };
          // (track, hit) of candidate k, the lane's j-th
          auto th = [&](uint32_t k, int j, uint32_t& t, uint32_t& h) {
            if constexpr (RING) { const uint32_t v = cpos_r[j]; t = v & kPosMask; h = v >> kPosBits; }
            else { const Cand c = M.cand[k]; t = c.a; h = c.b; }
          };
          auto live = [&](uint32_t t, uint32_t h) { return A.tmatch[t] == kNone && !T0.used[h]; };
          load_cands(nc);
          greedy_rounds<RING>(
              nc, sc,
              [&](bool first) {
                for_cands(nc, [&](uint32_t k, int j) {
                  uint32_t t, h;
                  th(k, j, t, h);
                  if (!first && !live(t, h)) return;
                  if constexpr (RING) {
                    atomicMin((unsigned long long*)(T0.best + h), (unsigned long long)cprio_r[j]);
                    atomicMin((unsigned long long*)(A.tbest + t), (unsigned long long)cprio_r[j]);
                  } else {
                    cas_min(T0.best + h, k, less_hit);
                    cas_min(A.tbest + t, k, less_trk);
                  }
                });
              },
              [&] {
                for_cands(nc, [&](uint32_t k, int j) {
                  uint32_t t, h;
                  th(k, j, t, h);
                  if (holds(T0.best + h, k, j) && holds(A.tbest + t, k, j)) {
                    A.tmatch[t] = h;
                    T0.used[h] = 1;
                  }
                });
              },
              [&] {
                bool any = false;
                for_cands(nc, [&](uint32_t k, int j) {
                  uint32_t t, h;
                  th(k, j, t, h);
                  T0.best[h] = kFree;
                  A.tbest[t] = kFree;
                  if (live(t, h)) any = true;
                });
                return any;
              });
        }
      }
      // apply: append matched hits, count misses
      for (uint32_t t = tid; t < n_act; t += NT) {
        const uint32_t h = A.tmatch[t];
        if (h != kNone) {
          const uint32_t nn = A.n[t];
          io.hit_idx[26ull * (io.slot_base + A.slot[t]) + nn] = base0 + (uint32_t)T0.kr[h];
          const float2 vh = T0.xy(h);
          const float xh = vh.x, yh = vh.y;
          const float dz = zl - zt[A.la[t]];
          const float4 v = A.st[t];
          A.st[t] = make_float4(xh, yh, (xh - v.x) / dz, (yh - v.y) / dz);
          A.la[t] = (uint8_t)l;
          A.n[t] = (uint8_t)(nn + 1);
          A.skip[t] = 0;
        } else {
          const int sk = A.skip[t] + 1;
          A.skip[t] = (uint8_t)sk;
          if (sk > P.max_skip) io.nhits[io.slot_base + A.slot[t]] = A.n[t];
        }
      }
    }
    // (no barrier: seeding touches neither the track table nor what the
    // matching changed since its last round's barrier; the workspace tier's
    // seed loop reads plane l's flags at once, so it needs the step-start
    // clearing published when no extension phase did)
    if constexpr (!RING) {
      if (n_act == 0) wg_barrier<RING>();
    }

    // ---- 2. seeds on planes (l+2, l+1, l) ----
    uint32_t n_new = 0;
    bool seed_rounds = false;  // conflict rounds ran (their barriers follow the staging's starts)
    const auto T1 = M.layer(io, l < kLayers - 1 ? l + 1 : l);
    const auto T2 = M.layer(io, l < kLayers - 2 ? l + 2 : l);
    uint32_t n1 = 0, n2 = 0;
    if (l <= kLayers - 3) {
      n1 = io.lnh[l + 1];
      n2 = io.lnh[l + 2];
      const float z0 = zt[l + 2], z1 = zt[l + 1], z2 = zl;
      const float dz01 = z1 - z0;
      const float d12 = z2 - z1;
      // third hit of a doublet (h0, h1): unused, within sqrt(s_seed) of the line
      auto triplets = [&](uint32_t i0, uint32_t i1, float tx, float ty) {
        const float2 v1 = T1.xy(i1);
        const float xp = v1.x + tx * d12;
        const float yp = v1.y + ty * d12;
        Ranges r2 = window(pangle(xp, yp), point_window(xp, yp, P.rho_seed), kNB);
        scan_window(T0, r2, [&](uint32_t i2, float x2, float y2) {
          const float dx = x2 - xp, dy = y2 - yp;
          const float s = dx * dx + dy * dy;
          if (s <= P.s_seed && !T0.used[i2]) {
            uint32_t k = atomicAdd(&sc.ncs, 1u);
            if (k < M.capC) {
              if constexpr (RING) {
                M.cprio[k] = ((uint64_t)__float_as_uint(s) << 32) |
                             ((uint64_t)T1.kr[i1] << (2 * kPosBits)) |
                             ((uint64_t)T2.kr[i0] << kPosBits) | (uint64_t)T0.kr[i2];
                M.cpos[k] = i0 | (i1 << kPosBits) | (i2 << (2 * kPosBits));
              } else {
                M.cand[k] = Cand{s, i0, i1, i2};
              }
            }
          }
        });
      };
      // doublet cuts of (h0 on l+2, h1 on l+1); returns false if rejected
      // (the division-free azimuth cuts first: most pairs fail them)
      auto doublet = [&](float x0, float y0, float x1, float y1, float& tx, float& ty) {
        const float cr = x0 * y1 - y0 * x1;
        const float r0s = x0 * x0 + y0 * y0;
        const float r1s = x1 * x1 + y1 * y1;
        if (!(cr * cr <= (P.sin2 * r0s) * r1s)) return false;
        if (!(x0 * x1 + y0 * y1 > 0.0f)) return false;
        tx = (x1 - x0) / dz01;
        ty = (y1 - y0) / dz01;
        return fabsf(tx) <= P.max_t && fabsf(ty) <= P.max_t;
      };
      // the slope cut |fl(d / dz01)| <= max_t without the division: the product
      // with the rounded reciprocal is within 2^-23 (relative) of the quotient, so
      // it decides every case outside a relative 1e-5 of the cut, and the
      // division decides the rest
      const float inv01 = 1.0f / dz01;
      const float t_in = P.max_t * 0.99999f, t_out = P.max_t * 1.00001f;
      auto slope_ok = [&](float d) {
        const float q = fabsf(d * inv01);
        if (q < t_in) return true;
        if (q > t_out) return false;
        return fabsf(d / dz01) <= P.max_t;
      };
      // the doublet cuts without the slopes' values (same decisions as doublet())
      auto doublet_ok = [&](float x0, float y0, float x1, float y1) {
        const float cr = x0 * y1 - y0 * x1;
        const float r0s = x0 * x0 + y0 * y0;
        const float r1s = x1 * x1 + y1 * y1;
        if (!(cr * cr <= (P.sin2 * r0s) * r1s)) return false;
        if (!(x0 * x1 + y0 * y1 > 0.0f)) return false;
        return slope_ok(x1 - x0) && slope_ok(y1 - y0);
      };
      if constexpr (RING) {
        // (a) window of every unused middle hit on plane l+2, prefix of the sizes
        uint32_t carry = 0;
        for (uint32_t b0 = 0; b0 < n1; b0 += NT) {
          const uint32_t i1 = b0 + tid;
          uint32_t cnt = 0;
          if (i1 < n1 && !T1.used[i1]) {
            const float2 v1 = T1.xy(i1);
            const Ranges r = window(pangle(v1.x, v1.y), P.win_doublet, kNB);
            const uint32_t s0 = T2.bstart[r.b0], l0 = T2.bstart[r.b1 + 1] - s0;
            uint32_t s1 = 0, l1 = 0;
            if (r.b2 <= r.b3) { s1 = T2.bstart[r.b2]; l1 = T2.bstart[r.b3 + 1] - s1; }
            M.w0[i1] = s0 | (l0 << 16);
            M.w1[i1] = s1 | (l1 << 16);
            cnt = l0 + l1;
          }
          uint32_t tot;
          const uint32_t ex = scan(cnt, &tot);
          if (i1 < n1) M.wp[i1] = carry + ex;
          if (n1 <= NT && cnt > 0) {
            // one pass: the middle hit whose pairs contain a lane's first pair
            // (below) is known here, so that lane need not search for it
            const uint32_t per = (tot + NT - 1) / NT;
            for (uint32_t L = (ex + per - 1) / per; L * per < ex + cnt; ++L) M.own[L] = i1;
          }
          carry += tot;
        }
        if (tid == 0) M.wp[n1] = carry;
        wg_barrier<RING>();
        // (b) all (h1, h0) pairs, split evenly over the lanes in contiguous chunks;
        // four pairs of one middle hit per step, their loads issued together
        const uint32_t total = carry, per = (total + NT - 1) / NT;
        uint32_t j = tid * per;
        const uint32_t jend = j + per < total ? j + per : total;
        if (j < jend) {
          uint32_t lo = 0, hi = n1 - 1;
          if (n1 <= NT) {
            lo = M.own[tid];
          } else {
            while (lo < hi) {
              const uint32_t mid = (lo + hi + 1) >> 1;
              if (M.wp[mid] <= j) lo = mid; else hi = mid - 1;
            }
          }
          for (uint32_t i1 = lo; j < jend; ++i1) {
            const uint32_t wb = M.wp[i1], we = M.wp[i1 + 1];
            if (we <= j) continue;
            const uint32_t w0 = M.w0[i1], w1 = M.w1[i1], l0 = w0 >> 16;
            const float2 v1 = T1.xy(i1);
            const float x1 = v1.x, y1 = v1.y;
            const uint32_t stop = we < jend ? we : jend;
            for (uint32_t g = j; g < stop; g += 4) {
              uint32_t pj[4];
              float x0[4], y0[4];
              uint8_t u0[4];
#pragma unroll
              for (uint32_t q = 0; q < 4; ++q) {
                const uint32_t jj = g + q < stop ? g + q : stop - 1;
                const uint32_t k = jj - wb;
                pj[q] = k < l0 ? (w0 & 0xFFFFu) + k : (w1 & 0xFFFFu) + (k - l0);
                const float2 v0 = T2.xy(pj[q]);
                x0[q] = v0.x;
                y0[q] = v0.y;
                u0[q] = T2.used[pj[q]];
              }
#pragma unroll
              for (uint32_t q = 0; q < 4; ++q) {
                if (g + q >= stop || u0[q]) continue;
                if (!doublet_ok(x0[q], y0[q], x1, y1)) continue;
                const uint32_t d = atomicAdd(&sc.nd, 1u);
                if (d < M.capD) M.dbl[d] = pj[q] | (i1 << 16);
              }
            }
            j = stop;
          }
        }
        wg_barrier<RING>();
        const uint32_t nd = sc.nd;
        if (nd > M.capD) return 1u;
        // (c) third hits, one doublet per lane
        for (uint32_t d = tid; d < nd; d += NT) {
          const Dbl r = M.dbl[d];
          const uint32_t i0 = r & 0xFFFFu, i1 = r >> 16;
          const float2 v1 = T1.xy(i1), v0 = T2.xy(i0);
          const float tx = (v1.x - v0.x) / dz01;
          const float ty = (v1.y - v0.y) / dz01;
          triplets(i0, i1, tx, ty);
        }
      } else {
        for (uint32_t i1 = tid; i1 < n1; i1 += NT) {
          if (T1.used[i1]) continue;
          const float2 v1 = T1.xy(i1);
          const Ranges r0 = window(pangle(v1.x, v1.y), P.win_doublet, kNB);
          const float x1 = v1.x, y1 = v1.y;
          scan_window(T2, r0, [&](uint32_t i0, float x0, float y0) {
            if (T2.used[i0]) return;
            float tx, ty;
            if (doublet(x0, y0, x1, y1, tx, ty)) triplets(i0, i1, tx, ty);
          });
        }
      }
      // staging of plane l-1: bucket ranks (published by the next barrier),
      // then the bucket starts (the slot's starts were last read by the
      // doublet search, which is over)
      if (l > 0) pf.count(M);
      wg_barrier<RING>();
      if (l > 0) pf.starts(io, l - 1, M);
      const uint32_t nc = sc.ncs;
      if (nc > VELO_MAX_CANDIDATES) return 2u;
      if (nc > M.capC) return 1u;
      seed_rounds = nc > 0;
      if (nc > 0) {
        // greedy independent set by (s, key1, key0, key2)
        auto less_seed = [&](uint32_t i, uint32_t j) {
          const Cand ci = M.cand[i], cj = M.cand[j];
          if (ci.s != cj.s) return ci.s < cj.s;
          if (ci.b != cj.b) return T1.kr[ci.b] < T1.kr[cj.b];
          if (ci.a != cj.a) return T2.kr[ci.a] < T2.kr[cj.a];
          return T0.kr[ci.c] < T0.kr[cj.c];
        };
        // hits (h0, h1, h2) of candidate k, the lane's j-th
        auto hits3 = [&](uint32_t k, int j, uint32_t& i0, uint32_t& i1, uint32_t& i2) {
          if constexpr (RING) {
            const uint32_t v = cpos_r[j];
            i0 = v & kPosMask; i1 = (v >> kPosBits) & kPosMask; i2 = (v >> (2 * kPosBits)) & kPosMask;
          } else {
            const Cand c = M.cand[k]; i0 = c.a; i1 = c.b; i2 = c.c;
          }
        };
        auto alive = [&](uint32_t i0, uint32_t i1, uint32_t i2) {
          return !T2.used[i0] && !T1.used[i1] && !T0.used[i2];
        };
        load_cands(nc);
        greedy_rounds<RING>(
            nc, sc,
            [&](bool first) {
              for_cands(nc, [&](uint32_t k, int j) {
                uint32_t i0, i1, i2;
                hits3(k, j, i0, i1, i2);
                if (!first && !alive(i0, i1, i2)) return;
                if constexpr (RING) {
                  const unsigned long long pr = cprio_r[j];
                  atomicMin((unsigned long long*)(T2.best + i0), pr);
                  atomicMin((unsigned long long*)(T1.best + i1), pr);
                  atomicMin((unsigned long long*)(T0.best + i2), pr);
                } else {
                  cas_min(T2.best + i0, k, less_seed);
                  cas_min(T1.best + i1, k, less_seed);
                  cas_min(T0.best + i2, k, less_seed);
                }
              });
            },
            [&] {
              for_cands(nc, [&](uint32_t k, int j) {
                uint32_t i0, i1, i2;
                hits3(k, j, i0, i1, i2);
                if (holds(T2.best + i0, k, j) && holds(T1.best + i1, k, j) &&
                    holds(T0.best + i2, k, j)) {
                  T2.used[i0] = 1;
                  T1.used[i1] = 1;
                  T0.used[i2] = 1;
                  if constexpr (RING) cpos_r[j] |= kAccepted;
                  else M.cand[k].s = -1.0f;  // accepted (every real s is >= 0)
                }
              });
            },
            [&] {
              bool any = false;
              for_cands(nc, [&](uint32_t k, int j) {
                uint32_t i0, i1, i2;
                hits3(k, j, i0, i1, i2);
                T2.best[i0] = kFree;
                T1.best[i1] = kFree;
                T0.best[i2] = kFree;
                if (alive(i0, i1, i2)) any = true;
              });
              return any;
            });
        // accepted seed of each h0, stored by the local index of h0 (the slots
        // are clear; nothing reads plane l+2 by position any more)
        for_cands(nc, [&](uint32_t k, int j) {
          uint32_t i0, i1, i2;
          hits3(k, j, i0, i1, i2);
          bool acc;
          if constexpr (RING) acc = (cpos_r[j] & kAccepted) != 0;
          else acc = M.cand[k].s < 0.0f;
          if (acc) T2.best[T2.kr[i0]] = (SLOT)k;
        });
        wg_barrier<RING>();
      }
    }

    // place plane l-1 into the slot of plane l+2, whose coordinates and local
    // indices the seeds no longer read (its round winners stay: they hold the
    // accepted seeds); steps without seeding count and scan here
    if (RING && l > 0) {
      if (l > kLayers - 3) {
        pf.count(M);
        wg_barrier<RING>();
        pf.starts(io, l - 1, M);
        wg_barrier<RING>();
      } else if (!seed_rounds) {
        wg_barrier<RING>();  // publishes the starts (no round barrier did)
      }
      pf.place(io, l - 1, M);
    }

    // ---- 3. active table: surviving tracks compacted in place, then new seeds ----
    // Every lane reads its entry before the scan's barrier and writes after it;
    // entries only move down, and a chunk writes below the entries of later chunks.
    const bool seeds = l <= kLayers - 3 && sc.ncs > 0;
    const uint32_t created = sc.n_created;  // read before any scan barrier (updated at the step end)
    // a new track from the accepted seed of h0 (local index i0 on plane l+2)
    auto create = [&](uint32_t i0, uint32_t k, uint32_t rank, uint32_t n_keep) {
      uint32_t cb, cc;
      if constexpr (RING) {
        const uint32_t v = M.cpos[k];
        cb = (v >> kPosBits) & kPosMask; cc = (v >> (2 * kPosBits)) & kPosMask;
      } else {
        const Cand c = M.cand[k]; cb = c.b; cc = c.c;
      }
      uint32_t* hi = io.hit_idx + 26ull * (io.slot_base + created + rank);
      hi[0] = io.lstart[l + 2] + i0;
      hi[1] = io.lstart[l + 1] + (uint32_t)T1.kr[cb];
      hi[2] = base0 + (uint32_t)T0.kr[cc];
      const uint32_t pos = n_keep + rank;
      if (pos < M.capT) {
        const float2 v1 = T1.xy(cb), v2 = T0.xy(cc);
        const float x1 = v1.x, y1 = v1.y, x2 = v2.x, y2 = v2.y;
        const float dz = zl - zt[l + 1];
        A.slot[pos] = (IDX)(created + rank);
        A.key0[pos] = (IDX)(((uint32_t)(l + 2) << M.KSH) | i0);
        A.st[pos] = make_float4(x2, y2, (x2 - x1) / dz, (y2 - y1) / dz);
        A.la[pos] = (uint8_t)l;
        A.n[pos] = 3;
        A.skip[pos] = 0;
      }
    };
    struct Keep { uint32_t slot, key0; float4 st; uint8_t la, n, skip; };
    auto read_keep = [&](uint32_t t) {
      return Keep{A.slot[t], A.key0[t], A.st[t], A.la[t], A.n[t], A.skip[t]};
    };
    auto write_keep = [&](uint32_t pos, const Keep& f) {
      A.slot[pos] = (IDX)f.slot; A.key0[pos] = (IDX)f.key0; A.st[pos] = f.st;
      A.la[pos] = f.la; A.n[pos] = f.n; A.skip[pos] = f.skip;
    };
    uint32_t n_keep;
    if (n_act <= NT && (!seeds || n2 <= NT)) {
      // one scan for both: survivors in the low half-word, new tracks in the high
      const bool keep = tid < n_act && (int)A.skip[tid] <= P.max_skip;
      Keep f{};
      if (keep) f = read_keep(tid);
      const uint32_t i0 = seeds && tid < n2 ? n2 - 1 - tid : kNone;
      const SLOT kk = i0 != kNone ? T2.best[i0] : kFree;
      uint32_t tot;
      const uint32_t ex = scan((keep ? 1u : 0u) | (kk != kFree ? 0x10000u : 0u), &tot);
      n_keep = tot & 0xFFFFu;
      n_new = tot >> 16;
      if (keep) write_keep(ex & 0xFFFFu, f);
      if (kk != kFree) create(i0, (uint32_t)kk, ex >> 16, n_keep);
    } else {
      uint32_t carry = 0;
      for (uint32_t b0 = 0; b0 < n_act; b0 += NT) {
        const uint32_t t = b0 + tid;
        const bool keep = t < n_act && (int)A.skip[t] <= P.max_skip;
        Keep f{};
        if (keep) f = read_keep(t);
        uint32_t tot;
        const uint32_t pos = carry + scan(keep ? 1u : 0u, &tot);
        if (keep) write_keep(pos, f);
        carry += tot;
      }
      n_keep = carry;
      if (seeds) {
        // seeds in decreasing key of h0 (decreasing local index on plane l+2)
        uint32_t c2 = 0;
        for (uint32_t b0 = 0; b0 < n2; b0 += NT) {
          const uint32_t i0 = b0 + tid < n2 ? n2 - 1 - (b0 + tid) : kNone;
          const SLOT kk = i0 != kNone ? T2.best[i0] : kFree;
          uint32_t tot;
          const uint32_t rank = c2 + scan(kk != kFree ? 1u : 0u, &tot);
          if (kk != kFree) create(i0, (uint32_t)kk, rank, n_keep);
          c2 += tot;
        }
        n_new = c2;
      }
    }
    if (n_keep + n_new > M.capT) return 1u;
    if (tid == 0) { sc.n_act = n_keep + n_new; sc.n_created += n_new; sc.ncf = 0; }
    wg_barrier<RING>();
  }
  // close the tracks still active after the first plane
  for (uint32_t t = tid; t < sc.n_act; t += NT) io.nhits[io.slot_base + A.slot[t]] = A.n[t];
  wg_barrier<RING>();
  return 0u;
}

// ---------------------------------------------------------------------------

// Lengths of the tiers' hand-over lists (and of the routing lists), cleared
// before the first tier runs.
__global__ __launch_bounds__(64) void k_clear_counts(uint32_t* __restrict__ esc_counts) {
  if (threadIdx.x < 5) esc_counts[threadIdx.x] = 0;
}

struct FindArgs {
  const float* X;  // hit coordinates in bucket order (absolute slots; workspace tier)
  const float* Y;
  const float* HX;  // hit coordinates in key order (the hits, absolute slots)
  const float* HY;
  const uint32_t* hstatus;
  const uint32_t* lstart;
  const uint32_t* lnh;
  const uint32_t* order;  // azimuth tables (absolute hit slots / per plane)
  const uint32_t* bst;
  const uint64_t* offsets;
  uint64_t n_pixels;
  uint32_t* n_tracks;
  uint8_t* nhits;
  uint32_t* hit_idx;
  uint32_t* tstatus;
  uint32_t* esc_count;  // events handed to the next tier
  uint32_t* esc_list;
};

__device__ __forceinline__ EventIO event_io(const FindArgs& a, uint32_t e) {
  const uint64_t b = a.offsets[e];
  return EventIO{a.X + b, a.Y + b, a.HX + b, a.HY + b, a.lstart + 27ull * e, a.lnh + 26ull * e, a.order + b,
                 a.bst + (uint64_t)e * kLayers * (kNB + 1), a.nhits, a.hit_idx, b / 3};
}

__device__ __forceinline__ bool event_skipped(const FindArgs& a, uint32_t e) {
  const uint64_t b = a.offsets[e], b1 = a.offsets[e + 1];
  return a.hstatus[e] != 0 || b1 <= b || b1 > a.n_pixels;
}

// Run one event in the given tier.  Returns true if it must go to the next.
template <int NT, typename IDX, bool RING>
__device__ __forceinline__ bool run_event(const FindArgs& a, const FindConst& P,
                                          const FindMem<IDX, RING>& M, FindScal& sc, uint32_t e) {
  if (event_skipped(a, e)) {
    if (threadIdx.x == 0) { a.n_tracks[e] = 0; a.tstatus[e] = 0; }
    return false;
  }
  EventIO io = event_io(a, e);
  for (uint32_t i = threadIdx.x; i < 27; i += NT) sc.lstart[i] = io.lstart[i];
  for (uint32_t i = threadIdx.x; i < 26; i += NT) { sc.lnh[i] = io.lnh[i]; sc.z[i] = kLayerZ[i]; }
  __syncthreads();
  io.lstart = sc.lstart;
  io.lnh = sc.lnh;
  const uint32_t r = find_event<NT>(io, P, M, sc);
  if (r == 1u) return true;
  if (threadIdx.x == 0) {
    a.n_tracks[e] = r == 0u ? sc.n_created : 0u;
    a.tstatus[e] = r == 0u ? 0u : (uint32_t)VELO_EV_OVERFLOW;
  }
  return false;
}

// LDS tiers: one event per workgroup (list == nullptr) or a persistent loop
// over a list of events.
template <int NT, uint32_t CAPL, uint32_t CAPT, uint32_t CAPC, uint32_t CAPD>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 256 ? (CAPL <= 192 ? 6 : 5) : (NT >= 512 ? 4 : 1)))) void k_find_lds(FindArgs a, FindConst P, uint32_t n_events,
                                                 const uint32_t* __restrict__ list,
                                                 const uint32_t* __restrict__ list_count,
                                                 uint32_t* __restrict__ steal) {
  __shared__ float2 s_hxy[3 * CAPL];  // x, y of every ring position
  __shared__ uint16_t s_kr[3 * CAPL];
  __shared__ uint8_t s_used[3 * CAPL];
  __shared__ uint64_t s_best[3 * CAPL];
  __shared__ uint16_t s_bstart[3 * (kNB + 1)];
  __shared__ uint16_t t_slot[CAPT], t_key0[CAPT];
  __shared__ float4 t_st[CAPT];
  __shared__ uint8_t t_la[CAPT], t_n[CAPT], t_skip[CAPT];
  // candidates (priorities, positions) share their space with the seed doublet
  // windows: the windows are dead before the first seed candidate is written,
  // and extension candidates are dead before the windows are built
  constexpr uint32_t kCandBytes = 12u * CAPC, kWinBytes = 4u * (3u * CAPL + 1u + NT);
  __shared__ uint64_t s_cw[((kCandBytes > kWinBytes ? kCandBytes : kWinBytes) + 7u) / 8u];
  // the matches and round winners of the extension step share their space with
  // the seed doublets: the doublets are written after the barrier that ends
  // the first seeding phase (every match is applied by then) and are dead
  // before the next step's extension phase
  static_assert(CAPT % 2 == 0 && CAPD % 2 == 0, "8-byte alignment of the shared region");
  constexpr uint32_t kTdBytes = 12u * CAPT > 4u * CAPD ? 12u * CAPT : 4u * CAPD;
  __shared__ uint64_t s_td[kTdBytes / 8];
  uint32_t* t_tmatch = reinterpret_cast<uint32_t*>(s_td);
  uint64_t* t_tbest = s_td + CAPT / 2;
  __shared__ uint32_t s_tw[NT >= 512 ? 3 * CAPT + 1 + NT : 1];  // balanced forward search only
  __shared__ uint32_t s_cnt[kNB / 2];  // bucket counters of the plane being staged
  __shared__ FindScal sc;
  FindMem<uint16_t, true> M;
  M.tw0 = s_tw; M.tw1 = s_tw + CAPT; M.twp = s_tw + 2 * CAPT; M.twown = s_tw + 3 * CAPT + 1;
  uint32_t* cw = reinterpret_cast<uint32_t*>(s_cw);
  M.w0 = cw; M.w1 = cw + CAPL; M.wp = cw + 2 * CAPL; M.own = cw + 3 * CAPL + 1; M.dbl = reinterpret_cast<Dbl*>(s_td); M.capD = CAPD;
  M.hx = reinterpret_cast<float*>(s_hxy); M.hy = M.hx + 1; M.kr = s_kr; M.used = s_used; M.best = s_best; M.bstart = s_bstart;
  M.cnt = s_cnt;
  M.T = TrackTab<uint64_t, uint16_t>{t_slot, t_key0, t_st, t_la, t_n, t_skip, t_tbest,
                                     t_tmatch};
  M.cand = nullptr;
  M.cprio = s_cw;
  M.cpos = cw + 2 * CAPC;
  M.capL = CAPL; M.capT = CAPT; M.capC = CAPC;
  static_assert(CAPL <= (uint32_t)(kPrefetch<NT> * NT), "a plane's hits fit the lanes' staging registers");
  static_assert(CAPC <= (uint32_t)(kCandPerLane<NT> * NT), "the candidates fit the lanes' registers");
  // work items: events 0..n-1 or list[0..count); round robin over the grid, or
  // stolen from the `steal` counter (persistent workgroups) when it is given
  const uint32_t count = list_count ? *list_count : n_events;
  for (uint32_t it = steal ? pop_item(steal, &sc.item) : blockIdx.x; it < count;
       it = steal ? pop_item(steal, &sc.item) : it + gridDim.x) {
    const uint32_t e = list ? list[it] : it;
    if (run_event<NT>(a, P, M, sc, e) && threadIdx.x == 0) a.esc_list[atomicAdd(a.esc_count, 1u)] = e;
    __syncthreads();
  }
}

// Workspace tier: any event size.
constexpr int kGThreads = 256;
constexpr uint32_t kGBlocks = 128;

struct GlobalTabs {
  uint32_t* best; uint8_t* used;                                      // [n_pixels]
  uint32_t* slot; uint32_t* key0; uint32_t* tbest; uint32_t* tmatch;  // [n_pixels / 3 + 1]
  float4* st;
  uint8_t* la; uint8_t* n; uint8_t* skip;
  Cand* cand;  // per block: VELO_MAX_CANDIDATES
};

__global__ __launch_bounds__(kGThreads) void k_find_global(FindArgs a, FindConst P, GlobalTabs g,
                                                           const uint32_t* __restrict__ list,
                                                           const uint32_t* __restrict__ list_count) {
  __shared__ FindScal sc;
  __shared__ uint32_t cnt[kNB];
  const uint32_t count = *list_count;
  for (uint32_t it = blockIdx.x; it < count; it += gridDim.x) {
    const uint32_t e = list[it];
    const uint64_t b = a.offsets[e];
    // this tier reads the azimuth tables in place: build them for the event
    if (!event_skipped(a, e)) {
      const AzOut az{const_cast<uint32_t*>(a.order), const_cast<float*>(a.X), const_cast<float*>(a.Y),
                     const_cast<uint32_t*>(a.bst)};
      for (uint32_t l = 0; l < (uint32_t)kLayers; ++l) {
        azimuth_tables<kGThreads>(a.HX, a.HY, b + a.lstart[27ull * e + l], a.lnh[26ull * e + l],
                                  26ull * e + l, cnt, sc.tmp[0], az);
        __syncthreads();  // the next plane clears the counters
      }
    }
    const uint32_t ne = (uint32_t)(a.offsets[e + 1] - b);
    FindMem<uint32_t, false> M;
    M.hx = nullptr; M.hy = nullptr; M.kr = nullptr; M.bstart = nullptr;
    M.used = g.used + b;
    M.best = g.best + b;
    const uint64_t tb = b / 3;
    M.T = TrackTab<uint32_t, uint32_t>{g.slot + tb, g.key0 + tb, g.st + tb,
                   g.la + tb, g.n + tb, g.skip + tb, g.tbest + tb, g.tmatch + tb};
    M.cand = g.cand + (size_t)blockIdx.x * VELO_MAX_CANDIDATES;
    M.cprio = nullptr;
    M.cpos = nullptr;
    M.capL = ne;
    M.capT = (uint32_t)((b + ne) / 3 - b / 3);
    M.capC = VELO_MAX_CANDIDATES;
    M.w0 = M.w1 = M.wp = M.own = nullptr;
    M.tw0 = M.tw1 = M.twp = M.twown = nullptr;
    M.dbl = nullptr;
    M.capD = 0;
    M.cnt = nullptr;
    if (run_event<kGThreads>(a, P, M, sc, e) && threadIdx.x == 0) {
      // cannot happen: the tables hold every possible hit and track
      a.n_tracks[e] = 0;
      a.tstatus[e] = VELO_EV_OVERFLOW;
    }
    __syncthreads();
  }
}

// small LDS tier: one workgroup per event
constexpr int kSThreads = 256;
constexpr uint32_t kSCapL = 288, kSCapT = 256, kSCapC = 384, kSCapD = 3 * kSCapT;
// tiny LDS tier (batched form, optional, ahead of the small tier): 23.5 KB of
// LDS and at most 80 VGPRs, so six workgroups share a CU instead of five
constexpr uint32_t kTCapL = 192, kTCapT = 192, kTCapC = 256, kTCapD = 512;
// middle and large LDS tiers: persistent workgroups over the events the tier
// below hands on
constexpr int kMThreads = 512;
constexpr uint32_t kMCapL = 640, kMCapT = 512, kMCapC = 1024, kMCapD = 2304, kMBlocks = 512;
static_assert(kMCapL <= (1u << kPosBits) && kMCapT <= (1u << kPosBits), "packed positions");
constexpr int kLThreads = 1024;
constexpr uint32_t kLCapL = 1024, kLCapT = 1024, kLCapC = 2048, kLCapD = 4096, kLBlocks = 256;

static size_t up256(size_t v) { return (v + 255) & ~size_t(255); }

struct FindWs {
  uint32_t* esc_counts;  // [5] list lengths: small -> middle -> large -> workspace tier hand-overs,
                         // then the routed events (or the tiny tier's hand-overs) and the small
                         // tier's events (routing)
  uint32_t *esc_count, *esc_list, *esc2_count, *esc2_list, *esc3_count, *esc3_list, *order, *bst;
  uint32_t *route_count, *route_list, *small_count, *small_list;
  float *xs, *ys;
  GlobalTabs g;
};

// carve the workspace; returns the bytes used
static size_t find_ws_layout(char* w, uint64_t n_pixels, uint32_t n_events, FindWs* out) {
  size_t o = 0;
  auto take = [&](size_t bytes) { char* r = w ? w + o : nullptr; o += up256(bytes); return r; };
  const uint64_t nt = n_pixels / 3 + 1;
  FindWs f;
  f.esc_counts = (uint32_t*)take(20);
  f.esc_count = f.esc_counts;
  f.esc2_count = f.esc_counts ? f.esc_counts + 1 : nullptr;
  f.esc3_count = f.esc_counts ? f.esc_counts + 2 : nullptr;
  f.route_count = f.esc_counts ? f.esc_counts + 3 : nullptr;
  f.small_count = f.esc_counts ? f.esc_counts + 4 : nullptr;
  f.esc_list = (uint32_t*)take(4ull * n_events);
  f.esc2_list = (uint32_t*)take(4ull * n_events);
  f.esc3_list = (uint32_t*)take(4ull * n_events);
  f.route_list = (uint32_t*)take(4ull * n_events);
  f.small_list = (uint32_t*)take(4ull * n_events);
  f.order = (uint32_t*)take(4ull * n_pixels);
  f.xs = (float*)take(4ull * n_pixels);
  f.ys = (float*)take(4ull * n_pixels);
  f.bst = (uint32_t*)take(4ull * n_events * kLayers * (kNB + 1));
  f.g.best = (uint32_t*)take(4ull * n_pixels);
  f.g.used = (uint8_t*)take(n_pixels);
  f.g.slot = (uint32_t*)take(4 * nt);
  f.g.key0 = (uint32_t*)take(4 * nt);
  f.g.tbest = (uint32_t*)take(4 * nt);
  f.g.tmatch = (uint32_t*)take(4 * nt);
  f.g.st = (float4*)take(16 * nt);
  f.g.la = (uint8_t*)take(nt);
  f.g.n = (uint8_t*)take(nt);
  f.g.skip = (uint8_t*)take(nt);
  f.g.cand = (Cand*)take(sizeof(Cand) * (size_t)kGBlocks * VELO_MAX_CANDIDATES);
  if (out) *out = f;
  return o;
}

size_t find_workspace_bytes(uint64_t n_pixels, uint32_t n_events) {
  return find_ws_layout(nullptr, n_pixels, n_events, nullptr);
}

FindConst make_find_const(const velo_params* p) {
  FindConst c;
  c.max_t = p->max_t;
  c.sin2 = p->sin2_phi;
  c.s_seed = p->s_seed;
  c.s_fwd = p->s_fwd;
  c.max_skip = p->max_skip;
  const double u2 = p->sin2_phi;
  // azimuth difference <= asin(sqrt(u2)) <= sqrt(u2 / (1 - u2)), times the pseudo-angle's slope
  c.win_doublet = (u2 >= 0.5 || u2 < 0) ? 4.0f
                                        : (float)(kPaSlope * sqrt(u2 / (1.0 - u2)) * 1.001 + 1e-3);
  c.rho_seed = (float)(sqrt((double)(p->s_seed > 0 ? p->s_seed : 0)) * 1.001 + 1e-6);
  c.rho_fwd = (float)(sqrt((double)(p->s_fwd > 0 ? p->s_fwd : 0)) * 1.001 + 1e-6);
  return c;
}

// Launch shape of the track-finding stage (the batched form's autotuner picks it).
struct FindCfg {
  int small_threads;          // 128 or 256 lanes per event in the small tier
  uint32_t small_grid;        // 0: one workgroup per event; else persistent work stealing
  const uint32_t* ev_order;   // descending-size order of the events (work stealing)
  uint32_t* counters;         // [3] zeroed work-stealing counters (work stealing)
  // persistent workgroups of the middle, large and workspace tiers over the
  // events handed on to them (0: kMBlocks, kLBlocks, kGBlocks; larger values
  // are clamped to those).  A tier's launch holds its workgroups' LDS until
  // every one of them has been placed and found the list empty, so a small
  // grid frees the GPU sooner when few events escalate.
  uint32_t esc_grid[3];
  // Routing (batched form; needs small_grid == 0): events with a plane above
  // the small tier's capacity, or with more than route_hits hits, go straight
  // to the middle tier instead of being handed on by the small tier, possibly
  // after part of their work (0: no routing).  side (may be null): the middle
  // tier of the routed events then runs on this stream, forked from `s` by
  // fork_ev and joined back by join_ev, beside the small tier.
  uint32_t route_hits;
  hipStream_t side;
  hipEvent_t fork_ev, join_ev;
  // small_grid == 0: the small tier (and routing) takes the events in
  // ev_order (largest first) instead of index order
  uint32_t ordered;
  // small_grid == 0, no routing, 256 lanes: the tiny tier runs every event
  // first and hands on to the small tier those above its capacities
  uint32_t tiny;
};

static uint32_t tier_grid(uint32_t want, uint32_t full) { return want == 0 || want > full ? full : want; }

// Routing (batched form): one lane per event (in `order` when given, so that
// the lists keep it within each wave).  A skipped event gets its
// empty outputs here (no tier sees it); an event with a plane above the small
// tier's capacity or more than route_hits hits goes to the routed list, the
// others to the small tier's list.
__global__ __launch_bounds__(256) void k_route(FindArgs a, uint32_t n_events, uint32_t route_hits,
                                               const uint32_t* __restrict__ order,
                                               uint32_t* __restrict__ route_count,
                                               uint32_t* __restrict__ route_list,
                                               uint32_t* __restrict__ small_count,
                                               uint32_t* __restrict__ small_list) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n_events) return;
  const uint32_t e = order ? order[i] : i;
  if (event_skipped(a, e)) {
    a.n_tracks[e] = 0;
    a.tstatus[e] = 0;
    return;
  }
  uint32_t mx = 0, tot = 0;
  for (int l = 0; l < kLayers; ++l) {
    const uint32_t v = a.lnh[26ull * e + l];
    mx = v > mx ? v : mx;
    tot += v;
  }
  if (mx > kSCapL || tot > route_hits) route_list[atomicAdd(route_count, 1u)] = e;
  else small_list[atomicAdd(small_count, 1u)] = e;
}

// ev (may be null): events recorded just before and after the per-event kernel
hipError_t launch_find_cfg(const velo_hits* h, const uint64_t* offsets, uint32_t n_events,
                           uint64_t n_pixels, const velo_params* p, const velo_tracks* t, void* ws,
                           hipStream_t s, const FindCfg& cfg, const hipEvent_t* ev = nullptr) {
  FindWs f;
  find_ws_layout((char*)ws, n_pixels, n_events, &f);
  FindArgs a{f.xs, f.ys, h->x, h->y, h->status, h->layer_start, h->layer_nhits, f.order, f.bst, offsets,
             n_pixels, t->n_tracks, t->nhits, t->hit_idx, t->status, f.esc_count, f.esc_list};
  const FindConst c = make_find_const(p);
  hipLaunchKernelGGL(k_clear_counts, dim3(1), dim3(64), 0, s, f.esc_counts);
  const bool route = cfg.route_hits != 0 && cfg.small_grid == 0;
  const bool ws_mode = cfg.small_grid != 0;
  const dim3 grid(ws_mode ? cfg.small_grid : n_events);
  const uint32_t* order = ws_mode || cfg.ordered ? cfg.ev_order : nullptr;
  uint32_t* steal = ws_mode ? cfg.counters : nullptr;
  FindArgs a2 = a;
  a2.esc_count = f.esc2_count;
  a2.esc_list = f.esc2_list;
  const dim3 mgrid(tier_grid(cfg.esc_grid[0], kMBlocks));
  if (route) {
    hipLaunchKernelGGL(k_route, dim3((n_events + 255) / 256), dim3(256), 0, s, a, n_events, cfg.route_hits,
                       order, f.route_count, f.route_list, f.small_count, f.small_list);
    // the middle tier on the routed events: beside the small tier on the side
    // stream, or before it
    hipStream_t ms = s;
    if (cfg.side) {
      hipError_t e = hipEventRecord(cfg.fork_ev, s);
      if (e == hipSuccess) e = hipStreamWaitEvent(cfg.side, cfg.fork_ev, 0);
      if (e != hipSuccess) return e;
      ms = cfg.side;
    }
    hipLaunchKernelGGL((k_find_lds<kMThreads, kMCapL, kMCapT, kMCapC, kMCapD>), mgrid, dim3(kMThreads), 0, ms,
                       a2, c, n_events, f.route_list, f.route_count, (uint32_t*)nullptr);
    if (cfg.side) {
      hipError_t e = hipEventRecord(cfg.join_ev, cfg.side);
      if (e != hipSuccess) return e;
    }
  }
  const uint32_t* slist = route ? f.small_list : order;
  const uint32_t* scount = route ? f.small_count : (const uint32_t*)nullptr;
  if (ev && ev[0]) (void)hipEventRecord(ev[0], s);
  if (cfg.tiny && !route && !ws_mode && cfg.small_threads == kSThreads) {
    // the tiny tier's hand-overs go through the (otherwise unused) routing list
    FindArgs a0 = a;
    a0.esc_count = f.route_count;
    a0.esc_list = f.route_list;
    hipLaunchKernelGGL((k_find_lds<kSThreads, kTCapL, kTCapT, kTCapC, kTCapD>), grid, dim3(kSThreads), 0, s, a0,
                       c, n_events, slist, scount, (uint32_t*)nullptr);
    slist = f.route_list;
    scount = f.route_count;
  }
  if (cfg.small_threads == 128)
    hipLaunchKernelGGL((k_find_lds<128, kSCapL, kSCapT, kSCapC, kSCapD>), grid, dim3(128), 0, s, a, c,
                       n_events, slist, scount, steal);
  else
    hipLaunchKernelGGL((k_find_lds<kSThreads, kSCapL, kSCapT, kSCapC, kSCapD>), grid, dim3(kSThreads),
                       0, s, a, c, n_events, slist, scount, steal);
  if (ev && ev[1]) (void)hipEventRecord(ev[1], s);
  if (route && cfg.side) {
    hipError_t e = hipStreamWaitEvent(s, cfg.join_ev, 0);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_find_lds<kMThreads, kMCapL, kMCapT, kMCapC, kMCapD>), mgrid,
                     dim3(kMThreads), 0, s, a2, c, n_events, f.esc_list, f.esc_count,
                     ws_mode ? cfg.counters + 1 : (uint32_t*)nullptr);
  FindArgs a3 = a;
  a3.esc_count = f.esc3_count;
  a3.esc_list = f.esc3_list;
  hipLaunchKernelGGL((k_find_lds<kLThreads, kLCapL, kLCapT, kLCapC, kLCapD>), dim3(tier_grid(cfg.esc_grid[1], kLBlocks)),
                     dim3(kLThreads), 0, s, a3, c, n_events, f.esc2_list, f.esc2_count,
                     ws_mode ? cfg.counters + 2 : (uint32_t*)nullptr);
  hipLaunchKernelGGL(k_find_global, dim3(tier_grid(cfg.esc_grid[2], kGBlocks)), dim3(kGThreads), 0, s, a3, c, f.g, f.esc3_list,
                     f.esc3_count);
  return hipGetLastError();
}

hipError_t launch_find(const velo_hits* h, const uint64_t* offsets, uint32_t n_events,
                       uint64_t n_pixels, const velo_params* p, const velo_tracks* t, void* ws,
                       hipStream_t s) {
  return launch_find_cfg(h, offsets, n_events, n_pixels, p, t, ws, s,
                         FindCfg{kSThreads, 0, nullptr, nullptr, {0, 0, 0}, 0, nullptr, nullptr, nullptr, 0, 0});
}

}  // namespace velo
