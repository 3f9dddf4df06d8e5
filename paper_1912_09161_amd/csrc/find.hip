// find.hip -- VELO track finding by triplet seeding and forwarding
// (paper Sec. 2.3.1, second paragraph: seeds of three hits on consecutive
// planes, extended to the other planes along straight lines; hits of every
// plane kept in azimuth order for fast look-up).
//
// One workgroup per event walks the planes from z = +750 mm down.  The three
// planes in use (l+2, l+1, l) are staged in a ring of per-plane tables:
// coordinates, a counting sort of the hits into azimuth buckets (a monotone
// pseudo-angle of x, y), used flags.  Candidate windows in pseudo-angle are
// derived conservatively from the exact cuts, so they only accelerate; every
// decision uses the exact binary32 cut expressions.
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
// Three tiers share one implementation: 64 lanes with small LDS tables, 256
// lanes with large LDS tables, and 256 lanes with tables in the caller's
// workspace at the event's own hit / track positions.  An event whose tables
// outgrow its tier is re-run from scratch by the next tier.
#include "velo_device.hpp"

namespace velo {

constexpr uint32_t kNone = 0xFFFFFFFFu;

struct FindConst {
  float max_t, sin2, s_seed, s_fwd;
  int max_skip;
  float win_doublet;  // pseudo-angle half width of the seed doublet search
  float rho_seed, rho_fwd;  // upper bounds of sqrt(s_seed), sqrt(s_fwd)
};

template <typename IDX>
struct LayerTab {
  float* hx;        // [cap] by local index (= rank of the hit's key in its plane)
  float* hy;
  IDX* bl;          // [cap] local indices in bucket order
  uint8_t* used;    // [cap] by local index
  uint32_t* best;   // [cap] by local index: candidate holding the hit in a round
  uint32_t* bstart; // [B+1]
  uint32_t* bcur;   // [B]
};

struct TrackTab {
  uint32_t* slot;   // output slot
  uint32_t* key0;   // first hit: plane << 22 | local index (orders like its key)
  float* xa;        // last hit
  float* ya;
  float* tx;        // slope through the last two hits
  float* ty;
  uint8_t* la;      // plane of the last hit
  uint8_t* n;       // hits so far
  uint8_t* skip;    // planes missed in a row
  uint32_t* tbest;  // per round: best candidate of the track
  uint32_t* tmatch; // local index of the hit taken at this plane
};

struct Cand {
  float s;
  uint32_t a, b, c;  // extension: track, hit; seed: h0, h1, h2 (local indices)
};

template <typename IDX>
struct FindMem {
  LayerTab<IDX> L[3];
  TrackTab T;
  Cand* cand;
  uint32_t capL, capT, capC, nb;  // capacities, number of azimuth buckets
};

// Monotone pseudo-angle of (x, y) in [0, 4]; its derivative with respect to
// the azimuth is between 1/2 and 1, so an azimuth window of half width d is
// contained in the pseudo-angle window of the same half width.
__device__ __forceinline__ float pangle(float x, float y) {
  float ax = fabsf(x), ay = fabsf(y), d = ax + ay;
  float r = d > 0.0f ? ay / d : 0.0f;
  if (y >= 0.0f) return x >= 0.0f ? r : 2.0f - r;
  return x < 0.0f ? 2.0f + r : 4.0f - r;
}

__device__ __forceinline__ uint32_t bucket_of(float pa, uint32_t nb) {
  int b = (int)(pa * (float)nb * 0.25f);
  return b < 0 ? 0u : (b >= (int)nb ? nb - 1 : (uint32_t)b);
}

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

// pseudo-angle half width for hits within rho of the point (x, y)
__device__ __forceinline__ float point_window(float x, float y, float rho) {
  float R2 = x * x + y * y;
  float rr = 2.25f * rho * rho;  // R <= 1.5 rho: whole plane
  if (R2 <= rr) return 4.0f;
  float u2 = (rho * rho) / R2;   // sin^2 of the largest angle
  return sqrtf(u2 / (1.0f - u2)) * 1.001f + 1e-3f;
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

struct EventIO {
  const float* X;          // hits of the event (absolute base applied)
  const float* Y;
  const uint32_t* lstart;  // [27]
  const uint32_t* lnh;     // [26]
  uint8_t* nhits;          // track outputs at the event's slot base
  uint32_t* hit_idx;
  uint64_t slot_base;
};

// shared scalars of one event
struct FindScal {
  uint32_t nc;       // candidates found this step (may exceed capC)
  uint32_t flag;     // any live candidate left
  uint32_t n_act;    // active tracks
  uint32_t n_created;
  uint32_t fail;     // 0 ok, 1 escalate, 2 overflow
  uint32_t tmp[8];   // scan scratch (NT/64 + 1)
};

// Load plane l into ring table `t`: coordinates, bucket counting sort.
template <int NT, typename IDX>
__device__ void load_plane(const EventIO& io, int l, LayerTab<IDX>& t, uint32_t nb, FindScal& sc) {
  const uint32_t n = io.lnh[l], base = io.lstart[l];
  for (uint32_t b = threadIdx.x; b < nb; b += NT) t.bcur[b] = 0;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += NT) {
    float x = io.X[base + i], y = io.Y[base + i];
    t.hx[i] = x;
    t.hy[i] = y;
    t.used[i] = 0;
    uint32_t b = bucket_of(pangle(x, y), nb);
    t.best[i] = b;
    atomicAdd(t.bcur + b, 1u);
  }
  __syncthreads();
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < nb; b0 += NT) {
    uint32_t b = b0 + threadIdx.x;
    uint32_t c = b < nb ? lda(t.bcur + b) : 0u;
    uint32_t tot;
    uint32_t ex = block_scan<NT>(c, sc.tmp, &tot);
    __syncthreads();
    if (b < nb) { t.bstart[b] = carry + ex; t.bcur[b] = carry + ex; }
    carry += tot;
  }
  if (threadIdx.x == 0) t.bstart[nb] = carry;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += NT) {
    uint32_t b = t.best[i];
    uint32_t pos = atomicAdd(t.bcur + b, 1u);
    t.bl[pos] = (IDX)i;
  }
  __syncthreads();
}

template <typename IDX, typename F>
__device__ __forceinline__ void scan_window(const LayerTab<IDX>& t, Ranges r, F f) {
  for (uint32_t p = t.bstart[r.b0], e = t.bstart[r.b1 + 1]; p < e; ++p) f((uint32_t)t.bl[p]);
  if (r.b2 <= r.b3)
    for (uint32_t p = t.bstart[r.b2], e = t.bstart[r.b3 + 1]; p < e; ++p) f((uint32_t)t.bl[p]);
}

// Returns 0 when done, 1 when the event needs a larger tier, 2 on overflow.
template <int NT, typename IDX>
__device__ uint32_t find_event(const EventIO& io, const FindConst& P, FindMem<IDX>& M, FindScal& sc) {
  const uint32_t tid = threadIdx.x;
  for (int l = 0; l < kLayers; ++l)
    if (io.lnh[l] > M.capL) return 1u;
  if (tid == 0) { sc.n_act = 0; sc.n_created = 0; sc.fail = 0; }
  __syncthreads();
  TrackTab& A = M.T;
  for (int l = kLayers - 1; l >= 0; --l) {
    LayerTab<IDX>& T0 = M.L[l % 3];
    load_plane<NT>(io, l, T0, M.nb, sc);
    const uint32_t n0 = io.lnh[l], base0 = io.lstart[l];
    const float zl = kLayerZ[l];
    const uint32_t n_act = sc.n_act;

    // ---- 1. extend active tracks into plane l ----
    if (tid == 0) sc.nc = 0;
    for (uint32_t t = tid; t < n_act; t += NT) { A.tmatch[t] = kNone; }
    __syncthreads();
    for (uint32_t t = tid; t < n_act; t += NT) {
      const float xa = A.xa[t], ya = A.ya[t], txf = A.tx[t], tyf = A.ty[t];
      const float za = kLayerZ[A.la[t]];
      const float d = zl - za;
      const float xp = xa + txf * d;
      const float yp = ya + tyf * d;
      Ranges r = window(pangle(xp, yp), point_window(xp, yp, P.rho_fwd), M.nb);
      scan_window(T0, r, [&](uint32_t h) {
        float dx = T0.hx[h] - xp, dy = T0.hy[h] - yp;
        float s = dx * dx + dy * dy;
        if (s <= P.s_fwd) {
          uint32_t k = atomicAdd(&sc.nc, 1u);
          if (k < M.capC) M.cand[k] = Cand{s, t, h, 0u};
        }
      });
    }
    __syncthreads();
    {
      const uint32_t nc = sc.nc;
      if (nc > VELO_MAX_CANDIDATES) return 2u;
      if (nc > M.capC) return 1u;
      // greedy matching by (s, first-hit key of the track, hit key)
      auto less_hit = [&](uint32_t i, uint32_t j) {
        const Cand ci = M.cand[i], cj = M.cand[j];
        if (ci.s != cj.s) return ci.s < cj.s;
        return A.key0[ci.a] < A.key0[cj.a];
      };
      auto less_trk = [&](uint32_t i, uint32_t j) {
        const Cand ci = M.cand[i], cj = M.cand[j];
        if (ci.s != cj.s) return ci.s < cj.s;
        return ci.b < cj.b;
      };
      // every round accepts the smallest live candidate, so nc rounds suffice
      for (uint32_t round = 0; round < nc; ++round) {
        for (uint32_t h = tid; h < n0; h += NT) T0.best[h] = kNone;
        for (uint32_t t = tid; t < n_act; t += NT) A.tbest[t] = kNone;
        if (tid == 0) sc.flag = 0;
        __syncthreads();
        for (uint32_t k = tid; k < nc; k += NT) {
          const Cand c = M.cand[k];
          if (A.tmatch[c.a] == kNone && !T0.used[c.b]) {
            cas_min(T0.best + c.b, k, less_hit);
            cas_min(A.tbest + c.a, k, less_trk);
          }
        }
        __syncthreads();
        for (uint32_t k = tid; k < nc; k += NT) {
          const Cand c = M.cand[k];
          if (A.tmatch[c.a] == kNone && !T0.used[c.b] && lda(T0.best + c.b) == k &&
              lda(A.tbest + c.a) == k) {
            A.tmatch[c.a] = c.b;
            T0.used[c.b] = 1;
          }
        }
        __syncthreads();
        bool live = false;
        for (uint32_t k = tid; k < nc; k += NT) {
          const Cand c = M.cand[k];
          if (A.tmatch[c.a] == kNone && !T0.used[c.b]) live = true;
        }
        if (live) sc.flag = 1;
        __syncthreads();
        if (!sc.flag) break;
        __syncthreads();
      }
    }
    // apply: append matched hits, count misses
    for (uint32_t t = tid; t < n_act; t += NT) {
      const uint32_t h = A.tmatch[t];
      if (h != kNone) {
        const uint32_t nn = A.n[t];
        io.hit_idx[26ull * A.slot[t] + nn] = base0 + h;
        const float xh = T0.hx[h], yh = T0.hy[h];
        const float dz = zl - kLayerZ[A.la[t]];
        A.tx[t] = (xh - A.xa[t]) / dz;
        A.ty[t] = (yh - A.ya[t]) / dz;
        A.xa[t] = xh;
        A.ya[t] = yh;
        A.la[t] = (uint8_t)l;
        A.n[t] = (uint8_t)(nn + 1);
        A.skip[t] = 0;
      } else {
        const int sk = A.skip[t] + 1;
        A.skip[t] = (uint8_t)sk;
        if (sk > P.max_skip) io.nhits[A.slot[t]] = A.n[t];
      }
    }
    __syncthreads();

    // ---- 2. seeds on planes (l+2, l+1, l) ----
    uint32_t n_new = 0;
    LayerTab<IDX>& T1 = M.L[(l + 1) % 3];
    LayerTab<IDX>& T2 = M.L[(l + 2) % 3];
    uint32_t n1 = 0, n2 = 0;
    if (l <= kLayers - 3) {
      n1 = io.lnh[l + 1];
      n2 = io.lnh[l + 2];
      const float z0 = kLayerZ[l + 2], z1 = kLayerZ[l + 1], z2 = zl;
      if (tid == 0) sc.nc = 0;
      __syncthreads();
      for (uint32_t i1 = tid; i1 < n1; i1 += NT) {
        if (T1.used[i1]) continue;
        const float x1 = T1.hx[i1], y1 = T1.hy[i1];
        Ranges r0 = window(pangle(x1, y1), P.win_doublet, M.nb);
        scan_window(T2, r0, [&](uint32_t i0) {
          if (T2.used[i0]) return;
          const float x0 = T2.hx[i0], y0 = T2.hy[i0];
          const float dz = z1 - z0;
          const float tx = (x1 - x0) / dz;
          const float ty = (y1 - y0) / dz;
          if (!(fabsf(tx) <= P.max_t && fabsf(ty) <= P.max_t)) return;
          const float cr = x0 * y1 - y0 * x1;
          const float r0s = x0 * x0 + y0 * y0;
          const float r1s = x1 * x1 + y1 * y1;
          if (!(cr * cr <= (P.sin2 * r0s) * r1s)) return;
          if (!(x0 * x1 + y0 * y1 > 0.0f)) return;
          const float d = z2 - z1;
          const float xp = x1 + tx * d;
          const float yp = y1 + ty * d;
          Ranges r2 = window(pangle(xp, yp), point_window(xp, yp, P.rho_seed), M.nb);
          scan_window(T0, r2, [&](uint32_t i2) {
            if (T0.used[i2]) return;
            const float dx = T0.hx[i2] - xp, dy = T0.hy[i2] - yp;
            const float s = dx * dx + dy * dy;
            if (s <= P.s_seed) {
              uint32_t k = atomicAdd(&sc.nc, 1u);
              if (k < M.capC) M.cand[k] = Cand{s, i0, i1, i2};
            }
          });
        });
      }
      __syncthreads();
      const uint32_t nc = sc.nc;
      if (nc > VELO_MAX_CANDIDATES) return 2u;
      if (nc > M.capC) return 1u;
      // greedy independent set by (s, key1, key0, key2)
      auto less_seed = [&](uint32_t i, uint32_t j) {
        const Cand ci = M.cand[i], cj = M.cand[j];
        if (ci.s != cj.s) return ci.s < cj.s;
        if (ci.b != cj.b) return ci.b < cj.b;
        if (ci.a != cj.a) return ci.a < cj.a;
        return ci.c < cj.c;
      };
      auto alive = [&](const Cand& c) { return !T2.used[c.a] && !T1.used[c.b] && !T0.used[c.c]; };
      for (uint32_t round = 0; round < nc; ++round) {
        for (uint32_t h = tid; h < n2; h += NT) T2.best[h] = kNone;
        for (uint32_t h = tid; h < n1; h += NT) T1.best[h] = kNone;
        for (uint32_t h = tid; h < n0; h += NT) T0.best[h] = kNone;
        if (tid == 0) sc.flag = 0;
        __syncthreads();
        for (uint32_t k = tid; k < nc; k += NT) {
          const Cand c = M.cand[k];
          if (alive(c)) {
            cas_min(T2.best + c.a, k, less_seed);
            cas_min(T1.best + c.b, k, less_seed);
            cas_min(T0.best + c.c, k, less_seed);
          }
        }
        __syncthreads();
        for (uint32_t k = tid; k < nc; k += NT) {
          const Cand c = M.cand[k];
          if (alive(c) && lda(T2.best + c.a) == k && lda(T1.best + c.b) == k &&
              lda(T0.best + c.c) == k) {
            T2.used[c.a] = 1;
            T1.used[c.b] = 1;
            T0.used[c.c] = 1;
            M.cand[k].s = -1.0f;  // accepted (every real s is >= 0)
          }
        }
        __syncthreads();
        bool live = false;
        for (uint32_t k = tid; k < nc; k += NT)
          if (alive(M.cand[k])) live = true;
        if (live) sc.flag = 1;
        __syncthreads();
        if (!sc.flag) break;
        __syncthreads();
      }
      // accepted seed of each h0 (its candidate index)
      for (uint32_t h = tid; h < n2; h += NT) T2.best[h] = kNone;
      __syncthreads();
      for (uint32_t k = tid; k < nc; k += NT)
        if (M.cand[k].s < 0.0f) T2.best[M.cand[k].a] = k;
      __syncthreads();
    }

    // ---- 3. active table: surviving tracks compacted in place, then new seeds ----
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < n_act; b0 += NT) {
      const uint32_t t = b0 + tid;
      const bool keep = t < n_act && (int)A.skip[t] <= P.max_skip;
      uint32_t f_slot = 0, f_key0 = 0;
      float f_xa = 0, f_ya = 0, f_tx = 0, f_ty = 0;
      uint8_t f_la = 0, f_n = 0, f_skip = 0;
      if (keep) {
        f_slot = A.slot[t]; f_key0 = A.key0[t]; f_xa = A.xa[t]; f_ya = A.ya[t];
        f_tx = A.tx[t]; f_ty = A.ty[t]; f_la = A.la[t]; f_n = A.n[t]; f_skip = A.skip[t];
      }
      uint32_t tot;
      const uint32_t pos = carry + block_scan<NT>(keep ? 1u : 0u, sc.tmp, &tot);
      __syncthreads();  // every entry of this chunk is read before any is overwritten
      if (keep) {
        A.slot[pos] = f_slot; A.key0[pos] = f_key0; A.xa[pos] = f_xa; A.ya[pos] = f_ya;
        A.tx[pos] = f_tx; A.ty[pos] = f_ty; A.la[pos] = f_la; A.n[pos] = f_n; A.skip[pos] = f_skip;
      }
      carry += tot;
      __syncthreads();
    }
    const uint32_t n_keep = carry;
    if (l <= kLayers - 3) {
      // seeds in decreasing key of h0 (decreasing local index on plane l+2)
      const uint32_t created = sc.n_created;
      uint32_t c2 = 0;
      for (uint32_t b0 = 0; b0 < n2; b0 += NT) {
        const uint32_t i0 = b0 + tid < n2 ? n2 - 1 - (b0 + tid) : kNone;
        const uint32_t k = i0 != kNone ? lda(T2.best + i0) : kNone;
        uint32_t tot;
        const uint32_t rank = c2 + block_scan<NT>(k != kNone ? 1u : 0u, sc.tmp, &tot);
        if (k != kNone) {
          const Cand c = M.cand[k];
          const uint32_t slot = (uint32_t)io.slot_base + created + rank;
          uint32_t* hi = io.hit_idx + 26ull * slot;
          hi[0] = io.lstart[l + 2] + c.a;
          hi[1] = io.lstart[l + 1] + c.b;
          hi[2] = base0 + c.c;
          const uint32_t pos = n_keep + rank;
          if (pos < M.capT) {
            const float x1 = T1.hx[c.b], y1 = T1.hy[c.b], x2 = T0.hx[c.c], y2 = T0.hy[c.c];
            const float dz = zl - kLayerZ[l + 1];
            A.slot[pos] = slot;
            A.key0[pos] = ((uint32_t)(l + 2) << 22) | c.a;
            A.xa[pos] = x2;
            A.ya[pos] = y2;
            A.tx[pos] = (x2 - x1) / dz;
            A.ty[pos] = (y2 - y1) / dz;
            A.la[pos] = (uint8_t)l;
            A.n[pos] = 3;
            A.skip[pos] = 0;
          }
        }
        c2 += tot;
      }
      n_new = c2;
    }
    if (n_keep + n_new > M.capT) return 1u;
    if (tid == 0) { sc.n_act = n_keep + n_new; sc.n_created += n_new; }
    __syncthreads();
  }
  // close the tracks still active after the first plane
  for (uint32_t t = tid; t < sc.n_act; t += NT) io.nhits[A.slot[t]] = A.n[t];
  __syncthreads();
  return 0u;
}

// ---------------------------------------------------------------------------

struct FindArgs {
  const float* X;  // hit arrays (absolute slots)
  const float* Y;
  const uint32_t* hstatus;
  const uint32_t* lstart;
  const uint32_t* lnh;
  const uint64_t* offsets;
  uint64_t n_pixels;
  uint32_t* n_tracks;
  uint8_t* nhits;
  uint32_t* hit_idx;
  uint32_t* tstatus;
  uint32_t* esc_count;  // events handed to the next tier
  uint32_t* esc_list;
};

// Run one event in the given tier.  Returns true if it must go to the next.
template <int NT, typename IDX>
__device__ bool run_event(const FindArgs& a, const FindConst& P, FindMem<IDX>& M, FindScal& sc,
                          uint32_t e) {
  const uint64_t b = a.offsets[e];
  if (a.hstatus[e] != 0 || a.offsets[e + 1] <= b || a.offsets[e + 1] > a.n_pixels) {
    if (threadIdx.x == 0) { a.n_tracks[e] = 0; a.tstatus[e] = 0; }
    return false;
  }
  EventIO io{a.X + b, a.Y + b, a.lstart + 27ull * e, a.lnh + 26ull * e, a.nhits, a.hit_idx, b / 3};
  const uint32_t r = find_event<NT>(io, P, M, sc);
  if (r == 1u) return true;
  if (threadIdx.x == 0) {
    a.n_tracks[e] = r == 0u ? sc.n_created : 0u;
    a.tstatus[e] = r == 0u ? 0u : (uint32_t)VELO_EV_OVERFLOW;
  }
  return false;
}

// LDS tier: one event per workgroup (list == nullptr) or a persistent loop
// over a list of events.
template <int NT, uint32_t CAPL, uint32_t CAPT, uint32_t CAPC, uint32_t NB>
__global__ __launch_bounds__(NT) void k_find_lds(FindArgs a, FindConst P, uint32_t n_events,
                                                 const uint32_t* __restrict__ list,
                                                 const uint32_t* __restrict__ list_count) {
  __shared__ float s_hx[3][CAPL], s_hy[3][CAPL];
  __shared__ uint16_t s_bl[3][CAPL];
  __shared__ uint8_t s_used[3][CAPL];
  __shared__ uint32_t s_best[3][CAPL];
  __shared__ uint32_t s_bstart[3][NB + 1], s_bcur[3][NB];
  __shared__ uint32_t t_slot[CAPT], t_key0[CAPT], t_tbest[CAPT], t_tmatch[CAPT];
  __shared__ float t_xa[CAPT], t_ya[CAPT], t_tx[CAPT], t_ty[CAPT];
  __shared__ uint8_t t_la[CAPT], t_n[CAPT], t_skip[CAPT];
  __shared__ Cand s_cand[CAPC];
  __shared__ FindScal sc;
  FindMem<uint16_t> M;
  for (int i = 0; i < 3; ++i)
    M.L[i] = LayerTab<uint16_t>{s_hx[i], s_hy[i], s_bl[i], s_used[i], s_best[i], s_bstart[i], s_bcur[i]};
  M.T = TrackTab{t_slot, t_key0, t_xa, t_ya, t_tx, t_ty, t_la, t_n, t_skip, t_tbest, t_tmatch};
  M.cand = s_cand;
  M.capL = CAPL; M.capT = CAPT; M.capC = CAPC; M.nb = NB;
  const uint32_t count = list ? *list_count : n_events;
  for (uint32_t it = blockIdx.x; it < count; it += gridDim.x) {
    const uint32_t e = list ? list[it] : it;
    if (run_event<NT>(a, P, M, sc, e) && threadIdx.x == 0) a.esc_list[atomicAdd(a.esc_count, 1u)] = e;
    __syncthreads();
  }
}

// Workspace tier: tables in global memory, any event size.
constexpr int kGThreads = 256;
constexpr uint32_t kGBuckets = 1024;
constexpr uint32_t kGBlocks = 64;

struct GlobalTabs {
  float* hx; float* hy; uint32_t* bl; uint32_t* best; uint8_t* used;  // [3 * n_pixels]
  uint32_t* slot; uint32_t* key0; uint32_t* tbest; uint32_t* tmatch;  // [n_pixels / 3 + 1]
  float* xa; float* ya; float* tx; float* ty;
  uint8_t* la; uint8_t* n; uint8_t* skip;
  uint32_t* buckets;  // per block: 3 * (2 * kGBuckets + 1)
  Cand* cand;         // per block: VELO_MAX_CANDIDATES
};

__global__ __launch_bounds__(kGThreads) void k_find_global(FindArgs a, FindConst P, GlobalTabs g,
                                                           const uint32_t* __restrict__ list,
                                                           const uint32_t* __restrict__ list_count) {
  __shared__ FindScal sc;
  const uint32_t count = *list_count;
  uint32_t* bk = g.buckets + (size_t)blockIdx.x * 3 * (2 * kGBuckets + 1);
  for (uint32_t it = blockIdx.x; it < count; it += gridDim.x) {
    const uint32_t e = list[it];
    const uint64_t b = a.offsets[e];
    const uint32_t ne = (uint32_t)(a.offsets[e + 1] - b);
    FindMem<uint32_t> M;
    for (int i = 0; i < 3; ++i) {
      const uint64_t o = 3 * b + (uint64_t)i * ne;
      uint32_t* bb = bk + i * (2 * kGBuckets + 1);
      M.L[i] = LayerTab<uint32_t>{g.hx + o, g.hy + o, g.bl + o, g.used + o, g.best + o, bb,
                                  bb + kGBuckets + 1};
    }
    const uint64_t tb = b / 3;
    M.T = TrackTab{g.slot + tb, g.key0 + tb, g.xa + tb, g.ya + tb, g.tx + tb, g.ty + tb,
                   g.la + tb, g.n + tb, g.skip + tb, g.tbest + tb, g.tmatch + tb};
    M.cand = g.cand + (size_t)blockIdx.x * VELO_MAX_CANDIDATES;
    M.capL = ne;
    M.capT = (uint32_t)((b + ne) / 3 - b / 3);
    M.capC = VELO_MAX_CANDIDATES;
    M.nb = kGBuckets;
    if (run_event<kGThreads>(a, P, M, sc, e) && threadIdx.x == 0) {
      // cannot happen: the tables hold every possible hit and track
      a.n_tracks[e] = 0;
      a.tstatus[e] = VELO_EV_OVERFLOW;
    }
    __syncthreads();
  }
}

constexpr int kSThreads = 256;
constexpr uint32_t kSCapL = 384, kSCapT = 384, kSCapC = 512, kSBuckets = 128;

static size_t up256(size_t v) { return (v + 255) & ~size_t(255); }

size_t find_workspace_bytes(uint64_t n_pixels, uint32_t n_events) {
  const uint64_t nt = n_pixels / 3 + 1;
  size_t s = up256(4) + up256(4ull * n_events);
  s += 4 * up256(4ull * 3 * n_pixels) + up256(3 * n_pixels);
  s += 8 * up256(4ull * nt) + 3 * up256(nt);
  s += up256(4ull * kGBlocks * 3 * (2 * kGBuckets + 1));
  s += up256(sizeof(Cand) * (size_t)kGBlocks * VELO_MAX_CANDIDATES);
  return s;
}

FindConst make_find_const(const velo_params* p) {
  FindConst c;
  c.max_t = p->max_t;
  c.sin2 = p->sin2_phi;
  c.s_seed = p->s_seed;
  c.s_fwd = p->s_fwd;
  c.max_skip = p->max_skip;
  const double u2 = p->sin2_phi;
  c.win_doublet = (u2 >= 0.5 || u2 < 0) ? 4.0f : (float)(sqrt(u2 / (1.0 - u2)) * 1.001 + 1e-3);
  c.rho_seed = (float)(sqrt((double)(p->s_seed > 0 ? p->s_seed : 0)) * 1.001 + 1e-6);
  c.rho_fwd = (float)(sqrt((double)(p->s_fwd > 0 ? p->s_fwd : 0)) * 1.001 + 1e-6);
  return c;
}

hipError_t launch_find(const velo_hits* h, const uint64_t* offsets, uint32_t n_events,
                       uint64_t n_pixels, const velo_params* p, const velo_tracks* t, void* ws,
                       hipStream_t s) {
  char* w = (char*)ws;
  size_t o = 0;
  auto take = [&](size_t bytes) { char* r = w + o; o += up256(bytes); return r; };
  const uint64_t nt = n_pixels / 3 + 1;
  uint32_t* esc_count = (uint32_t*)take(4);
  uint32_t* esc_list = (uint32_t*)take(4ull * n_events);
  GlobalTabs g;
  g.hx = (float*)take(4ull * 3 * n_pixels);
  g.hy = (float*)take(4ull * 3 * n_pixels);
  g.bl = (uint32_t*)take(4ull * 3 * n_pixels);
  g.best = (uint32_t*)take(4ull * 3 * n_pixels);
  g.used = (uint8_t*)take(3 * n_pixels);
  g.slot = (uint32_t*)take(4 * nt);
  g.key0 = (uint32_t*)take(4 * nt);
  g.tbest = (uint32_t*)take(4 * nt);
  g.tmatch = (uint32_t*)take(4 * nt);
  g.xa = (float*)take(4 * nt);
  g.ya = (float*)take(4 * nt);
  g.tx = (float*)take(4 * nt);
  g.ty = (float*)take(4 * nt);
  g.la = (uint8_t*)take(nt);
  g.n = (uint8_t*)take(nt);
  g.skip = (uint8_t*)take(nt);
  g.buckets = (uint32_t*)take(4ull * kGBlocks * 3 * (2 * kGBuckets + 1));
  g.cand = (Cand*)take(sizeof(Cand) * (size_t)kGBlocks * VELO_MAX_CANDIDATES);
  FindArgs a{h->x, h->y, h->status, h->layer_start, h->layer_nhits, offsets, n_pixels,
             t->n_tracks, t->nhits, t->hit_idx, t->status, esc_count, esc_list};
  const FindConst c = make_find_const(p);
  hipLaunchKernelGGL(k_clear, dim3(1), dim3(64), 0, s, esc_count, 0u, esc_count);
  hipLaunchKernelGGL((k_find_lds<kSThreads, kSCapL, kSCapT, kSCapC, kSBuckets>), dim3(n_events),
                     dim3(kSThreads), 0, s, a, c, n_events, (const uint32_t*)nullptr,
                     (const uint32_t*)nullptr);
  hipLaunchKernelGGL(k_find_global, dim3(kGBlocks), dim3(kGThreads), 0, s, a, c, g, esc_list,
                     esc_count);
  return hipGetLastError();
}

}  // namespace velo
