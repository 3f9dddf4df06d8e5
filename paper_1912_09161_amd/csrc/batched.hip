// batched.hip -- the batched form: events of very uneven occupancy in one
// launch sequence, with persistent work-stealing workgroups, the whole
// pipeline captured once as a HIP graph and replayed, and launch shapes picked
// by an autotuner that times candidates on the live batch.
//
// The paper runs its sequence with a custom scheduler and memory manager and
// one GPU stream per CPU thread (Sec. 2.2, Sec. 3.2); here the device itself
// balances the work: after validation, k_order_* counting-sort the (event,
// plane) segments and the events by size, largest first, and the persistent
// clustering and track-finding workgroups pop items from device counters in
// that order.  Every item writes its results at positions fixed by the input,
// so the outputs are identical to the plain form whatever the schedule.
#include "cluster.hip"
#include "find.hip"
#include "fit.hip"

#include <string.h>

namespace velo {

constexpr uint32_t kSegClasses = 64;   // segment size classes (16 words wide)
constexpr uint32_t kEvClasses = 256;   // event size classes (64 words wide)

struct OrderWs {
  uint32_t* counters;  // [16]: work-stealing counters (zeroed every run)
  uint32_t* seg_hist;  // [kSegClasses] then cursors
  uint32_t* ev_hist;   // [kEvClasses] then cursors
  uint32_t* seg_order; // [E * 26]
  uint32_t* ev_order;  // [E]
};

static size_t up256b(size_t v) { return (v + 255) & ~size_t(255); }

static size_t order_ws_layout(char* w, uint32_t n_events, OrderWs* out) {
  size_t o = 0;
  auto take = [&](size_t bytes) { char* r = w ? w + o : nullptr; o += up256b(bytes); return r; };
  OrderWs f;
  f.counters = (uint32_t*)take(4 * (16 + kSegClasses + kEvClasses));
  f.seg_hist = f.counters ? f.counters + 16 : nullptr;
  f.ev_hist = f.counters ? f.counters + 16 + kSegClasses : nullptr;
  f.seg_order = (uint32_t*)take(4ull * n_events * kLayers);
  f.ev_order = (uint32_t*)take(4ull * n_events);
  if (out) *out = f;
  return o;
}

__global__ void k_zero(uint32_t* __restrict__ p, uint32_t n) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

__device__ __forceinline__ uint32_t seg_class(const uint64_t* offsets, const uint32_t* status,
                                              const uint32_t* layer_start, uint64_t n_pixels,
                                              uint32_t seg) {
  const uint32_t e = seg / kLayers, l = seg % kLayers;
  if (status[e] != 0 || !event_ok(offsets, e, n_pixels)) return 0;
  const uint32_t n = layer_start[27ull * e + l + 1] - layer_start[27ull * e + l];
  const uint32_t c = n >> 4;
  return c < kSegClasses ? c : kSegClasses - 1;
}

__device__ __forceinline__ uint32_t ev_class(const uint64_t* offsets, uint64_t n_pixels, uint32_t e) {
  if (!event_ok(offsets, e, n_pixels)) return 0;
  const uint64_t c = (offsets[e + 1] - offsets[e]) >> 6;
  return c < kEvClasses ? (uint32_t)c : kEvClasses - 1;
}

constexpr int kOrderThreads = 256;
constexpr uint32_t kOrderSegs = 1u, kOrderEvents = 2u;  // which orders to build

// Items of the ordering kernels, one per lane: the (event, plane) segments
// when their order is wanted (the first segment of every event also counts
// the event), else the events.
__host__ __device__ __forceinline__ uint32_t order_items(uint32_t n_events, uint32_t mode) {
  return (mode & kOrderSegs) ? n_events * kLayers : n_events;
}

// Segment and event classes of one item (0xFFFFFFFF when it has none).
__device__ __forceinline__ void order_classes(const uint64_t* offsets, const uint32_t* status,
                                              const uint32_t* layer_start, uint32_t n_events,
                                              uint64_t n_pixels, uint32_t mode, uint32_t item,
                                              uint32_t* sc, uint32_t* ec, uint32_t* ev) {
  *sc = 0xFFFFFFFFu;
  *ec = 0xFFFFFFFFu;
  *ev = 0xFFFFFFFFu;
  if (item >= order_items(n_events, mode)) return;
  if (mode & kOrderSegs) {
    *sc = seg_class(offsets, status, layer_start, n_pixels, item);
    if ((mode & kOrderEvents) && item % kLayers == 0) *ev = item / kLayers;
  } else {
    *ev = item;
  }
  if (*ev != 0xFFFFFFFFu) *ec = ev_class(offsets, n_pixels, *ev);
}

// class sizes: LDS histograms per workgroup, one global add per non-empty bin
__global__ __launch_bounds__(kOrderThreads) void k_order_hist(
    const uint64_t* __restrict__ offsets, const uint32_t* __restrict__ status,
    const uint32_t* __restrict__ layer_start, uint32_t n_events, uint64_t n_pixels, uint32_t mode,
    OrderWs w) {
  __shared__ uint32_t sh[kSegClasses], eh[kEvClasses];
  for (uint32_t k = threadIdx.x; k < kSegClasses; k += kOrderThreads) sh[k] = 0;
  for (uint32_t k = threadIdx.x; k < kEvClasses; k += kOrderThreads) eh[k] = 0;
  __syncthreads();
  uint32_t sc, ec, ev;
  order_classes(offsets, status, layer_start, n_events, n_pixels, mode,
                blockIdx.x * kOrderThreads + threadIdx.x, &sc, &ec, &ev);
  if (sc != 0xFFFFFFFFu) atomicAdd(sh + sc, 1u);
  if (ec != 0xFFFFFFFFu) atomicAdd(eh + ec, 1u);
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < kSegClasses; k += kOrderThreads)
    if (sh[k]) atomicAdd(w.seg_hist + k, sh[k]);
  for (uint32_t k = threadIdx.x; k < kEvClasses; k += kOrderThreads)
    if (eh[k]) atomicAdd(w.ev_hist + k, eh[k]);
}

// exclusive scans in descending class order (largest items first)
__global__ __launch_bounds__(kOrderThreads) void k_order_scan(OrderWs w) {
  __shared__ uint32_t tmp[kOrderThreads / kWave + 1];
  static_assert(kEvClasses == kOrderThreads && kSegClasses <= kOrderThreads, "one class per lane");
  const uint32_t t = threadIdx.x;
  uint32_t tot;
  const uint32_t vs = t < kSegClasses ? w.seg_hist[kSegClasses - 1 - t] : 0u;
  const uint32_t xs = block_scan<kOrderThreads>(vs, tmp, &tot);
  if (t < kSegClasses) w.seg_hist[kSegClasses - 1 - t] = xs;
  const uint32_t ve = w.ev_hist[kEvClasses - 1 - t];
  const uint32_t xe = block_scan<kOrderThreads>(ve, tmp, &tot);
  w.ev_hist[kEvClasses - 1 - t] = xe;
}

// positions: every workgroup reserves one range per non-empty bin, its lanes
// take positions in it with LDS atomics (order inside a class is arbitrary)
__global__ __launch_bounds__(kOrderThreads) void k_order_scatter(
    const uint64_t* __restrict__ offsets, const uint32_t* __restrict__ status,
    const uint32_t* __restrict__ layer_start, uint32_t n_events, uint64_t n_pixels, uint32_t mode,
    OrderWs w) {
  __shared__ uint32_t sh[kSegClasses], eh[kEvClasses];
  for (uint32_t k = threadIdx.x; k < kSegClasses; k += kOrderThreads) sh[k] = 0;
  for (uint32_t k = threadIdx.x; k < kEvClasses; k += kOrderThreads) eh[k] = 0;
  __syncthreads();
  uint32_t sc, ec, ev;
  const uint32_t item = blockIdx.x * kOrderThreads + threadIdx.x;
  order_classes(offsets, status, layer_start, n_events, n_pixels, mode, item, &sc, &ec, &ev);
  uint32_t ps = 0, pe = 0;  // rank inside the workgroup's share of the class
  if (sc != 0xFFFFFFFFu) ps = atomicAdd(sh + sc, 1u);
  if (ec != 0xFFFFFFFFu) pe = atomicAdd(eh + ec, 1u);
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < kSegClasses; k += kOrderThreads)
    if (sh[k]) sh[k] = atomicAdd(w.seg_hist + k, sh[k]);
  for (uint32_t k = threadIdx.x; k < kEvClasses; k += kOrderThreads)
    if (eh[k]) eh[k] = atomicAdd(w.ev_hist + k, eh[k]);
  __syncthreads();
  if (sc != 0xFFFFFFFFu) w.seg_order[sh[sc] + ps] = item;
  if (ec != 0xFFFFFFFFu) w.ev_order[eh[ec] + pe] = ev;
}

// ---------------------------------------------------------------------------

struct BatchedCfg {
  uint32_t small_grid;   // persistent clustering workgroups (0: one per segment)
  uint32_t mid_grid;
  int find_threads;
  uint32_t find_grid;    // persistent track-finding workgroups (0: one per event)
  int fit_threads;
  uint32_t esc_grid[3];  // workgroups of the middle, large and workspace track-finding tiers
  uint32_t route_hits;   // events routed past the small track-finding tier (0: none; find_grid == 0)
  uint32_t fork;         // routed events' middle tier on the side stream, beside the small tier
  uint32_t find_order;   // find_grid == 0: workgroups take the events largest first
  uint32_t tiny;         // find_grid == 0, no routing, 256 lanes: the tiny tier ahead of the small one
};

// The side stream and the two events of a fork (side == null: no fork).
struct Fork {
  hipStream_t side;
  hipEvent_t fork_ev, join_ev;
};

size_t batched_workspace_bytes(uint64_t n_pixels, uint32_t n_events) {
  const size_t a = cluster_workspace_bytes(n_pixels, n_events);
  const size_t b = find_workspace_bytes(n_pixels, n_events);
  return (a > b ? a : b) + order_ws_layout(nullptr, n_events, nullptr);
}

struct BatchedCall {
  const uint32_t* px;
  const uint64_t* offsets;
  uint32_t n_events;
  uint64_t n_pixels;
  velo_params params;
  bool has_mlp;
  velo_mlp mlp;
  velo_hits hits;
  velo_tracks tracks;
  velo_states states;
  void* ws;
  size_t ws_bytes;
};

// ordering + the three stages with the given launch shapes
static hipError_t enqueue_batched(const BatchedCall& c, const BatchedCfg& k, hipStream_t s,
                                  const Fork& fk, int stages = 7) {
  const size_t main_ws = c.ws_bytes - order_ws_layout(nullptr, c.n_events, nullptr);
  OrderWs ow;
  order_ws_layout((char*)c.ws + main_ws, c.n_events, &ow);
  if (stages & 1) {
    // clearing (only the persistent kernels and the size orders use the
    // counters), validation, size ordering, clustering
    const uint32_t mode = (k.small_grid ? kOrderSegs : 0u) | (k.find_grid || k.find_order ? kOrderEvents : 0u);
    if (mode)
      hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, ow.counters, 16u + kSegClasses + kEvClasses);
    launch_validate(c.px, c.offsets, c.n_events, c.n_pixels, c.hits.status, c.hits.layer_start,
                    (uint32_t*)c.ws, s);
    // size orders for the persistent kernels that use them
    if (mode) {
      const uint32_t og = (order_items(c.n_events, mode) + kOrderThreads - 1) / kOrderThreads;
      hipLaunchKernelGGL(k_order_hist, dim3(og), dim3(kOrderThreads), 0, s, c.offsets, c.hits.status,
                         c.hits.layer_start, c.n_events, c.n_pixels, mode, ow);
      hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(kOrderThreads), 0, s, ow);
      hipLaunchKernelGGL(k_order_scatter, dim3(og), dim3(kOrderThreads), 0, s, c.offsets,
                         c.hits.status, c.hits.layer_start, c.n_events, c.n_pixels, mode, ow);
    }
    const ClusterCfg cc{k.small_grid, k.mid_grid, ow.seg_order, ow.counters};
    hipError_t e = launch_cluster_cfg(c.px, c.offsets, c.n_events, c.n_pixels, &c.hits, c.ws, s, cc, true);
    if (e != hipSuccess) return e;
  }
  if (stages & 2) {
    if (k.find_grid)  // work-stealing counters of the persistent track-finding tiers
      hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, ow.counters + 2, 3u);
    const bool fork = k.fork && k.route_hits && fk.side;
    const FindCfg fc{k.find_threads, k.find_grid, ow.ev_order, ow.counters + 2,
                     {k.esc_grid[0], k.esc_grid[1], k.esc_grid[2]}, k.find_grid ? 0u : k.route_hits,
                     fork ? fk.side : nullptr, fk.fork_ev, fk.join_ev, k.find_grid ? 0u : k.find_order,
                     k.find_grid || k.route_hits || k.find_threads != kSThreads ? 0u : k.tiny};
    hipError_t e = launch_find_cfg(&c.hits, c.offsets, c.n_events, c.n_pixels, &c.params, &c.tracks,
                                   c.ws, s, fc);
    if (e != hipSuccess) return e;
  }
  if (stages & 4) {
    hipError_t e = launch_fit_cfg(&c.hits, &c.tracks, c.offsets, c.n_events, c.n_pixels, &c.params,
                                  c.has_mlp ? &c.mlp : nullptr, &c.states, s, k.fit_threads);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace velo

// ---------------------------------------------------------------------------

struct velo_context {
  // classifier held by the context (velo_mlp_load): params[1377], mean[8],
  // std[8] in one device buffer, Adam moments, gradient, loss, workspace
  float* net = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* grad = nullptr;
  float* loss = nullptr;
  void* mlp_ws = nullptr;
  size_t mlp_ws_bytes = 0;
  float threshold = 0.0f;
  velo_params params{};  // used when a call passes no parameters
  bool tuned = false;
  int source = 0;  // how cfg was chosen: 1 tuned here, 2 tune cache, 3 set by the caller
  velo::BatchedCfg cfg{2048, 512, 256, 1024, 128, {velo::kMBlocks, velo::kLBlocks, velo::kGBlocks}, 0, 0, 0, 0};
  // side stream and events of the forked track-finding tier, made with the
  // context on side_dev (calls on another device run unforked)
  velo::Fork fork{nullptr, nullptr, nullptr};
  int side_dev = -1;
  float tuned_ms[5] = {0, 0, 0, 0, 0};
  // captured graphs of recent call shapes (buffers, sizes, parameters, stream)
  static constexpr int kGraphs = 32;
  struct Entry {
    velo::BatchedCall key;
    hipStream_t stream;
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint64_t last_use;
  };
  Entry graphs[kGraphs];
  int n_graphs = 0;
  uint64_t clock = 0;
};

namespace {

bool same_call(const velo::BatchedCall& a, const velo::BatchedCall& b) {
  return memcmp(&a, &b, sizeof(velo::BatchedCall)) == 0;
}

void drop_entry(velo_context::Entry& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g.exec = nullptr;
  g.graph = nullptr;
}

void drop_graphs(velo_context* ctx) {
  for (int i = 0; i < ctx->n_graphs; ++i) drop_entry(ctx->graphs[i]);
  ctx->n_graphs = 0;
}

// time one stage (min of `reps` runs) with events on the stream
hipError_t time_stage(const velo::BatchedCall& c, const velo::BatchedCfg& k, const velo::Fork& fk, int stage,
                      hipStream_t s, int reps, float* ms) {
  hipEvent_t a, b;
  hipError_t e = hipEventCreate(&a);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&b);
  if (e != hipSuccess) { (void)hipEventDestroy(a); return e; }
  float best = 1e30f;
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    e = hipEventRecord(a, s);
    if (e == hipSuccess) e = velo::enqueue_batched(c, k, s, fk, stage);
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (t < best) best = t;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = best;
  return e;
}

}  // namespace

namespace velo {

// A persistent grid is taken only if it beats one workgroup per item by this
// factor on the tuning stream.  The tuner times one stream, while callers
// often keep several streams busy; there one workgroup per item interleaves
// with the other streams' kernels, whereas a persistent grid holds its slots
// until its queue drains, so a small latency gain alone does not carry over.
constexpr float kPersistentGain = 0.85f;
// Track finding (compared with the best per-event configuration, its options
// included): at high occupancy a persistent grid was 16 % faster on the
// tuning stream and 5 % faster under two streams; at nominal occupancy 1 %
// faster on one stream and 4 % slower under twelve.
constexpr float kPersistentGainFind = 0.90f;

// Pick the launch shapes stage by stage on the live batch: clustering first
// (its output feeds the next stage), then track finding, then the fit.
static hipError_t autotune(velo_context* ctx, const BatchedCall& c, hipStream_t s, const Fork& fk) {
  BatchedCfg best = ctx->cfg;
  best.find_order = 1;  // the clustering stage builds the event order the track-finding candidates use
  float t;
  hipError_t e;
  // clustering: one workgroup per segment, or persistent grids of several
  // sizes; then the smallest large-segment grid within 2 % of the chosen
  // time (like the track-finding tiers below, a persistent launch with LDS-
  // heavy workgroups holds its reservations until every workgroup is placed)
  {
    const uint32_t smalls[] = {0, 1024, 2048, 4096, 8192};
    constexpr int kNM = 4;
    const uint32_t mids[kNM] = {1024, 512, 256, 64};
    float bt[2] = {1e30f, 1e30f};  // one workgroup per segment, persistent
    float tm[5][kNM];
    BatchedCfg k = best, pick[2] = {best, best};
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < kNM; ++j) {
        k.small_grid = smalls[i];
        k.mid_grid = mids[j];
        if ((e = time_stage(c, k, fk, 1, s, 3, &t)) != hipSuccess) return e;
        tm[i][j] = t;
        const int p = smalls[i] != 0;
        if (t < bt[p]) { bt[p] = t; pick[p] = k; }
      }
    const int p = bt[1] < kPersistentGain * bt[0];
    best.small_grid = pick[p].small_grid;
    best.mid_grid = pick[p].mid_grid;
    for (int i = 0; i < 5; ++i)
      if (smalls[i] == best.small_grid)
        for (int j = 0; j < kNM; ++j)
          if (tm[i][j] <= 1.02f * bt[p]) best.mid_grid = mids[j];
    ctx->tuned_ms[0] = bt[p];
    ctx->tuned_ms[3] = bt[0];
    if ((e = enqueue_batched(c, best, s, fk, 1)) != hipSuccess) return e;
  }
  // track finding: lanes per event x (one workgroup per event | persistent
  // grid), each side then with its hand-over tier grids (and, one workgroup
  // per event, its options); the persistent side is taken only if it beats
  // the best per-event configuration by kPersistentGainFind
  {
    best.find_order = 0;
    const int threads[] = {128, 256};
    const uint32_t grids[] = {0, 512, 768, 1024, 1536};
    float bt[2] = {1e30f, 1e30f};  // one workgroup per event, persistent
    BatchedCfg k = best, pick[2] = {best, best};
    for (int nt : threads)
      for (uint32_t g : grids) {
        k.find_threads = nt;
        k.find_grid = g;
        if ((e = time_stage(c, k, fk, 2, s, 3, &t)) != hipSuccess) return e;
        const int p = g != 0;
        if (t < bt[p]) { bt[p] = t; pick[p] = k; }
      }
    ctx->tuned_ms[4] = bt[0];
    // workgroups of the tiers that take the events the first tier hands on:
    // the smallest grids within 2 % of the best time on the tuning stream
    // (a tier's launch keeps its grid's LDS reserved until every workgroup
    // has been placed, which delays other streams' work when only a few
    // events escalate)
    const uint32_t esc[3][3] = {{kMBlocks, kLBlocks, kGBlocks}, {64, 32, 32}, {16, 8, 8}};
    int pe[2] = {0, 0};
    for (int p = 0; p < 2; ++p) {
      float et[3];
      BatchedCfg k2 = pick[p];
      for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) k2.esc_grid[j] = esc[i][j];
        if ((e = time_stage(c, k2, fk, 2, s, 3, &et[i])) != hipSuccess) return e;
      }
      float tb = et[0];
      for (int i = 1; i < 3; ++i) tb = et[i] < tb ? et[i] : tb;
      for (int i = 0; i < 3; ++i)
        if (et[i] <= 1.02f * tb) pe[p] = i;
      for (int j = 0; j < 3; ++j) pick[p].esc_grid[j] = esc[pe[p]][j];
      bt[p] = tb;
    }
    // One workgroup per event: the tiny tier ahead of the small one (six
    // workgroups per CU for the events within its capacities; the others are
    // handed on at once or after part of their work), and, for batches that
    // fill the GPU on their own (at least 8192 events; a smaller batch
    // starts all its events at once, and beside other streams the extra
    // kernels and launches cost more than they save): the events largest
    // first (a shorter tail), and routing: events with a plane above the small
    // tier's capacity go straight to the middle tier, which, with a fork, runs
    // beside the small tier.  Taken only when they beat the plain sequence by
    // 1 % on the tuning stream.  The tier grids are tried again at full size,
    // which the routed events may need.
    {
      constexpr int kNR = 7;
      const uint32_t ro[kNR][4] = {// tiny, order, route, fork
                                   {1, 0, 0, 0}, {1, 1, 0, 0}, {0, 1, 0, 0}, {0, 0, 0xFFFFFFFFu, 0},
                                   {0, 1, 0xFFFFFFFFu, 0}, {0, 0, 0xFFFFFFFFu, 1}, {0, 1, 0xFFFFFFFFu, 1}};
      const bool big = c.n_events >= 8192, can_fork = fk.side != nullptr;
      float rbest = bt[0];
      BatchedCfg k3 = pick[0], rpick = pick[0];
      for (int i = 0; i < kNR; ++i) {
        if (ro[i][0] && pick[0].find_threads != kSThreads) continue;
        if ((ro[i][1] || ro[i][2]) && !big) continue;
        if (ro[i][3] && !can_fork) continue;
        for (int g = 0; g < (pe[0] == 0 ? 1 : 2); ++g) {
          k3.tiny = ro[i][0];
          k3.find_order = ro[i][1];
          k3.route_hits = ro[i][2];
          k3.fork = ro[i][3];
          for (int j = 0; j < 3; ++j) k3.esc_grid[j] = esc[g == 0 ? pe[0] : 0][j];
          if ((e = time_stage(c, k3, fk, 2, s, 3, &t)) != hipSuccess) return e;
          if (t < rbest) { rbest = t; rpick = k3; }
        }
      }
      if (rbest < 0.99f * bt[0]) {
        pick[0] = rpick;
        bt[0] = rbest;
      }
    }
    const int p = bt[1] < kPersistentGainFind * bt[0];
    best.find_threads = pick[p].find_threads;
    best.find_grid = pick[p].find_grid;
    for (int j = 0; j < 3; ++j) best.esc_grid[j] = pick[p].esc_grid[j];
    best.tiny = pick[p].tiny;
    best.find_order = pick[p].find_order;
    best.route_hits = pick[p].route_hits;
    best.fork = pick[p].fork;
    ctx->tuned_ms[1] = bt[p];
    if ((e = enqueue_batched(c, best, s, fk, 2)) != hipSuccess) return e;
  }
  // fit: lanes per event
  {
    const int threads[] = {64, 128, 256};
    float bt = 1e30f;
    BatchedCfg k = best;
    for (int nt : threads) {
      k.fit_threads = nt;
      if ((e = time_stage(c, k, fk, 4, s, 3, &t)) != hipSuccess) return e;
      if (t < bt) { bt = t; best.fit_threads = nt; }
    }
    ctx->tuned_ms[2] = bt;
  }
  ctx->cfg = best;
  ctx->tuned = true;
  return hipStreamSynchronize(s);
}

}  // namespace velo

