// velo_capi.hip -- the C ABI of libvelo.so (declared in include/velo.h):
// argument checks, workspace carving and the ordered launch of the kernels.
// Built as one translation unit with the kernels it launches.
#include "batched.hip"
#include "pv.hip"
#include "ut.hip"
#include "pipeline.hip"

#include <math.h>
#include <string.h>

#include <mutex>

namespace velo {

// OR of the status words of one or two per-event arrays (one workgroup)
__global__ __launch_bounds__(1024) void k_status_or(const uint32_t* __restrict__ a,
                                                    const uint32_t* __restrict__ b, uint32_t n,
                                                    uint32_t* __restrict__ out) {
  __shared__ uint32_t acc;
  if (threadIdx.x == 0) acc = 0;
  __syncthreads();
  uint32_t v = 0;
  for (uint32_t i = threadIdx.x; i < n; i += 1024) v |= (a ? a[i] : 0u) | (b ? b[i] : 0u);
  if (v) atomicOr(&acc, v);
  __syncthreads();
  if (threadIdx.x == 0) *out = acc;
}

}  // namespace velo

namespace {

velo_status hip_status(hipError_t e) { return e == hipSuccess ? VELO_OK : VELO_ERR_HIP; }

bool hits_ok(const velo_hits* h) {
  return h && h->x && h->y && h->key && h->aux && h->layer_start && h->layer_nhits && h->n_hits &&
         h->status;
}
bool tracks_ok(const velo_tracks* t) { return t && t->n_tracks && t->nhits && t->hit_idx && t->status; }
bool states_ok(const velo_states* s) {
  return s && s->x && s->y && s->z && s->tx && s->ty && s->cov_x && s->cov_y && s->chi2 && s->ndof &&
         s->accepted;
}
// the caller's statement of the detector model equals the built-in one
bool geometry_ok(const velo_geometry* g) {
  if (!g || g->n_layers != VELO_N_LAYERS || g->n_cols != 1536 || g->n_rows != 1536 ||
      g->pitch_mm != 0.055f || g->hole_r_mm != 5.1f)
    return false;
  for (int l = 0; l < VELO_N_LAYERS; ++l)
    if (__builtin_bit_cast(uint32_t, g->z_mm[l]) !=
        __builtin_bit_cast(uint32_t, (float)(-280.0 + 1030.0 * (double)l / 25.0)))
      return false;
  return true;
}

bool mlp_ok(const velo_mlp* m) { return m && m->params && m->mean && m->std && isfinite(m->threshold); }
bool params_ok(const velo_params* p) {
  return p && p->max_skip >= 0 && p->max_skip < 26 && p->pt0_mev > 0.0f && p->sigma_meas > 0.0f &&
         isfinite(p->max_t) && isfinite(p->sin2_phi) && isfinite(p->s_seed) && isfinite(p->s_fwd) &&
         isfinite(p->x_over_x0) && p->x_over_x0 >= 0.0f;
}

// Process-wide cache of tuned launch shapes, so that a new context meets a
// workload class it has seen before without timing candidates again.  Key:
// the device's architecture name, the event count and the mean words per
// event (both in quarter-octave classes), the classifier flag and the cut
// parameters.  Up to kTuneCache entries, the oldest replaced first.
struct TuneKey {
  char arch[64];
  int32_t ev_class, px_class, mlp;
  velo_params params;
};
struct TuneEntry {
  TuneKey key;
  velo::BatchedCfg cfg;
  float ms[5];
};
constexpr int kTuneCache = 64;
TuneEntry g_tune[kTuneCache];
int g_tune_n = 0, g_tune_next = 0;
std::mutex g_tune_mu;

int32_t quarter_octave(double v) { return v < 1.0 ? -1 : (int32_t)floor(4.0 * log2(v)); }

bool tune_key(const velo::BatchedCall& c, TuneKey* k) {
  memset(k, 0, sizeof(*k));
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
  strncpy(k->arch, prop.gcnArchName, sizeof(k->arch) - 1);
  k->ev_class = quarter_octave((double)c.n_events);
  k->px_class = quarter_octave((double)c.n_pixels / (double)c.n_events);
  k->mlp = c.has_mlp ? 1 : 0;
  k->params = c.params;
  return true;
}

bool tune_lookup(const TuneKey& k, velo::BatchedCfg* cfg, float* ms) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (int i = 0; i < g_tune_n; ++i)
    if (memcmp(&g_tune[i].key, &k, sizeof(k)) == 0) {
      *cfg = g_tune[i].cfg;
      memcpy(ms, g_tune[i].ms, sizeof(g_tune[i].ms));
      return true;
    }
  return false;
}

void tune_store(const TuneKey& k, const velo::BatchedCfg& cfg, const float* ms) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (int i = 0; i < g_tune_n; ++i)
    if (memcmp(&g_tune[i].key, &k, sizeof(k)) == 0) return;
  TuneEntry& e = g_tune[g_tune_n < kTuneCache ? g_tune_n++ : g_tune_next];
  if (g_tune_n == kTuneCache) g_tune_next = (g_tune_next + 1) % kTuneCache;
  e.key = k;
  e.cfg = cfg;
  memcpy(e.ms, ms, sizeof(e.ms));
}

// Scratch of velo_reconstruct_noalloc: the workspace of velo_reconstruct in
// a file-scope device array, so that the call allocates nothing.  Each device
// the library runs on holds its own copy until the process ends.  In host
// code the array's name is only a stand-in: the device address of each
// device's copy comes from hipGetSymbolAddress, taken once per device with
// that device current, and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[VELO_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of the current device's scratch copy (nullptr on error).
void* scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

void velo_geometry_default(velo_geometry* g) {
  if (!g) return;
  g->n_layers = VELO_N_LAYERS;
  for (int l = 0; l < VELO_N_LAYERS; ++l) g->z_mm[l] = (float)(-280.0 + 1030.0 * (double)l / 25.0);
  g->pitch_mm = 0.055f;
  g->n_cols = 1536;
  g->n_rows = 1536;
  g->hole_r_mm = 5.1f;
}

void velo_params_default(velo_params* p) {
  if (!p) return;
  p->max_t = 0.4f;
  p->sin2_phi = 9e-4f;
  p->s_seed = 0.025f;
  p->s_fwd = 0.04f;
  p->max_skip = 1;
  p->sigma_meas = 0.055f / sqrtf(12.0f);
  p->pt0_mev = 400.0f;
  p->x_over_x0 = 5.94e-4f;
  p->qc3 = 4.0f;
  p->qc4 = 10.0f;
}

size_t velo_workspace_bytes(uint64_t n_pixels, uint32_t n_events) {
  size_t a = velo::cluster_workspace_bytes(n_pixels, n_events);
  size_t b = velo::find_workspace_bytes(n_pixels, n_events);
  return a > b ? a : b;
}

velo_status velo_cluster(const uint32_t* d_pixels, const uint64_t* d_offsets, uint32_t n_events,
                         uint64_t n_pixels, const velo_geometry* geom, const velo_hits* out, void* d_ws,
                         size_t ws_bytes, hipStream_t stream) {
  if (!geometry_ok(geom)) return VELO_ERR_ARG;
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(out) || (n_pixels > 0 && !d_pixels) || !d_ws) return VELO_ERR_ARG;
  if (n_pixels >= (1ull << 32) * 3) return VELO_ERR_ARG;
  if (ws_bytes < velo::cluster_workspace_bytes(n_pixels, n_events)) return VELO_ERR_WORKSPACE;
  return hip_status(velo::launch_cluster(d_pixels, d_offsets, n_events, n_pixels, out, d_ws, stream));
}

velo_status velo_find_tracks(const velo_hits* hits, const uint64_t* d_offsets, uint32_t n_events,
                             uint64_t n_pixels, const velo_geometry* geom, const velo_params* params,
                             const velo_tracks* out, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if (!geometry_ok(geom)) return VELO_ERR_ARG;
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(out) || !params_ok(params) || !d_ws)
    return VELO_ERR_ARG;
  if (n_pixels >= (1ull << 32) * 3) return VELO_ERR_ARG;
  if (ws_bytes < velo::find_workspace_bytes(n_pixels, n_events)) return VELO_ERR_WORKSPACE;
  return hip_status(velo::launch_find(hits, d_offsets, n_events, n_pixels, params, out, d_ws, stream));
}

velo_status velo_fit(const velo_hits* hits, const velo_tracks* tracks, const uint64_t* d_offsets,
                     uint32_t n_events, uint64_t n_pixels, const velo_geometry* geom,
                     const velo_params* params, const velo_states* out, hipStream_t stream) {
  if (!geometry_ok(geom)) return VELO_ERR_ARG;
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(tracks) || !states_ok(out) || !params_ok(params))
    return VELO_ERR_ARG;
  return hip_status(velo::launch_fit(hits, tracks, d_offsets, n_events, n_pixels, params, out, stream));
}

velo_status velo_fit_momentum(const velo_hits* hits, const velo_tracks* tracks,
                              const uint64_t* d_offsets, uint32_t n_events, uint64_t n_pixels,
                              const velo_geometry* geom, const velo_params* params,
                              const float* d_p_mev, const velo_states* out, hipStream_t stream) {
  if (!geometry_ok(geom)) return VELO_ERR_ARG;
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(tracks) || !states_ok(out) || !params_ok(params) ||
      !d_p_mev)
    return VELO_ERR_ARG;
  return hip_status(velo::launch_fit_momentum(hits, tracks, d_offsets, n_events, n_pixels, params,
                                              d_p_mev, out, stream));
}

velo_status velo_reconstruct(const uint32_t* d_pixels, const uint64_t* d_offsets, uint32_t n_events,
                             uint64_t n_pixels, const velo_geometry* geom, const velo_params* params,
                             const velo_hits* hits, const velo_tracks* tracks,
                             const velo_states* states, void* d_ws, size_t ws_bytes,
                             hipStream_t stream) {
  if (!geometry_ok(geom)) return VELO_ERR_ARG;
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(tracks) || !states_ok(states) ||
      !params_ok(params) || (n_pixels > 0 && !d_pixels) || !d_ws)
    return VELO_ERR_ARG;
  if (n_pixels >= (1ull << 32) * 3) return VELO_ERR_ARG;
  if (ws_bytes < velo_workspace_bytes(n_pixels, n_events)) return VELO_ERR_WORKSPACE;
  velo_status st =
      velo_cluster(d_pixels, d_offsets, n_events, n_pixels, geom, hits, d_ws, ws_bytes, stream);
  if (st != VELO_OK) return st;
  st = velo_find_tracks(hits, d_offsets, n_events, n_pixels, geom, params, tracks, d_ws, ws_bytes,
                        stream);
  if (st != VELO_OK) return st;
  return velo_fit(hits, tracks, d_offsets, n_events, n_pixels, geom, params, states, stream);
}

velo_status velo_reconstruct_timed(const uint32_t* d_pixels, const uint64_t* d_offsets,
                                   uint32_t n_events, uint64_t n_pixels, const velo_geometry* geom,
                                   const velo_params* params, const velo_hits* hits,
                                   const velo_tracks* tracks, const velo_states* states, void* d_ws,
                                   size_t ws_bytes, hipStream_t stream, const hipEvent_t* ev6) {
  if (!ev6 || !geometry_ok(geom)) return VELO_ERR_ARG;
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(tracks) || !states_ok(states) ||
      !params_ok(params) || (n_pixels > 0 && !d_pixels) || !d_ws)
    return VELO_ERR_ARG;
  if (n_pixels >= (1ull << 32) * 3) return VELO_ERR_ARG;
  if (ws_bytes < velo_workspace_bytes(n_pixels, n_events)) return VELO_ERR_WORKSPACE;
  hipError_t e = velo::launch_cluster_cfg(d_pixels, d_offsets, n_events, n_pixels, hits, d_ws, stream,
                                          velo::ClusterCfg{0, 512, nullptr, nullptr}, false, ev6);
  if (e == hipSuccess)
    e = velo::launch_find_cfg(hits, d_offsets, n_events, n_pixels, params, tracks, d_ws, stream,
                              velo::FindCfg{velo::kSThreads, 0, nullptr, nullptr, {0, 0, 0}}, ev6 + 2);
  if (e == hipSuccess)
    e = velo::launch_fit_cfg(hits, tracks, d_offsets, n_events, n_pixels, params, nullptr, states,
                             stream, velo::kFitThreads, ev6 + 4);
  return hip_status(e);
}

velo_status velo_fit_mlp(const velo_hits* hits, const velo_tracks* tracks, const uint64_t* d_offsets,
                         uint32_t n_events, uint64_t n_pixels, const velo_geometry* geom,
                         const velo_params* params, const velo_mlp* mlp, const velo_states* out,
                         hipStream_t stream) {
  if (!geometry_ok(geom)) return VELO_ERR_ARG;
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(tracks) || !states_ok(out) || !out->score ||
      !params_ok(params) || !mlp_ok(mlp))
    return VELO_ERR_ARG;
  return hip_status(
      velo::launch_fit_mlp(hits, tracks, d_offsets, n_events, n_pixels, params, mlp, out, stream));
}

velo_status velo_reconstruct_mlp(const uint32_t* d_pixels, const uint64_t* d_offsets,
                                 uint32_t n_events, uint64_t n_pixels, const velo_geometry* geom,
                                 const velo_params* params, const velo_mlp* mlp,
                                 const velo_hits* hits, const velo_tracks* tracks,
                                 const velo_states* states, void* d_ws, size_t ws_bytes,
                                 hipStream_t stream) {
  if (!geometry_ok(geom)) return VELO_ERR_ARG;
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(tracks) || !states_ok(states) || !states->score ||
      !params_ok(params) || !mlp_ok(mlp) || (n_pixels > 0 && !d_pixels) || !d_ws)
    return VELO_ERR_ARG;
  if (n_pixels >= (1ull << 32) * 3) return VELO_ERR_ARG;
  if (ws_bytes < velo_workspace_bytes(n_pixels, n_events)) return VELO_ERR_WORKSPACE;
  velo_status st =
      velo_cluster(d_pixels, d_offsets, n_events, n_pixels, geom, hits, d_ws, ws_bytes, stream);
  if (st != VELO_OK) return st;
  st = velo_find_tracks(hits, d_offsets, n_events, n_pixels, geom, params, tracks, d_ws, ws_bytes,
                        stream);
  if (st != VELO_OK) return st;
  return velo_fit_mlp(hits, tracks, d_offsets, n_events, n_pixels, geom, params, mlp, states, stream);
}

velo_status velo_track_features(const velo_hits* hits, const velo_tracks* tracks,
                                const velo_states* states, const uint64_t* d_offsets,
                                uint32_t n_events, uint64_t n_pixels, const velo_geometry* geom,
                                float* d_feat, hipStream_t stream) {
  if (!geometry_ok(geom)) return VELO_ERR_ARG;
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(tracks) || !states_ok(states) || !d_feat)
    return VELO_ERR_ARG;
  return hip_status(velo::launch_features(hits, tracks, states, d_offsets, n_events, n_pixels, d_feat,
                                          stream));
}

size_t velo_mlp_workspace_bytes(uint32_t n_samples) { return velo::mlp_workspace_bytes(n_samples); }

velo_status velo_feature_stats(const float* d_feat, uint64_t n, float* d_mean, float* d_std,
                               void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if (!d_feat || !d_mean || !d_std || !d_ws) return VELO_ERR_ARG;
  if (ws_bytes < velo::mlp_workspace_bytes(0)) return VELO_ERR_WORKSPACE;
  return hip_status(velo::launch_feature_stats(d_feat, n, d_mean, d_std, d_ws, stream));
}

velo_status velo_mlp_fwd_bwd(const float* d_params, const float* d_mean, const float* d_std,
                             const float* d_feat, const float* d_label, const uint32_t* d_idx,
                             uint32_t n, float* d_grad, float* d_loss, void* d_ws, size_t ws_bytes,
                             hipStream_t stream) {
  if (!d_params || !d_mean || !d_std || !d_feat || !d_label || !d_grad || !d_ws) return VELO_ERR_ARG;
  if (ws_bytes < velo::mlp_workspace_bytes(n)) return VELO_ERR_WORKSPACE;
  return hip_status(velo::launch_mlp_grad(d_params, d_mean, d_std, d_feat, d_label, d_idx, n, d_grad,
                                          d_loss, d_ws, stream));
}

velo_status velo_mlp_adam_step(float* d_params, float* d_m, float* d_v, const float* d_grad,
                               uint32_t step, float lr, hipStream_t stream) {
  if (!d_params || !d_m || !d_v || !d_grad || step == 0 || !(lr > 0.0f)) return VELO_ERR_ARG;
  return hip_status(velo::launch_adam(d_params, d_m, d_v, d_grad, step, lr, stream));
}

velo_status velo_mlp_infer(const velo_mlp* mlp, const float* d_feat, uint32_t n, float* d_logit,
                           hipStream_t stream) {
  if (n == 0) return VELO_OK;
  if (!mlp_ok(mlp) || !d_feat || !d_logit) return VELO_ERR_ARG;
  return hip_status(
      velo::launch_mlp_infer(mlp->params, mlp->mean, mlp->std, d_feat, n, d_logit, stream));
}

size_t velo_batched_workspace_bytes(uint64_t n_pixels, uint32_t n_events) {
  return velo::batched_workspace_bytes(n_pixels, n_events);
}

velo_status velo_context_create(velo_context** ctx, const velo_geometry* geom,
                                const velo_params* params) {
  if (!ctx || !geometry_ok(geom) || !params_ok(params)) return VELO_ERR_ARG;
  velo_context* c = new velo_context();
  c->params = *params;
  // side stream of the forked track-finding tier (default priority); without
  // it the batched form runs unforked
  int dev = -1;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipStreamCreateWithFlags(&c->fork.side, hipStreamNonBlocking) == hipSuccess) {
    if (hipEventCreateWithFlags(&c->fork.fork_ev, hipEventDisableTiming) == hipSuccess &&
        hipEventCreateWithFlags(&c->fork.join_ev, hipEventDisableTiming) == hipSuccess) {
      c->side_dev = dev;
    } else {
      if (c->fork.fork_ev) (void)hipEventDestroy(c->fork.fork_ev);
      (void)hipStreamDestroy(c->fork.side);
      c->fork = velo::Fork{nullptr, nullptr, nullptr};
    }
  } else {
    c->fork.side = nullptr;
  }
  (void)hipGetLastError();
  *ctx = c;
  return VELO_OK;
}

void velo_context_destroy(velo_context* ctx) {
  if (!ctx) return;
  drop_graphs(ctx);
  void* bufs[] = {ctx->net, ctx->adam_m, ctx->adam_v, ctx->grad, ctx->loss, ctx->mlp_ws};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (ctx->fork.side) {
    (void)hipStreamSynchronize(ctx->fork.side);
    (void)hipEventDestroy(ctx->fork.fork_ev);
    (void)hipEventDestroy(ctx->fork.join_ev);
    (void)hipStreamDestroy(ctx->fork.side);
  }
  delete ctx;
}

velo_status velo_context_set_config(velo_context* ctx, const int32_t* in12) {
  if (!ctx || !in12) return VELO_ERR_ARG;
  const int32_t cg = in12[0], mg = in12[1], ft = in12[2], fg = in12[3], fit = in12[4];
  const int32_t route = in12[8], fork = in12[9], order = in12[10], tiny = in12[11];
  if (cg < 0 || cg > 65536 || mg < 1 || mg > 65536 || (ft != 128 && ft != 256) || fg < 0 ||
      fg > 65536 || (fit != 64 && fit != 128 && fit != 256))
    return VELO_ERR_ARG;
  if (route < -1 || (route != 0 && fg != 0) || (fork != 0 && fork != 1) || (fork && !route) ||
      (order != 0 && order != 1) || (order && fg != 0) || (tiny != 0 && tiny != 1) ||
      (tiny && (fg != 0 || route != 0 || ft != 256)))
    return VELO_ERR_ARG;
  const uint32_t full[3] = {velo::kMBlocks, velo::kLBlocks, velo::kGBlocks};
  for (int i = 0; i < 3; ++i)
    if (in12[5 + i] < 1 || (uint32_t)in12[5 + i] > full[i]) return VELO_ERR_ARG;
  ctx->cfg = velo::BatchedCfg{(uint32_t)cg, (uint32_t)mg, ft, (uint32_t)fg, fit,
                              {(uint32_t)in12[5], (uint32_t)in12[6], (uint32_t)in12[7]},
                              route == -1 ? 0xFFFFFFFFu : (uint32_t)route, (uint32_t)fork, (uint32_t)order,
                              (uint32_t)tiny};
  ctx->tuned = true;
  ctx->source = 3;
  for (int i = 0; i < 5; ++i) ctx->tuned_ms[i] = 0.0f;
  drop_graphs(ctx);
  return VELO_OK;
}

velo_status velo_context_config(const velo_context* ctx, int32_t* out13, float* tuned_ms5) {
  if (!ctx || !out13) return VELO_ERR_ARG;
  out13[0] = ctx->tuned ? ctx->source : 0;
  out13[1] = (int32_t)ctx->cfg.small_grid;
  out13[2] = (int32_t)ctx->cfg.mid_grid;
  out13[3] = ctx->cfg.find_threads;
  out13[4] = (int32_t)ctx->cfg.find_grid;
  out13[5] = ctx->cfg.fit_threads;
  for (int i = 0; i < 3; ++i) out13[6 + i] = (int32_t)ctx->cfg.esc_grid[i];
  out13[9] = ctx->cfg.route_hits == 0xFFFFFFFFu ? -1 : (int32_t)ctx->cfg.route_hits;
  out13[10] = (int32_t)ctx->cfg.fork;
  out13[11] = (int32_t)ctx->cfg.find_order;
  out13[12] = (int32_t)ctx->cfg.tiny;
  if (tuned_ms5)
    for (int i = 0; i < 5; ++i) tuned_ms5[i] = ctx->tuned_ms[i];
  return VELO_OK;
}

velo_status velo_reconstruct_batched(velo_context* ctx, const uint32_t* d_pixels,
                                     const uint64_t* d_offsets, uint32_t n_events, uint64_t n_pixels,
                                     const velo_params* params, const velo_mlp* mlp,
                                     const velo_hits* hits, const velo_tracks* tracks,
                                     const velo_states* states, void* d_ws, size_t ws_bytes,
                                     hipStream_t stream) {
  if (!ctx) return VELO_ERR_ARG;
  if (!params) params = &ctx->params;
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(tracks) || !states_ok(states) ||
      !params_ok(params) || (n_pixels > 0 && !d_pixels) || !d_ws || (mlp && (!mlp_ok(mlp) || !states->score)))
    return VELO_ERR_ARG;
  if (n_pixels >= (1ull << 32) * 3) return VELO_ERR_ARG;
  if (ws_bytes < velo::batched_workspace_bytes(n_pixels, n_events)) return VELO_ERR_WORKSPACE;
  velo_mlp held;  // the context's own classifier when the call names none
  if (!mlp && ctx->net) {
    held = velo_mlp{ctx->net, ctx->net + VELO_MLP_PARAMS, ctx->net + VELO_MLP_PARAMS + VELO_MLP_FEATURES,
                    ctx->threshold};
    if (!states->score) return VELO_ERR_ARG;
    mlp = &held;
  }
  velo::BatchedCall c;
  memset(&c, 0, sizeof(c));
  c.px = d_pixels;
  c.offsets = d_offsets;
  c.n_events = n_events;
  c.n_pixels = n_pixels;
  c.params = *params;
  c.has_mlp = mlp != nullptr;
  if (mlp) c.mlp = *mlp;
  c.hits = *hits;
  c.tracks = *tracks;
  c.states = *states;
  c.ws = d_ws;
  c.ws_bytes = ws_bytes;
  hipError_t e;
  // a stream the caller is capturing: enqueue into the caller's graph with the
  // current shapes (no tuning, which synchronises, and no graph of our own)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (stream != nullptr && hipStreamIsCapturing(stream, &cs) != hipSuccess) return VELO_ERR_HIP;
  // the fork's side stream serves calls on the device the context was made on
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return VELO_ERR_HIP;
  const velo::Fork fk = dev == ctx->side_dev ? ctx->fork : velo::Fork{nullptr, nullptr, nullptr};
  if (cs != hipStreamCaptureStatusNone) return hip_status(velo::enqueue_batched(c, ctx->cfg, stream, fk));
  if (!ctx->tuned) {
    TuneKey k;
    const bool keyed = tune_key(c, &k);
    if (keyed && tune_lookup(k, &ctx->cfg, ctx->tuned_ms)) {
      ctx->tuned = true;
      ctx->source = 2;
    } else {
      if ((e = velo::autotune(ctx, c, stream, fk)) != hipSuccess) return VELO_ERR_HIP;
      ctx->source = 1;
      if (keyed) tune_store(k, ctx->cfg, ctx->tuned_ms);
    }
    drop_graphs(ctx);
  }
  if (stream == nullptr)  // the legacy default stream cannot be captured
    return hip_status(velo::enqueue_batched(c, ctx->cfg, stream, fk));
  ctx->clock++;
  for (int i = 0; i < ctx->n_graphs; ++i) {
    velo_context::Entry& g = ctx->graphs[i];
    if (g.stream == stream && same_call(g.key, c)) {
      g.last_use = ctx->clock;
      return hip_status(hipGraphLaunch(g.exec, stream));
    }
  }
  // capture a new graph, replacing the least recently used one when full
  int slot = ctx->n_graphs;
  if (slot == velo_context::kGraphs) {
    slot = 0;
    for (int i = 1; i < ctx->n_graphs; ++i)
      if (ctx->graphs[i].last_use < ctx->graphs[slot].last_use) slot = i;
    drop_entry(ctx->graphs[slot]);
  } else {
    ctx->n_graphs++;
  }
  velo_context::Entry& g = ctx->graphs[slot];
  g.graph = nullptr;
  g.exec = nullptr;
  if ((e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
    g = ctx->graphs[ctx->n_graphs - 1];  // drop the empty slot
    ctx->n_graphs--;
    return VELO_ERR_HIP;
  }
  const hipError_t le = velo::enqueue_batched(c, ctx->cfg, stream, fk);
  e = hipStreamEndCapture(stream, &g.graph);
  if (le == hipSuccess && e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
  if (le != hipSuccess || e != hipSuccess) {
    drop_entry(g);
    g = ctx->graphs[ctx->n_graphs - 1];
    ctx->n_graphs--;
    return VELO_ERR_HIP;
  }
  g.key = c;
  g.stream = stream;
  g.last_use = ctx->clock;
  return hip_status(hipGraphLaunch(g.exec, stream));
}

velo_status velo_mlp_load(velo_context* ctx, const void* h_blob, size_t bytes) {
  if (!ctx || !h_blob || bytes != VELO_MLP_BLOB_BYTES) return VELO_ERR_ARG;
  uint32_t head[4];
  memcpy(head, h_blob, sizeof(head));
  if (head[0] != VELO_MLP_BLOB_MAGIC || head[1] != 1u || head[2] != VELO_MLP_PARAMS ||
      head[3] != VELO_MLP_FEATURES)
    return VELO_ERR_ARG;
  constexpr int kNet = VELO_MLP_PARAMS + 2 * VELO_MLP_FEATURES;
  float v[kNet + 1];
  memcpy(v, (const char*)h_blob + sizeof(head), sizeof(v));
  for (int i = 0; i < kNet + 1; ++i)
    if (!isfinite(v[i])) return VELO_ERR_ARG;
  for (int i = 0; i < VELO_MLP_FEATURES; ++i)
    if (!(v[VELO_MLP_PARAMS + VELO_MLP_FEATURES + i] > 0.0f)) return VELO_ERR_ARG;
  hipError_t e = hipSuccess;
  if (!ctx->net) {
    e = hipMalloc((void**)&ctx->net, kNet * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->adam_m, VELO_MLP_PARAMS * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->adam_v, VELO_MLP_PARAMS * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->grad, VELO_MLP_PARAMS * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->loss, sizeof(float));
    if (e != hipSuccess) return VELO_ERR_HIP;
  }
  e = hipMemcpy(ctx->net, v, kNet * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(ctx->adam_m, 0, VELO_MLP_PARAMS * sizeof(float));
  if (e == hipSuccess) e = hipMemset(ctx->adam_v, 0, VELO_MLP_PARAMS * sizeof(float));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return VELO_ERR_HIP;
  ctx->threshold = v[kNet];
  drop_graphs(ctx);
  return VELO_OK;
}

velo_status velo_mlp_save(const velo_context* ctx, void* h_blob, size_t bytes) {
  if (!ctx || !h_blob || bytes != VELO_MLP_BLOB_BYTES || !ctx->net) return VELO_ERR_ARG;
  constexpr int kNet = VELO_MLP_PARAMS + 2 * VELO_MLP_FEATURES;
  const uint32_t head[4] = {VELO_MLP_BLOB_MAGIC, 1u, VELO_MLP_PARAMS, VELO_MLP_FEATURES};
  float v[kNet + 1];
  if (hipMemcpy(v, ctx->net, kNet * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) return VELO_ERR_HIP;
  v[kNet] = ctx->threshold;
  memcpy(h_blob, head, sizeof(head));
  memcpy((char*)h_blob + sizeof(head), v, sizeof(v));
  return VELO_OK;
}

velo_status velo_mlp_train_step(velo_context* ctx, const float* d_feat, const float* d_label,
                                const uint32_t* d_idx, uint32_t n, float lr, uint32_t step,
                                float* d_loss, hipStream_t stream) {
  if (!ctx || !ctx->net || !d_feat || !d_label || n == 0 || step == 0 || !(lr > 0.0f) || !isfinite(lr))
    return VELO_ERR_ARG;
  const size_t need = velo::mlp_workspace_bytes(n);
  if (ctx->mlp_ws_bytes < need) {
    if (ctx->mlp_ws) {
      if (hipStreamSynchronize(stream) != hipSuccess || hipFree(ctx->mlp_ws) != hipSuccess) return VELO_ERR_HIP;
      ctx->mlp_ws = nullptr;
      ctx->mlp_ws_bytes = 0;
    }
    if (hipMalloc(&ctx->mlp_ws, need) != hipSuccess) return VELO_ERR_HIP;
    ctx->mlp_ws_bytes = need;
  }
  float* P = ctx->net;
  hipError_t e = velo::launch_mlp_grad(P, P + VELO_MLP_PARAMS, P + VELO_MLP_PARAMS + VELO_MLP_FEATURES,
                                       d_feat, d_label, d_idx, n, ctx->grad, d_loss ? d_loss : ctx->loss,
                                       ctx->mlp_ws, stream);
  if (e == hipSuccess) e = velo::launch_adam(P, ctx->adam_m, ctx->adam_v, ctx->grad, step, lr, stream);
  return hip_status(e);
}

velo_status velo_check_status(const uint32_t* d_status_a, const uint32_t* d_status_b, uint32_t n_events,
                              uint32_t* d_word, uint32_t* h_or, hipStream_t stream) {
  if (!h_or || !d_word || (!d_status_a && !d_status_b)) return VELO_ERR_ARG;
  *h_or = 0;
  if (n_events == 0) return VELO_OK;
  hipLaunchKernelGGL(velo::k_status_or, dim3(1), dim3(1024), 0, stream, d_status_a, d_status_b, n_events,
                     d_word);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h_or, d_word, sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return VELO_ERR_HIP;
  return *h_or ? VELO_ERR_INPUT : VELO_OK;
}

void velo_pv_params_default(velo_pv_params* p) {
  if (!p) return;
  p->z0 = -256.0f;
  p->bin_w = 0.5f;
  p->n_bins = 1024;
  p->max_var = 4.0f;
  p->seed_min = 8;
  p->nms = 2;
  p->chi2_cut = 9.0f;
  p->n_iter = 8;
  p->min_weight = 3.0f;
}

velo_status velo_find_pvs(const velo_tracks* tracks, const velo_states* states,
                          const uint64_t* d_offsets, uint32_t n_events, uint64_t n_pixels,
                          const velo_pv_params* p, const velo_pvs* out, hipStream_t stream) {
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !tracks || !tracks->n_tracks || !states || !states->z || !states->tx ||
      !states->ty || !states->cov_x || !states->cov_y || !states->accepted || !out || !out->n_pv ||
      !out->z || !out->var || !out->weight || !out->status || !p)
    return VELO_ERR_ARG;
  if (!(p->n_bins >= 1 && p->n_bins <= velo::kPvBins) || !(p->bin_w > 0.0f) || !isfinite(p->bin_w) ||
      !isfinite(p->z0) || !isfinite(p->z0 + p->bin_w * (float)p->n_bins) || !(p->max_var > 0.0f) ||
      p->seed_min < 1 || p->nms < 0 || p->nms > 64 || !(p->chi2_cut > 0.0f) ||
      !isfinite(p->chi2_cut) || p->n_iter < 0 || p->n_iter > 64 || !isfinite(p->min_weight))
    return VELO_ERR_ARG;
  return hip_status(velo::launch_find_pvs(tracks, states, d_offsets, n_events, n_pixels, p, out, stream));
}

void velo_ut_params_default(velo_ut_params* p) {
  if (!p) return;
  p->p_min_mev = 3000.0f;
  p->kick_mev = 45.0f;
  p->z_kick = 1000.0f;
  p->tol_u = 1.0f;
  p->tol_y = 10.0f;
}

velo_status velo_ut_windows(const uint32_t* d_ut_words, const uint64_t* d_ut_offsets,
                            uint32_t n_events, uint64_t n_ut, const velo_tracks* tracks,
                            const velo_states* states, const uint64_t* d_offsets,
                            uint64_t n_pixels, const velo_ut_params* params,
                            const velo_ut_out* out, hipStream_t stream) {
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_ut_offsets || (n_ut > 0 && !d_ut_words) || !d_offsets || !tracks || !tracks->n_tracks ||
      !states || !states->x || !states->y || !states->z || !states->tx || !states->ty ||
      !states->accepted || !params || !out || !out->sorted || !out->region || !out->status ||
      !out->win || ((uintptr_t)out->win & 15u) != 0)
    return VELO_ERR_ARG;
  if (!(params->p_min_mev > 0.0f) || !isfinite(params->p_min_mev) || !isfinite(params->kick_mev) ||
      !isfinite(params->z_kick) || !isfinite(params->tol_u) || !isfinite(params->tol_y))
    return VELO_ERR_ARG;
  return hip_status(velo::launch_ut(d_ut_words, d_ut_offsets, n_events, n_ut, d_offsets, n_pixels, tracks,
                                    states, params, out, stream));
}

velo_status velo_reconstruct_noalloc(const uint32_t* d_pixels, const uint64_t* d_offsets,
                                     uint32_t n_events, uint64_t n_pixels, const velo_geometry* geom,
                                     const velo_params* params, const velo_hits* hits,
                                     const velo_tracks* tracks, const velo_states* states,
                                     hipStream_t stream) {
  if (!geometry_ok(geom)) return VELO_ERR_ARG;
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(tracks) || !states_ok(states) ||
      !params_ok(params) || (n_pixels > 0 && !d_pixels))
    return VELO_ERR_ARG;
  if (n_pixels >= (1ull << 32) * 3) return VELO_ERR_ARG;
  const size_t need = velo_workspace_bytes(n_pixels, n_events);
  if (need > (size_t)VELO_NOALLOC_SCRATCH_BYTES) return VELO_ERR_WORKSPACE;
  void* ws = scratch_address();
  if (!ws) return VELO_ERR_HIP;
  // every counter and list the kernels use is cleared by the kernels
  // themselves (no memset node, no allocation)
  return velo_reconstruct(d_pixels, d_offsets, n_events, n_pixels, geom, params, hits, tracks, states,
                          ws, (size_t)VELO_NOALLOC_SCRATCH_BYTES, stream);
}

velo_status velo_pipeline_create(velo_pipeline** out, const velo_pipeline_config* cfg,
                                 const velo_geometry* geom, const velo_params* params,
                                 const velo_mlp* mlp, const velo_pv_params* pv_params) {
  if (!out || !cfg || !geometry_ok(geom) || !params_ok(params) || (mlp && !mlp_ok(mlp)))
    return VELO_ERR_ARG;
  if (cfg->n_streams < 1 || cfg->n_streams > 32 || cfg->events_per_batch < 1 ||
      cfg->events_per_batch > VELO_MAX_EVENTS || cfg->words_per_batch < 1 ||
      cfg->words_per_batch >= (1ull << 32) * 3)
    return VELO_ERR_ARG;
  velo_pipeline* p = new velo_pipeline();
  p->cfg = *cfg;
  p->geom = *geom;
  p->params = *params;
  p->has_mlp = mlp != nullptr;
  if (mlp) p->mlp = *mlp;
  if (pv_params) p->pvp = *pv_params;
  else velo_pv_params_default(&p->pvp);
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return VELO_ERR_HIP;
  }
  p->slots.resize(cfg->n_streams);
  for (Slot& s : p->slots)
    if (make_slot(s, cfg->events_per_batch, cfg->words_per_batch) != hipSuccess) {
      velo_pipeline_destroy(p);
      return VELO_ERR_HIP;
    }
  *out = p;
  return VELO_OK;
}

void velo_pipeline_destroy(velo_pipeline* p) {
  if (!p) return;
  for (Slot& s : p->slots) free_slot(s);
  delete p;
}

velo_status velo_pipeline_run(velo_pipeline* p, const uint32_t* h_pixels, uint64_t n_pixels,
                              const uint64_t* h_offsets, uint32_t n_events,
                              const velo_pipeline_result* out, uint64_t* n_rows) {
  if (!p || !out || !n_rows) return VELO_ERR_ARG;
  *n_rows = 0;
  if (n_events == 0) return VELO_OK;
  if (!h_offsets || (n_pixels > 0 && !h_pixels) || !out->status || !out->n_tracks ||
      !out->first_track || (out->track_capacity > 0 && !out->tracks) ||
      (out->n_pv && (!out->pv_z || !out->pv_var)))
    return VELO_ERR_ARG;
  // global event cut and batches (on the host, from the event sizes)
  std::vector<uint32_t> sel;
  std::vector<Batch> batches;
  uint64_t before = 0;
  for (uint32_t e = 0; e < n_events; ++e) {
    const uint64_t a = h_offsets[e], b = h_offsets[e + 1];
    const bool usable = a <= b && b <= n_pixels && a >= before;
    if (a > before) before = a;
    const uint64_t n = usable ? b - a : 0;
    uint32_t st = 0;
    if (!usable) st = VELO_EV_BAD_OFFSETS;
    else if ((p->cfg.gec_max_words && n > p->cfg.gec_max_words) || n > p->cfg.words_per_batch)
      st = VELO_EV_GEC;
    out->status[e] = st;
    out->n_tracks[e] = 0;
    out->first_track[e] = 0;
    if (out->n_pv) {
      out->n_pv[e] = 0;
      memset(out->pv_z + (size_t)e * VELO_MAX_PVS, 0, VELO_MAX_PVS * 4);
      memset(out->pv_var + (size_t)e * VELO_MAX_PVS, 0, VELO_MAX_PVS * 4);
    }
    if (st) continue;
    if (batches.empty() || batches.back().n == p->cfg.events_per_batch ||
        batches.back().words + n > p->cfg.words_per_batch)
      batches.push_back(Batch{(uint64_t)sel.size(), 0, 0});
    batches.back().n++;
    batches.back().words += n;
    sel.push_back(e);
  }
  RunShared R;
  R.px = h_pixels;
  R.off = h_offsets;
  R.sel = &sel;
  R.batches = &batches;
  R.out = out;
  const int S = (int)p->slots.size();
  const int used = (int)(batches.size() < (size_t)S ? batches.size() : (size_t)S);
  std::vector<std::thread> th;
  std::vector<velo_status> st(used, VELO_OK);
  for (int k = 0; k < used; ++k)
    th.emplace_back([&, k] {
      st[k] = slot_run(p, k, &R);
      if (st[k] != VELO_OK) R.err.store((int)st[k]);
    });
  for (std::thread& t : th) t.join();
  const uint64_t rows = R.rows.load();
  *n_rows = rows < out->track_capacity ? rows : out->track_capacity;
  for (int k = 0; k < used; ++k)
    if (st[k] != VELO_OK) return st[k];
  return VELO_OK;
}

const char* velo_status_string(velo_status s) {
  switch (s) {
    case VELO_OK: return "ok";
    case VELO_ERR_ARG: return "invalid argument";
    case VELO_ERR_INPUT: return "at least one event is flagged";
    case VELO_ERR_WORKSPACE: return "workspace too small";
    case VELO_ERR_HIP: return "HIP launch error";
  }
  return "unknown status";
}

}  // extern "C"
