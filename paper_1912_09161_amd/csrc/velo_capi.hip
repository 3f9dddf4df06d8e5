// velo_capi.hip -- the C ABI of libvelo.so (declared in include/velo.h):
// argument checks, workspace carving and the ordered launch of the kernels.
// Built as one translation unit with the kernels it launches.
#include "batched.hip"

#include <math.h>

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
bool mlp_ok(const velo_mlp* m) { return m && m->params && m->mean && m->std && isfinite(m->threshold); }
bool params_ok(const velo_params* p) {
  return p && p->max_skip >= 0 && p->max_skip < 26 && p->pt0_mev > 0.0f && p->sigma_meas > 0.0f &&
         isfinite(p->max_t) && isfinite(p->sin2_phi) && isfinite(p->s_seed) && isfinite(p->s_fwd) &&
         isfinite(p->x_over_x0) && p->x_over_x0 >= 0.0f;
}

}  // namespace

extern "C" {

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
                         uint64_t n_pixels, const velo_hits* out, void* d_ws, size_t ws_bytes,
                         hipStream_t stream) {
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(out) || (n_pixels > 0 && !d_pixels) || !d_ws) return VELO_ERR_ARG;
  if (n_pixels >= (1ull << 32) * 3) return VELO_ERR_ARG;
  if (ws_bytes < velo::cluster_workspace_bytes(n_pixels, n_events)) return VELO_ERR_WORKSPACE;
  return hip_status(velo::launch_cluster(d_pixels, d_offsets, n_events, n_pixels, out, d_ws, stream));
}

velo_status velo_find_tracks(const velo_hits* hits, const uint64_t* d_offsets, uint32_t n_events,
                             uint64_t n_pixels, const velo_params* params, const velo_tracks* out,
                             void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(out) || !params_ok(params) || !d_ws)
    return VELO_ERR_ARG;
  if (n_pixels >= (1ull << 32) * 3) return VELO_ERR_ARG;
  if (ws_bytes < velo::find_workspace_bytes(n_pixels, n_events)) return VELO_ERR_WORKSPACE;
  return hip_status(velo::launch_find(hits, d_offsets, n_events, n_pixels, params, out, d_ws, stream));
}

velo_status velo_fit(const velo_hits* hits, const velo_tracks* tracks, const uint64_t* d_offsets,
                     uint32_t n_events, uint64_t n_pixels, const velo_params* params,
                     const velo_states* out, hipStream_t stream) {
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(tracks) || !states_ok(out) || !params_ok(params))
    return VELO_ERR_ARG;
  return hip_status(velo::launch_fit(hits, tracks, d_offsets, n_events, n_pixels, params, out, stream));
}

velo_status velo_reconstruct(const uint32_t* d_pixels, const uint64_t* d_offsets, uint32_t n_events,
                             uint64_t n_pixels, const velo_params* params, const velo_hits* hits,
                             const velo_tracks* tracks, const velo_states* states, void* d_ws,
                             size_t ws_bytes, hipStream_t stream) {
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(tracks) || !states_ok(states) ||
      !params_ok(params) || (n_pixels > 0 && !d_pixels) || !d_ws)
    return VELO_ERR_ARG;
  if (n_pixels >= (1ull << 32) * 3) return VELO_ERR_ARG;
  if (ws_bytes < velo_workspace_bytes(n_pixels, n_events)) return VELO_ERR_WORKSPACE;
  velo_status st = velo_cluster(d_pixels, d_offsets, n_events, n_pixels, hits, d_ws, ws_bytes, stream);
  if (st != VELO_OK) return st;
  st = velo_find_tracks(hits, d_offsets, n_events, n_pixels, params, tracks, d_ws, ws_bytes, stream);
  if (st != VELO_OK) return st;
  return velo_fit(hits, tracks, d_offsets, n_events, n_pixels, params, states, stream);
}

velo_status velo_fit_mlp(const velo_hits* hits, const velo_tracks* tracks, const uint64_t* d_offsets,
                         uint32_t n_events, uint64_t n_pixels, const velo_params* params,
                         const velo_mlp* mlp, const velo_states* out, hipStream_t stream) {
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(tracks) || !states_ok(out) || !out->score ||
      !params_ok(params) || !mlp_ok(mlp))
    return VELO_ERR_ARG;
  return hip_status(
      velo::launch_fit_mlp(hits, tracks, d_offsets, n_events, n_pixels, params, mlp, out, stream));
}

velo_status velo_reconstruct_mlp(const uint32_t* d_pixels, const uint64_t* d_offsets,
                                 uint32_t n_events, uint64_t n_pixels, const velo_params* params,
                                 const velo_mlp* mlp, const velo_hits* hits,
                                 const velo_tracks* tracks, const velo_states* states, void* d_ws,
                                 size_t ws_bytes, hipStream_t stream) {
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(tracks) || !states_ok(states) || !states->score ||
      !params_ok(params) || !mlp_ok(mlp) || (n_pixels > 0 && !d_pixels) || !d_ws)
    return VELO_ERR_ARG;
  if (n_pixels >= (1ull << 32) * 3) return VELO_ERR_ARG;
  if (ws_bytes < velo_workspace_bytes(n_pixels, n_events)) return VELO_ERR_WORKSPACE;
  velo_status st = velo_cluster(d_pixels, d_offsets, n_events, n_pixels, hits, d_ws, ws_bytes, stream);
  if (st != VELO_OK) return st;
  st = velo_find_tracks(hits, d_offsets, n_events, n_pixels, params, tracks, d_ws, ws_bytes, stream);
  if (st != VELO_OK) return st;
  return velo_fit_mlp(hits, tracks, d_offsets, n_events, n_pixels, params, mlp, states, stream);
}

velo_status velo_track_features(const velo_hits* hits, const velo_tracks* tracks,
                                const velo_states* states, const uint64_t* d_offsets,
                                uint32_t n_events, uint64_t n_pixels, float* d_feat,
                                hipStream_t stream) {
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

velo_status velo_context_create(velo_context** ctx) {
  if (!ctx) return VELO_ERR_ARG;
  *ctx = new velo_context();
  return VELO_OK;
}

void velo_context_destroy(velo_context* ctx) {
  if (!ctx) return;
  drop_graphs(ctx);
  delete ctx;
}

velo_status velo_context_config(const velo_context* ctx, int32_t* out6, float* tuned_ms5) {
  if (!ctx || !out6) return VELO_ERR_ARG;
  out6[0] = ctx->tuned ? 1 : 0;
  out6[1] = (int32_t)ctx->cfg.small_grid;
  out6[2] = (int32_t)ctx->cfg.mid_grid;
  out6[3] = ctx->cfg.find_threads;
  out6[4] = (int32_t)ctx->cfg.find_grid;
  out6[5] = ctx->cfg.fit_threads;
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
  if (n_events == 0) return VELO_OK;
  if (n_events > VELO_MAX_EVENTS) return VELO_ERR_ARG;
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(tracks) || !states_ok(states) ||
      !params_ok(params) || (n_pixels > 0 && !d_pixels) || !d_ws || (mlp && (!mlp_ok(mlp) || !states->score)))
    return VELO_ERR_ARG;
  if (n_pixels >= (1ull << 32) * 3) return VELO_ERR_ARG;
  if (ws_bytes < velo::batched_workspace_bytes(n_pixels, n_events)) return VELO_ERR_WORKSPACE;
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
  if (cs != hipStreamCaptureStatusNone) return hip_status(velo::enqueue_batched(c, ctx->cfg, stream));
  if (!ctx->tuned) {
    if ((e = velo::autotune(ctx, c, stream)) != hipSuccess) return VELO_ERR_HIP;
    drop_graphs(ctx);
  }
  if (stream == nullptr)  // the legacy default stream cannot be captured
    return hip_status(velo::enqueue_batched(c, ctx->cfg, stream));
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
  const hipError_t le = velo::enqueue_batched(c, ctx->cfg, stream);
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

const char* velo_status_string(velo_status s) {
  switch (s) {
    case VELO_OK: return "ok";
    case VELO_ERR_ARG: return "invalid argument";
    case VELO_ERR_WORKSPACE: return "workspace too small";
    case VELO_ERR_HIP: return "HIP launch error";
  }
  return "unknown status";
}

}  // extern "C"
