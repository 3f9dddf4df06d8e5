// velo_capi.hip -- the C ABI of libvelo.so (declared in include/velo.h):
// argument checks, workspace carving and the ordered launch of the kernels.
// Built as one translation unit with the kernels it launches.
#include "cluster.hip"
#include "find.hip"
#include "fit.hip"

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
  if (!d_offsets || !hits_ok(out) || (n_pixels > 0 && !d_pixels) || !d_ws) return VELO_ERR_ARG;
  if (n_pixels >= (1ull << 32) * 3) return VELO_ERR_ARG;
  if (ws_bytes < velo::cluster_workspace_bytes(n_pixels, n_events)) return VELO_ERR_WORKSPACE;
  return hip_status(velo::launch_cluster(d_pixels, d_offsets, n_events, n_pixels, out, d_ws, stream));
}

velo_status velo_find_tracks(const velo_hits* hits, const uint64_t* d_offsets, uint32_t n_events,
                             uint64_t n_pixels, const velo_params* params, const velo_tracks* out,
                             void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if (n_events == 0) return VELO_OK;
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
  if (!d_offsets || !hits_ok(hits) || !tracks_ok(tracks) || !states_ok(out) || !params_ok(params))
    return VELO_ERR_ARG;
  return hip_status(velo::launch_fit(hits, tracks, d_offsets, n_events, n_pixels, params, out, stream));
}

velo_status velo_reconstruct(const uint32_t* d_pixels, const uint64_t* d_offsets, uint32_t n_events,
                             uint64_t n_pixels, const velo_params* params, const velo_hits* hits,
                             const velo_tracks* tracks, const velo_states* states, void* d_ws,
                             size_t ws_bytes, hipStream_t stream) {
  if (n_events == 0) return VELO_OK;
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
