/*
 * velo.h -- C ABI of libvelo.so, an MI355X (gfx950) implementation of the
 * VELO reconstruction of the first-level GPU trigger described in
 * "Allen: A high level trigger on GPUs for LHCb" (arXiv:1912.09161).
 *
 * The paper's Velo chain (Sec. 2.3.1) runs over thousands of independent
 * events at once (Sec. 2.2): raw pixel data are decoded and grouped into
 * clusters ("hits") per plane, straight-line tracks are seeded from three
 * hits on consecutive planes and extended plane by plane, and every track is
 * fitted by a simple Kalman filter and extrapolated to the beamline.
 *
 * Conventions of every entry point
 *   - d_* arguments and the buffers inside the structs are DEVICE pointers,
 *     allocated and owned by the caller; the library allocates nothing on
 *     these paths and never synchronises: work is enqueued on `stream` and
 *     the call returns at once.
 *   - Argument errors (null pointer, workspace too small, n_events == 0 with
 *     a null buffer) return VELO_ERR_ARG / VELO_ERR_WORKSPACE before anything
 *     is enqueued.  Content errors are reported per event in status arrays;
 *     an event with a status bit set contributes no hits and no tracks and
 *     does not affect other events.  Launch failures return VELO_ERR_HIP.
 *   - n_pixels must equal offsets[n_events]; events whose offsets are not
 *     non-decreasing or exceed n_pixels get VELO_EV_BAD_OFFSETS.
 *
 * Raw input (the paper's raw data segmented by readout unit, Sec. 2.2):
 *   pixels[n_pixels]  one uint32 word per fired pixel:
 *                     bits [0,11) column, [11,22) row, [22,27) plane,
 *                     [27,31) charge (1..15), bit 31 must be 0.
 *   offsets[n+1]      uint64; event e owns words [offsets[e], offsets[e+1]).
 *                     Words of an event are grouped by ascending plane; any
 *                     order inside a plane.
 * Detector model: 26 planes at z = -280 + 41.2 l mm, 1536 x 1536 pixels of
 * 55 um centred on the beam axis, pixels with centre radius < 5.1 mm
 * ((2c-1535)^2 + (2r-1535)^2 <= 34393) inactive.
 */
#ifndef VELO_H
#define VELO_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VELO_N_LAYERS 26
/* Most candidates (seed triplets, or track-hit pairs) one track-finding step
   of one event may produce; beyond it the event gets VELO_EV_OVERFLOW. */
#define VELO_MAX_CANDIDATES 65536u
/* Largest n_events of one call (launch grids hold 26 x 64 lanes per event
 * within 32 bits); larger batches return VELO_ERR_ARG. */
#define VELO_MAX_EVENTS 2097152u

typedef enum {
    VELO_OK = 0,
    VELO_ERR_ARG = 1,
    VELO_ERR_WORKSPACE = 3,
    VELO_ERR_HIP = 4
} velo_status;

/* per-event status bits */
enum {
    VELO_EV_BAD_WORD = 1u,     /* bit 31 set, plane >= 26, row/col >= 1536 or charge 0 */
    VELO_EV_LAYER_ORDER = 2u,  /* plane field decreases along the event's words */
    VELO_EV_DUPLICATE = 4u,    /* two words with one address (reported only if no other bit) */
    VELO_EV_HOLE = 8u,         /* a valid word addresses an inactive (beam-hole) pixel */
    VELO_EV_OVERFLOW = 16u,    /* a track-finding step exceeded VELO_MAX_CANDIDATES */
    VELO_EV_BAD_OFFSETS = 32u  /* offsets of the event are inconsistent */
};

/* Cut and filter constants.  The paper fixes only pt0 = 400 MeV for the
   scattering noise of the simple Kalman filter (Sec. 2.3.1); the rest are
   this implementation's working point (velo_params_default). */
typedef struct {
    float max_t;       /* |tx|, |ty| limit of a seed doublet */
    float sin2_phi;    /* sin^2 of the largest azimuth difference of a seed doublet */
    float s_seed;      /* mm^2: squared distance of the third seed hit to the doublet line */
    float s_fwd;       /* mm^2: squared distance of an added hit to the track line */
    int32_t max_skip;  /* planes a track may miss in a row before it is closed */
    float sigma_meas;  /* mm: hit resolution */
    float pt0_mev;     /* transverse momentum assumed for scattering noise */
    float x_over_x0;   /* radiation-length fraction of one plane */
    float qc3, qc4;    /* chi2/ndof limits of 3-hit and >= 4-hit tracks */
} velo_params;

/* Hits: the output of velo_cluster.  Capacity n_pixels slots.
   Hits of plane l of event e occupy slots offsets[e] + layer_start[27e+l] + k,
   k < layer_nhits[26e+l], ordered by ascending key (layer_start[27e+l] is the
   index of the plane's first word inside the event; [27e+26] = words of e).
   x, y    mm, charge-weighted mean of the pixel centres (binary32)
   key     smallest 27-bit pixel address of the cluster: plane<<22|row<<11|col
   aux     min(pixels,65535) << 16 | min(charge sum,65535)                   */
typedef struct {
    float* x;
    float* y;
    uint32_t* key;
    uint32_t* aux;
    uint32_t* layer_start;  /* [n_events * 27] */
    uint32_t* layer_nhits;  /* [n_events * 26] */
    uint32_t* n_hits;       /* [n_events] */
    uint32_t* status;       /* [n_events] VELO_EV_* bits */
} velo_hits;

/* Tracks: the output of velo_find_tracks.  Track t of event e lives in slot
   floor(offsets[e] / 3) + t; capacity floor(n_pixels / 3) slots (max 1).
   hit_idx[26*slot + j] is the event-relative hit slot (offsets[e] + value
   indexes the hit arrays) of the j-th hit, j < nhits[slot], in decreasing z.
   Tracks of an event are ordered by decreasing key of their first hit.      */
typedef struct {
    uint32_t* n_tracks;  /* [n_events] */
    uint8_t* nhits;      /* [cap] */
    uint32_t* hit_idx;   /* [cap * 26] */
    uint32_t* status;    /* [n_events] 0 or VELO_EV_OVERFLOW */
} velo_tracks;

/* Fitted states at the point of closest approach to the beamline (z axis),
   one per track slot.  cov_x[3*slot] = (var x, cov(x,tx), var tx), cov_y
   likewise; ndof = 2 n - 4.  accepted: the plain chi2/ndof cut (velo_fit) or
   the learned classifier (velo_fit_mlp).  score (may be NULL for velo_fit):
   chi2/ndof (velo_fit) or the classifier's logit (velo_fit_mlp, required). */
typedef struct {
    float* x;
    float* y;
    float* z;
    float* tx;
    float* ty;
    float* cov_x;  /* [cap * 3] */
    float* cov_y;  /* [cap * 3] */
    float* chi2;
    int32_t* ndof;
    uint8_t* accepted;
    float* score;
} velo_states;

/* Learned track-quality classifier (not in the paper; a learned replacement
   of the plain cut after the fit).  Features of a track: chi2/ndof, n hits,
   missed planes = (first plane - last plane + 1) - n, tx, ty,
   eta = asinh(1/sqrt(tx^2+ty^2)), z of the first and of the last hit plane;
   standardised g = (f - mean) / std.  Network: h1 = relu(W1 g + b1) (32),
   h2 = relu(W2 h1 + b2) (32), logit = w3 . h2 + b3.  params: 1377 binary32
   values W1[32][8], b1[32], W2[32][32], b2[32], w3[32], b3.  All three
   pointers are device pointers; accepted = logit >= threshold.              */
#define VELO_MLP_FEATURES 8
#define VELO_MLP_PARAMS 1377
typedef struct {
    const float* params;  /* [1377] */
    const float* mean;    /* [8] */
    const float* std;     /* [8] */
    float threshold;
} velo_mlp;

/* Default working point (see velo_params). */
void velo_params_default(velo_params* p);

/* Device workspace needed by velo_cluster / velo_find_tracks /
   velo_reconstruct for a batch of n_pixels words and n_events events. */
size_t velo_workspace_bytes(uint64_t n_pixels, uint32_t n_events);

/* Decoding and clustering (paper Sec. 2.3.1, first paragraph: connected
   component labelling of the fired pixels of each plane; here two pixels
   are connected when they touch by side or corner).  Every component gives
   one hit: key = its smallest address, position = charge-weighted mean of
   the pixel centres computed from integer sums, (float)sum(q c)/(float)sum(q),
   in binary32.  Fills every array of `out`.                                 */
velo_status velo_cluster(const uint32_t* d_pixels, const uint64_t* d_offsets, uint32_t n_events,
                         uint64_t n_pixels, const velo_hits* out, void* d_ws, size_t ws_bytes,
                         hipStream_t stream);

/* Track finding by triplet seeding and forwarding (paper Sec. 2.3.1, second
   paragraph).  Planes are visited from z = +750 mm down; at plane l every
   active track takes the closest unused hit within sqrt(s_fwd) of its line
   (greedy by (s, first-hit key, hit key)), a track that misses more than
   max_skip planes in a row is closed, then seeds (h0 on l+2, h1 on l+1, h2
   on l) of unused hits are formed: slopes within max_t, same azimuth within
   asin(sqrt(sin2_phi)), third hit within sqrt(s_seed) of the doublet line,
   accepted greedily by (s, key1, key0, key2).  Each hit joins at most one
   track.  Reads hits from velo_cluster; fills `out`.                        */
velo_status velo_find_tracks(const velo_hits* hits, const uint64_t* d_offsets, uint32_t n_events,
                             uint64_t n_pixels, const velo_params* params, const velo_tracks* out,
                             void* d_ws, size_t ws_bytes, hipStream_t stream);

/* Simple Kalman filter per projection, x and y independent, with multiple
   scattering noise for a constant transverse momentum pt0 (paper Sec. 2.3.1,
   third paragraph), then transport to the point of closest approach to the
   beamline (fourth paragraph), chi2, ndof and the plain quality cut.
   Tracks given by the caller are checked, not trusted: a count above
   floor((offsets[e+1] - offsets[e]) / 3) is clamped to it, and a slot whose
   nhits is outside [3, 26] or whose hit_idx points outside its event is
   skipped (its state is left as it was).                                    */
velo_status velo_fit(const velo_hits* hits, const velo_tracks* tracks, const uint64_t* d_offsets,
                     uint32_t n_events, uint64_t n_pixels, const velo_params* params,
                     const velo_states* out, hipStream_t stream);

/* velo_cluster, velo_find_tracks and velo_fit enqueued back to back. */
velo_status velo_reconstruct(const uint32_t* d_pixels, const uint64_t* d_offsets, uint32_t n_events,
                             uint64_t n_pixels, const velo_params* params, const velo_hits* hits,
                             const velo_tracks* tracks, const velo_states* states, void* d_ws,
                             size_t ws_bytes, hipStream_t stream);

/* velo_fit followed by the classifier in the same kernel: bfloat16 (round to
   nearest even) weights and activations into matrix-core instructions with
   binary32 accumulation; writes score (logit) and accepted.                */
velo_status velo_fit_mlp(const velo_hits* hits, const velo_tracks* tracks, const uint64_t* d_offsets,
                         uint32_t n_events, uint64_t n_pixels, const velo_params* params,
                         const velo_mlp* mlp, const velo_states* out, hipStream_t stream);

/* velo_cluster, velo_find_tracks and velo_fit_mlp enqueued back to back. */
velo_status velo_reconstruct_mlp(const uint32_t* d_pixels, const uint64_t* d_offsets,
                                 uint32_t n_events, uint64_t n_pixels, const velo_params* params,
                                 const velo_mlp* mlp, const velo_hits* hits,
                                 const velo_tracks* tracks, const velo_states* states, void* d_ws,
                                 size_t ws_bytes, hipStream_t stream);

/* Raw classifier features (binary32) of every track slot: d_feat[8*slot+k],
   capacity floor(n_pixels/3) slots; needs states from velo_fit.           */
velo_status velo_track_features(const velo_hits* hits, const velo_tracks* tracks,
                                const velo_states* states, const uint64_t* d_offsets,
                                uint32_t n_events, uint64_t n_pixels, float* d_feat,
                                hipStream_t stream);

/* Workspace of velo_feature_stats / velo_mlp_fwd_bwd for n samples. */
size_t velo_mlp_workspace_bytes(uint32_t n_samples);

/* Mean and standard deviation (population) of n feature rows d_feat[8*i+k]. */
velo_status velo_feature_stats(const float* d_feat, uint64_t n, float* d_mean, float* d_std,
                               void* d_ws, size_t ws_bytes, hipStream_t stream);

/* FP32 training: mean binary cross-entropy-with-logits loss over n samples
   and its gradient.  Sample i is row d_idx[i] (d_idx may be NULL: row i) of
   d_feat (raw features) with label d_label[row] in {0, 1}.  The sums run in
   a fixed order, so the result is deterministic.                          */
velo_status velo_mlp_fwd_bwd(const float* d_params, const float* d_mean, const float* d_std,
                             const float* d_feat, const float* d_label, const uint32_t* d_idx,
                             uint32_t n, float* d_grad, float* d_loss, void* d_ws, size_t ws_bytes,
                             hipStream_t stream);

/* Adam update (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; step >= 1)
   of the 1377 parameters with moment buffers d_m, d_v.                    */
velo_status velo_mlp_adam_step(float* d_params, float* d_m, float* d_v, const float* d_grad,
                               uint32_t step, float lr, hipStream_t stream);

/* Classifier logits of n raw feature rows (the inference of velo_fit_mlp). */
velo_status velo_mlp_infer(const velo_mlp* mlp, const float* d_feat, uint32_t n, float* d_logit,
                           hipStream_t stream);

/* Batched form.  Events of very uneven occupancy in one launch sequence.
   On the first call the context autotunes the launch shapes stage by stage
   (clustering: one workgroup per (event, plane) segment or a persistent grid
   of some size; track finding: lanes per event, one workgroup per event or a
   persistent grid; fit: lanes per workgroup) by timing candidates on that
   call's batch; that call synchronises the stream.  A persistent grid is
   chosen only if it is at least 15 % faster than one workgroup per item on
   the tuning stream (under several busy streams one workgroup per item
   interleaves better with the other streams' work).  Persistent grids take
   their items from device counters in descending size order (the orders are
   built on the device, only for the stages that use them: work stealing).
   The pipeline of a call is captured as a HIP graph and replayed on later
   calls with the same buffers, sizes, parameters and stream (the context
   keeps the 32 most recently used graphs).  Results are identical to
   velo_reconstruct (mlp == NULL) or velo_reconstruct_mlp.  On a stream the
   caller is capturing, the call only enqueues the pipeline into the caller's
   graph with the context's current shapes (no tuning, no graph of its own).
   The context owns the tuned configuration and the graphs; calls on one
   context must not overlap (one host thread at a time).  d_ws:
   velo_batched_workspace_bytes bytes.                                      */
typedef struct velo_context velo_context;
velo_status velo_context_create(velo_context** ctx);
void velo_context_destroy(velo_context* ctx);
/* out6 = {tuned, clustering grid (0 = one workgroup per segment), large-segment
   grid, track-finding lanes per event, track-finding grid (0 = one workgroup
   per event), fit lanes per event}; tuned_ms5 (may be NULL) = tuning-stream
   times of the chosen clustering, track-finding and fit shapes, then the best
   clustering time with one workgroup per segment and the best track-finding
   time with one workgroup per event.                                       */
velo_status velo_context_config(const velo_context* ctx, int32_t* out6, float* tuned_ms5);
size_t velo_batched_workspace_bytes(uint64_t n_pixels, uint32_t n_events);
velo_status velo_reconstruct_batched(velo_context* ctx, const uint32_t* d_pixels,
                                     const uint64_t* d_offsets, uint32_t n_events, uint64_t n_pixels,
                                     const velo_params* params, const velo_mlp* mlp,
                                     const velo_hits* hits, const velo_tracks* tracks,
                                     const velo_states* states, void* d_ws, size_t ws_bytes,
                                     hipStream_t stream);

const char* velo_status_string(velo_status s);

#ifdef __cplusplus
}
#endif
#endif
