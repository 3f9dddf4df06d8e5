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
 *   - Argument errors (null pointer, workspace too small, a geometry other
 *     than the built-in detector model) return VELO_ERR_ARG /
 *     VELO_ERR_WORKSPACE before anything is enqueued.  Content errors are reported per event in status arrays;
 *     an event with a status bit set contributes no hits and no tracks and
 *     does not affect other events.  Launch failures return VELO_ERR_HIP.
 *   - n_pixels is the length of the pixel buffer (normally offsets[n_events]).
 *     Event e is usable only if offsets[e] <= offsets[e+1] <= n_pixels and no
 *     earlier offset exceeds offsets[e]; then no two usable events share a
 *     word or an output slot.  Any other event gets VELO_EV_BAD_OFFSETS (and
 *     no other bit), no hits and no tracks; the rest of the batch is
 *     unaffected.
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
    VELO_ERR_INPUT = 2,      /* velo_check_status: at least one event is flagged */
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
    VELO_EV_BAD_OFFSETS = 32u, /* offsets unusable: decreasing, beyond n_pixels, or below an
                                  earlier offset (see the conventions above) */
    VELO_EV_PV_OVERFLOW = 64u  /* vertex finding: more than 2048 admitted tracks (no PVs) or
                                  more than VELO_MAX_PVS candidates (the first kept) */
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

/* Detector model.  The kernels are built for one model: 26 planes at
   z = -280 + 1030 l / 25 mm (evaluated in double, rounded once to binary32),
   1536 x 1536 pixels of 55 um centred on the beam axis, pixels whose centre
   lies within 5.1 mm of the axis inactive.  Every call that decodes pixels or
   uses plane positions takes the caller's statement of the model and
   returns VELO_ERR_ARG before enqueuing anything when it differs from the
   built-in one (field by field, plane positions bit for bit), so a caller
   with another detector cannot silently get results for this one.        */
typedef struct {
    int32_t n_layers;        /* 26 */
    float z_mm[26];          /* plane positions */
    float pitch_mm;          /* 0.055 */
    int32_t n_cols, n_rows;  /* 1536, 1536 */
    float hole_r_mm;         /* 5.1 */
} velo_geometry;
void velo_geometry_default(velo_geometry* g);

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
                         uint64_t n_pixels, const velo_geometry* geom, const velo_hits* out, void* d_ws, size_t ws_bytes,
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
                             uint64_t n_pixels, const velo_geometry* geom, const velo_params* params, const velo_tracks* out,
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
                     uint32_t n_events, uint64_t n_pixels, const velo_geometry* geom,
                     const velo_params* params,
                     const velo_states* out, hipStream_t stream);

/* The fit with a measured momentum (paper Sec. 2.3.5: the Velo-only Kalman
   filter is run again with the momentum estimated from the whole track,
   which improves the impact-parameter resolution).  d_p_mev[slot] (device,
   capacity floor(n_pixels/3) slots) is the momentum of the track in that
   slot in MeV.  The filter is velo_fit's with the slope variance added per
   plane crossed = 13.6^2 X/X0 / p^2 (Highland without its logarithm), and
   the transport from the last hit to the beamline point of closest approach
   is taken plane by plane through the planes in between, adding that
   variance at each (the particle crosses them before it reaches the last
   hit).  A momentum that is not a positive finite number gives velo_fit's
   result for that track.  accepted: the plain cut; score (may be NULL):
   chi2/ndof.  Track counts are checked as in velo_fit.  d_p_mev NULL:
   VELO_ERR_ARG.                                                            */
velo_status velo_fit_momentum(const velo_hits* hits, const velo_tracks* tracks,
                              const uint64_t* d_offsets, uint32_t n_events, uint64_t n_pixels,
                              const velo_geometry* geom, const velo_params* params,
                              const float* d_p_mev, const velo_states* out, hipStream_t stream);

/* velo_cluster, velo_find_tracks and velo_fit enqueued back to back. */
velo_status velo_reconstruct(const uint32_t* d_pixels, const uint64_t* d_offsets, uint32_t n_events,
                             uint64_t n_pixels, const velo_geometry* geom, const velo_params* params, const velo_hits* hits,
                             const velo_tracks* tracks, const velo_states* states, void* d_ws,
                             size_t ws_bytes, hipStream_t stream);

/* Measurement hook: velo_reconstruct with HIP events recorded on `stream`
   around the main kernel of each stage, for timing a kernel by itself:
   ev6[0], ev6[1] around the clustering kernel of the (event, plane) segments,
   ev6[2], ev6[3] around the per-event track-finding kernel, ev6[4], ev6[5]
   around the fit kernel.  Null entries are not recorded; the results equal
   velo_reconstruct's.                                                       */
velo_status velo_reconstruct_timed(const uint32_t* d_pixels, const uint64_t* d_offsets,
                                   uint32_t n_events, uint64_t n_pixels, const velo_geometry* geom,
                                   const velo_params* params,
                                   const velo_hits* hits, const velo_tracks* tracks,
                                   const velo_states* states, void* d_ws, size_t ws_bytes,
                                   hipStream_t stream, const hipEvent_t* ev6);

/* velo_fit followed by the classifier in the same kernel: bfloat16 (round to
   nearest even) weights and activations into matrix-core instructions with
   binary32 accumulation; writes score (logit) and accepted.                */
velo_status velo_fit_mlp(const velo_hits* hits, const velo_tracks* tracks, const uint64_t* d_offsets,
                         uint32_t n_events, uint64_t n_pixels, const velo_geometry* geom,
                         const velo_params* params,
                         const velo_mlp* mlp, const velo_states* out, hipStream_t stream);

/* velo_cluster, velo_find_tracks and velo_fit_mlp enqueued back to back. */
velo_status velo_reconstruct_mlp(const uint32_t* d_pixels, const uint64_t* d_offsets,
                                 uint32_t n_events, uint64_t n_pixels, const velo_geometry* geom,
                                 const velo_params* params,
                                 const velo_mlp* mlp, const velo_hits* hits,
                                 const velo_tracks* tracks, const velo_states* states, void* d_ws,
                                 size_t ws_bytes, hipStream_t stream);

/* Raw classifier features (binary32) of every track slot: d_feat[8*slot+k],
   capacity floor(n_pixels/3) slots; needs states from velo_fit.           */
velo_status velo_track_features(const velo_hits* hits, const velo_tracks* tracks,
                                const velo_states* states, const uint64_t* d_offsets,
                                uint32_t n_events, uint64_t n_pixels, const velo_geometry* geom,
                                float* d_feat,
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
   chosen only if it is at least 15 % faster (clustering) or 10 % faster
   (track finding, against the best per-event configuration with its
   options) than one workgroup per item on the tuning stream (under several
   busy streams one workgroup per item interleaves better with the other
   streams' work).  Persistent grids take
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
   velo_batched_workspace_bytes bytes.  With mlp == NULL the context's own
   classifier applies if one was loaded (velo_mlp_load), else the plain cut. */
typedef struct velo_context velo_context;
/* The context keeps the geometry (checked here) and the parameters, which
   velo_reconstruct_batched uses when its params argument is NULL.  It also
   creates a side stream (default priority) and two events on the current
   device, for the forked track-finding tier; if that fails, or on calls made
   with another device current, the batched form runs unforked.  Destroy
   waits for the side stream.                                              */
velo_status velo_context_create(velo_context** ctx, const velo_geometry* geom,
                                const velo_params* params);
void velo_context_destroy(velo_context* ctx);
/* out13 = {how the shapes were chosen (0 not yet, 1 tuned on this context's
   first batch, 2 taken from the process-wide tune cache, 3 set by
   velo_context_set_config), clustering grid (0 = one workgroup per segment),
   large-segment grid, track-finding lanes per event, track-finding grid
   (0 = one workgroup per event), fit lanes per event, then the workgroups of
   the three track-finding tiers that take the events the first one hands on
   (middle 512 lanes, large 1024 lanes, workspace tier), routing, fork,
   event order, tiny tier}.
   The tuner picks those three as the smallest of {512, 256, 128},
   {64, 32, 32}, {16, 8, 8} within 2 % of the best tuning-stream time: a
   tier's launch keeps its grid's LDS reserved until every workgroup has been
   placed, which delays other streams when few events escalate.
   Routing (one workgroup per event only): 0 none; -1 events with a plane
   above the first tier's capacity go straight to the middle tier; n > 0 so
   do events of more than n hits.  Fork 1: the middle tier of the routed
   events runs on a side stream the context owns, beside the first tier, and
   joins the caller's stream before the next tier (inside captured graphs
   too).  Event order 1 (one workgroup per event only): the first tier's
   workgroups take the events largest first.  Tiny tier 1 (one workgroup
   per event, 256 lanes, no routing): a tier for at most 192 hits per plane,
   192 active tracks, 256 candidates and 512 doublets, six workgroups per CU,
   runs every event first and hands the others on to the small tier.  The
   tuner tries order, routing by plane capacity and fork only for batches
   of 8192 events or more (a smaller batch starts all its events at once,
   and beside other streams the extra kernels cost more than they save),
   the tiny tier for any batch, and takes them only when they beat none of
   them by 1 %.  tuned_ms5 (may be
   NULL) = tuning-stream times of the chosen clustering, track-finding and fit
   shapes, then the best clustering time with one workgroup per segment and
   the best track-finding time with one workgroup per event (zeros when set
   by the caller).
   The tuned shapes are kept in a process-wide cache (64 entries) keyed by
   the device architecture, the event count and mean words per event (in
   quarter-octave classes), the classifier flag and the parameters: a new
   context whose first batch falls in a cached class takes the shapes from
   there without timing anything.                                           */
velo_status velo_context_config(const velo_context* ctx, int32_t* out13, float* tuned_ms5);
/* Fix the launch shapes of a context instead of tuning them (for callers that
   know their workload, and for tests that run every shape):
   in12 = {clustering grid 0..65536 (0 = one workgroup per segment),
   large-segment grid 1..65536, track-finding lanes 128 or 256, track-finding
   grid 0..65536 (0 = one workgroup per event), fit lanes 64, 128 or 256,
   middle-tier workgroups 1..512, large-tier workgroups 1..256,
   workspace-tier workgroups 1..128, routing -1..2^31-1 (non-zero only with
   track-finding grid 0), fork 0 or 1 (1 only with routing), event order 0
   or 1 (1 only with track-finding grid 0), tiny tier 0 or 1 (1 only with
   track-finding grid 0, 256 lanes and no routing)}.
   Other values return VELO_ERR_ARG and leave the context unchanged.  Drops
   the context's captured graphs; results do not depend on the shapes.      */
velo_status velo_context_set_config(velo_context* ctx, const int32_t* in12);
size_t velo_batched_workspace_bytes(uint64_t n_pixels, uint32_t n_events);
velo_status velo_reconstruct_batched(velo_context* ctx, const uint32_t* d_pixels,
                                     const uint64_t* d_offsets, uint32_t n_events, uint64_t n_pixels,
                                     const velo_params* params, const velo_mlp* mlp,
                                     const velo_hits* hits, const velo_tracks* tracks,
                                     const velo_states* states, void* d_ws, size_t ws_bytes,
                                     hipStream_t stream);

/* Classifier held by a batched-form context.  velo_mlp_load copies a
   network into device memory the context owns (allocated on the first load)
   and resets its Adam moments; from then on velo_reconstruct_batched with
   mlp == NULL applies it (fused after the fit, as with an explicit mlp;
   states->score is then required).  Blob (VELO_MLP_BLOB_BYTES, host
   memory, little-endian): uint32 magic 0x504C4D56 ("VMLP"), uint32 version
   1, uint32 1377, uint32 8, then binary32 params[1377], mean[8], std[8]
   (each > 0), threshold; every value finite, else VELO_ERR_ARG with the
   context unchanged.  Load and save synchronise the device.               */
#define VELO_MLP_BLOB_MAGIC 0x504C4D56u
#define VELO_MLP_BLOB_BYTES (16u + 4u * (VELO_MLP_PARAMS + 2u * VELO_MLP_FEATURES + 1u))
typedef struct velo_context velo_context;
velo_status velo_mlp_load(velo_context* ctx, const void* h_blob, size_t bytes);
velo_status velo_mlp_save(const velo_context* ctx, void* h_blob, size_t bytes);
/* One training step of the context's classifier on the GPU: the FP32 forward
   and backward pass of velo_mlp_fwd_bwd over n samples (rows d_idx[i], or
   rows 0..n-1 when d_idx is NULL, of d_feat with labels d_label), then the
   Adam update of velo_mlp_adam_step with this step number (>= 1) and
   learning rate.  The mean loss goes to d_loss (may be NULL).  Needs a
   loaded network; grows the context's workspace (a device allocation) the
   first time a larger n is seen.  Asynchronous on `stream`.               */
velo_status velo_mlp_train_step(velo_context* ctx, const float* d_feat, const float* d_label,
                                const uint32_t* d_idx, uint32_t n, float lr, uint32_t step,
                                float* d_loss, hipStream_t stream);

/* Synchronous check of per-event status arrays (either may be NULL, e.g.
   hits.status and tracks.status): the OR of all their words over n_events
   goes to *h_or (d_word: one device word of scratch).  Synchronises
   `stream`; returns VELO_ERR_INPUT if any bit is set, else VELO_OK.       */
velo_status velo_check_status(const uint32_t* d_status_a, const uint32_t* d_status_b, uint32_t n_events,
                              uint32_t* d_word, uint32_t* h_or, hipStream_t stream);

/* Primary vertices (paper Sec. 2.3.1, last paragraph): PV candidates are
   peaks of a histogram of the tracks' beamline z, and every candidate is
   fitted with every track, the track's weight shared among the candidates,
   so the candidates are fitted in parallel.
     admission   accepted tracks with tx^2 + ty^2 >= 1e-6, beamline-z variance
                 var = (tx^2 var_x + ty^2 var_y) / (tx^2 + ty^2)^2 in
                 (0, max_var], z in [z0, z0 + n_bins bin_w); at most 2048 per
                 event (more: VELO_EV_PV_OVERFLOW and no PVs)
     histogram   a track in bin b = floor((z - z0) / bin_w) adds 2 to b and
                 1 to b - 1 and b + 1
     candidates  bins with count >= seed_min, above the nms bins before and
                 at least the nms bins after; seeded at the bin centre
     fit         n_iter rounds, all candidates at once: chi2 = (z - z_v)^2 /
                 var, r = (1 - chi2/chi2_cut)^2 below the cut (else 0),
                 w = r * (r / sum of the track's r over the candidates),
                 z_v = sum(w z / var) / sum(w / var)
     output      var_v = 1 / sum(w / var) and weight sum W_v = sum(w) at the
                 final positions; PVs are the candidates with W_v >=
                 min_weight, in increasing seed z.
   Sums run over tracks in slot order and over candidates in order, in
   binary32 without contraction: results are reproducible bit for bit.    */
#define VELO_MAX_PVS 64
typedef struct {
    float z0;          /* mm, lower edge of the histogram (-256) */
    float bin_w;       /* mm, bin width (0.5) */
    int32_t n_bins;    /* 1..1024 (1024) */
    float max_var;     /* mm^2, largest admitted beamline-z variance (4) */
    int32_t seed_min;  /* smallest count of a candidate bin (8) */
    int32_t nms;       /* bins on each side a candidate dominates, 0..64 (2) */
    float chi2_cut;    /* Tukey cut (9) */
    int32_t n_iter;    /* fit rounds, 0..64 (8) */
    float min_weight;  /* smallest weight sum of a PV (3) */
} velo_pv_params;
void velo_pv_params_default(velo_pv_params* p);
/* Output, per event: n_pv[e]; z, var (variance of z) and weight (weight sum)
   of PV k at e * VELO_MAX_PVS + k, zero beyond n_pv[e]; status[e] = 0 or
   VELO_EV_PV_OVERFLOW.                                                      */
typedef struct {
    uint32_t* n_pv;   /* [n_events] */
    float* z;         /* [n_events * VELO_MAX_PVS] */
    float* var;
    float* weight;
    uint32_t* status; /* [n_events] */
} velo_pvs;
/* Reads the fitted states (z, tx, ty, cov_x[0], cov_y[0], accepted) of the
   track slots of every event (counts clamped like velo_fit's); one workgroup
   per event, no workspace.                                                 */
velo_status velo_find_pvs(const velo_tracks* tracks, const velo_states* states,
                          const uint64_t* d_offsets, uint32_t n_events, uint64_t n_pixels,
                          const velo_pv_params* params, const velo_pvs* out, hipStream_t stream);

/* Velo-to-UT search windows (paper Sec. 2.3.2: the upstream tracker's hits
   are decoded into regions and sorted for a fast look-up, and every Velo
   track is extrapolated to it with the largest bending a particle above
   3 GeV can have).  The paper gives only four strip planes, the outer two
   with vertical strips and the inner two tilted by +5 and -5 degrees; the
   model of this library:
     planes    k = 0..3 at z = 2327.5, 2372.5, 2597.5, 2642.5 mm, strip angles
               0, +5, -5, 0 degrees; a strip measures u = x c_k + y s_k with
               (c_k, s_k) = (1, 0), (0.9961947, 0.08715574),
               (0.9961947, -0.08715574), (1, 0) in binary32;
     strips    8192 of 0.1875 mm: strip n has u = ((float)n + 0.5) 0.1875 - 768;
               each cut into 14 sensor rows of 100 mm, row j covering y in
               [-700 + 100 j, -600 + 100 j);
     raw word  bits [0,13) strip, [13,17) sensor row (< 14), [17,19) plane,
               the rest 0; any order inside an event;
     regions   region r = 14 k + j; an event's words sorted ascending (plane,
               row, strip) make every region a run sorted along u.
   Per event e (UT words [ut_offsets[e], ut_offsets[e+1]), same usable-offsets
   rule as the pixel offsets, at most VELO_UT_MAX_HITS):
     sorted[ut_offsets[e] + i]  the event's words in ascending order (written
                                only for events whose UT status is 0)
     region[57 e + r]           index (event-relative) of the first word of
                                region r, [56] = words; zeros for a flagged event
     status[e]                  VELO_EV_BAD_OFFSETS (UT offsets), UT_OVERFLOW,
                                BAD_WORD, or DUPLICATE (only when no other bit)
   Per track slot s = floor(offsets[e]/3) + t, t < n_tracks[e] (clamped like
   velo_fit's, none when offsets[e+1] < offsets[e] or > n_pixels), 8 words
   win[8 s + 2 k + i] = first | count << 16: the hits of plane k in the i-th
   sensor row the track may cross (rows j with yp + tol_y >= y_lo(j) and
   yp - tol_y < y_hi(j), at most two, increasing j), first = event-relative
   index in `sorted`, count = hits with up - w_k <= u <= up + w_k, 0 if none,
   where from the beamline state dz = z_k - z, xp = x + tx dz, yp = y + ty dz,
   up = xp c_k + yp s_k and w_k = ((kick / p_min) (z_k - z_kick)) c_k + tol_u
   (the largest x bending of a particle above p_min for one transverse kick at
   z_kick).  Tracks not accepted, or of a flagged event, get zeros.  win must
   be 16-byte aligned.  One workgroup per event, no workspace.              */
#define VELO_UT_MAX_HITS 8192u
#define VELO_UT_REGIONS 56
#define VELO_EV_UT_OVERFLOW 256u  /* more than VELO_UT_MAX_HITS UT words in the event */
typedef struct {
    float p_min_mev;  /* smallest momentum the window admits (3000) */
    float kick_mev;   /* transverse-momentum kick between Velo and UT (45) */
    float z_kick;     /* mm, z of that kick (1000) */
    float tol_u;      /* mm, added to the half width along u (1) */
    float tol_y;      /* mm, margin of the sensor rows in y (10) */
} velo_ut_params;
void velo_ut_params_default(velo_ut_params* p);
typedef struct {
    uint32_t* sorted;  /* [n_ut] */
    uint32_t* region;  /* [n_events * 57] */
    uint32_t* status;  /* [n_events] */
    uint32_t* win;     /* [track capacity * 8] */
} velo_ut_out;
/* Reads the states (x, y, z, tx, ty, accepted) of the tracks; params must be
   finite with p_min_mev > 0.                                               */
velo_status velo_ut_windows(const uint32_t* d_ut_words, const uint64_t* d_ut_offsets,
                            uint32_t n_events, uint64_t n_ut, const velo_tracks* tracks,
                            const velo_states* states, const uint64_t* d_offsets,
                            uint64_t n_pixels, const velo_ut_params* params,
                            const velo_ut_out* out, hipStream_t stream);

/* Streaming form (paper Sec. 2.2: raw events are copied to the GPU and only
   tracks and vertices come back; Sec. 3.2: several host-thread / GPU-stream
   pairs keep transfers and kernels of different batches overlapped).
   A pipeline owns n_streams slots, each a host thread with its own HIP
   stream, pinned host staging and device buffers for one batch of at most
   events_per_batch events and words_per_batch raw words.  velo_pipeline_run
   takes raw events in ordinary host memory and
     - applies the global event cut on the host: an event with more raw
       words than gec_max_words (0: no cut), or more than words_per_batch,
       gets VELO_EV_GEC and is not processed (Sec. 2.3: the busiest events
       are removed before the sequence); an event whose host offsets break
       the usable-offsets rule gets VELO_EV_BAD_OFFSETS;
     - packs the remaining events into batches, batch k on slot k mod
       n_streams; per batch: copy in, velo_reconstruct (or
       velo_reconstruct_mlp with the pipeline's classifier), velo_find_pvs,
       gather the tracks into dense rows, copy back counts, statuses and
       vertices, then exactly the rows that exist;
     - fills the caller's result: per event its status (clustering, track
       finding and vertex bits, or VELO_EV_GEC), its track count and the
       index of its first row in `tracks`, and its vertices.  Rows of one
       event are contiguous and in the event's track order; the order of
       the batches in the table depends on which slot finishes first.
   Returns after every slot has finished (synchronous); VELO_ERR_WORKSPACE
   if the rows exceed track_capacity (total raw words / 3 always suffices).
   The pipeline allocates its buffers at creation (about 0.7 GB per slot
   for 1000 events of nominal occupancy); runs of one pipeline must not
   overlap.                                                                */
#define VELO_EV_GEC 128u
typedef struct {
    int32_t n_streams;          /* slots (host-thread / stream pairs), 1..32 */
    uint32_t events_per_batch;  /* 1..VELO_MAX_EVENTS */
    uint64_t words_per_batch;   /* raw-word capacity of a batch */
    uint32_t gec_max_words;     /* global event cut: most raw words of an event (0: none) */
} velo_pipeline_config;
typedef struct {
    float x, y, z, tx, ty, chi2;  /* beamline state and chi2 */
    int32_t ndof;
    uint8_t accepted;             /* quality decision (plain cut or classifier) */
    uint8_t nhits;
    uint16_t pad;
} velo_track_row;                 /* 32 bytes */
typedef struct {
    uint32_t* status;        /* [n_events] */
    uint32_t* n_tracks;      /* [n_events] */
    uint64_t* first_track;   /* [n_events] */
    velo_track_row* tracks;  /* [track_capacity] */
    uint64_t track_capacity;
    uint32_t* n_pv;          /* [n_events], NULL: vertices not copied out */
    float* pv_z;             /* [n_events * VELO_MAX_PVS] */
    float* pv_var;           /* [n_events * VELO_MAX_PVS] */
} velo_pipeline_result;
typedef struct velo_pipeline velo_pipeline;
/* mlp (device pointers, kept valid by the caller for the pipeline's life)
   may be NULL: plain cut; pv_params NULL: velo_pv_params_default.        */
velo_status velo_pipeline_create(velo_pipeline** out, const velo_pipeline_config* cfg,
                                 const velo_geometry* geom, const velo_params* params, const velo_mlp* mlp,
                                 const velo_pv_params* pv_params);
void velo_pipeline_destroy(velo_pipeline* p);
/* h_pixels[n_pixels], h_offsets[n_events + 1]: host memory; *n_rows receives
   the number of rows written.                                             */
velo_status velo_pipeline_run(velo_pipeline* p, const uint32_t* h_pixels, uint64_t n_pixels,
                              const uint64_t* h_offsets, uint32_t n_events,
                              const velo_pipeline_result* out, uint64_t* n_rows);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   reconstruction as velo_reconstruct with the workspace taken from a
   library-owned device array of VELO_NOALLOC_SCRATCH_BYTES (512 MiB), one per
   device, set up on the first call on that device and held until the
   process ends.  The call allocates nothing and needs no d_ws; the caller
   still passes inputs and outputs.  A batch whose velo_workspace_bytes
   exceeds the array returns VELO_ERR_WORKSPACE before anything is enqueued
   (about 1600 events of the nominal occupancy fit).  Every call on one device
   shares that device's array: calls that overlap in time on one device (on
   different streams, or from different host threads) race and must be
   serialised by the caller.  The kernels clear what must start at zero. */
#define VELO_NOALLOC_SCRATCH_BYTES (512ull << 20)
velo_status velo_reconstruct_noalloc(const uint32_t* d_pixels, const uint64_t* d_offsets,
                                     uint32_t n_events, uint64_t n_pixels, const velo_geometry* geom,
                                     const velo_params* params,
                                     const velo_hits* hits, const velo_tracks* tracks,
                                     const velo_states* states, hipStream_t stream);

const char* velo_status_string(velo_status s);

#ifdef __cplusplus
}
#endif
#endif
