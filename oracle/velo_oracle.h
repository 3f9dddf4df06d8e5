/*
 * velo_oracle.h -- plain CPU oracle of the VELO reconstruction path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to judge the HIP
 * implementation; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no source with the HIP library.
 *
 * What it computes (paper: "Allen: A high level trigger on GPUs for LHCb",
 * Sec. 2.3.1 "Velo detector"; Sec. 2.2 for the event-level data layout):
 *   velo_oracle_cluster      decode raw pixel words and group the fired
 *                            pixels of each plane into 8-connected clusters
 *                            (the connected-component labelling of Sec. 2.3.1)
 *   velo_oracle_find_tracks  straight-line search by triplet: seeds of three
 *                            hits on consecutive planes, extended plane by
 *                            plane (Sec. 2.3.1, second paragraph)
 *   velo_oracle_fit          x/y-independent simple Kalman filter with a
 *                            constant 400 MeV transverse momentum for the
 *                            scattering noise, then extrapolation to the
 *                            point of closest approach to the beamline
 *                            (Sec. 2.3.1, third and fourth paragraphs)
 *   velo_oracle_find_pvs     primary vertices from a histogram of the
 *                            tracks' beamline z and a weighted fit of every
 *                            candidate with every track (Sec. 2.3.1, last
 *                            paragraph)
 *   velo_oracle_fit_momentum the fit with a measured momentum (Sec. 2.3.5)
 *   velo_oracle_ut           UT hits sorted into regions and the search
 *                            windows of every Velo track (Sec. 2.3.2)
 *
 * Every rule the paper leaves open (raw format, connectivity, cuts, tie
 * breaks, filter initialisation) is a written reading of the paper, stated
 * next to the code that implements it.  Floating point is IEEE
 * binary32 in the order written, compiled without contraction, because the
 * same decisions (cuts, sorting) are taken in binary32 by the GPU code.
 *
 * All pointers are host pointers.  Arrays indexed "absolute" use the
 * position of the data in the whole batch (pixel offsets), so a caller may
 * pass `offsets + e0` and a sub-range of events.
 */
#ifndef VELO_ORACLE_H
#define VELO_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VO_N_LAYERS 26

/* per-event status bits */
#define VO_EV_BAD_WORD     1u  /* bit 31 set, layer >= 26, row/col >= 1536 or charge 0 */
#define VO_EV_LAYER_ORDER  2u  /* layer field decreases somewhere along the event's words */
#define VO_EV_DUPLICATE    4u  /* two words with the same address (only reported when no other bit is set) */
#define VO_EV_HOLE         8u  /* an otherwise valid word addresses an inactive (beam-hole) pixel */
#define VO_EV_OVERFLOW    16u  /* a track-finding step exceeded VO_MAX_CANDIDATES candidates */
#define VO_EV_BAD_OFFSETS 32u  /* offsets[e] > offsets[e+1], offsets[e+1] > n_pixels, or an
                                  earlier offset above offsets[e] (the event's words may
                                  overlap another event's) */

#define VO_EV_PV_OVERFLOW 64u  /* more than VO_MAX_PVS vertex candidates (the first are kept) */

/* Upper bound on the candidates (seed triplets, or track-hit pairs) of one
   track-finding step.  An event exceeding it is flagged and gets no tracks. */
#define VO_MAX_CANDIDATES 65536u

typedef struct {
    float max_t;        /* |tx|,|ty| limit of a seed doublet */
    float sin2_phi;     /* sin^2 of the largest azimuth difference of a seed doublet */
    float s_seed;       /* mm^2, squared distance of the third seed hit to the doublet line */
    float s_fwd;        /* mm^2, squared distance of a forwarded hit to the track line */
    int32_t max_skip;   /* planes a track may miss in a row before it is closed */
    float sigma_meas;   /* mm, hit resolution */
    float pt0_mev;      /* transverse momentum assumed for scattering noise */
    float x_over_x0;    /* radiation length fraction of one plane */
    float qc3, qc4;     /* chi2/ndof limits of 3-hit / >=4-hit tracks */
} vo_params;

/* Clustering of events [e0, e1) of a batch.
   pixels        raw words, absolute positions; n_pixels words
   offsets[E+1]  absolute word offsets (uint64) of the whole batch (the
                 offsets rule looks at every offset before the event)
   out hits      x, y, key, aux at absolute slot offsets[e] + layer_start[e][l] + rank
   layer_start   [E*27] event-relative first slot of each layer (= index of the
                 layer's first word in the event); [26] = words in the event
   layer_nhits   [E*26] clusters per layer
   n_hits        [E]    clusters per event
   status        [E]    VO_EV_* bits; an event with any bit set has no hits and
                        all its layer_start / layer_nhits entries are 0
   (per-event arrays indexed by the absolute event number)
   returns the OR of the statuses of events [e0, e1) */
uint32_t velo_oracle_cluster(const uint32_t* pixels, const uint64_t* offsets, uint32_t e0,
                             uint32_t e1, uint64_t n_pixels,
                             float* x, float* y, uint32_t* key, uint32_t* aux,
                             uint32_t* layer_start, uint32_t* layer_nhits,
                             uint32_t* n_hits, uint32_t* status);

/* Track finding of events [0, n_events) on clustered hits.
   Track slots of event e start at floor(offsets[e]/3) (absolute).
   n_tracks[n], trk_nhits[slot], hit_idx[slot*26 + j] = event-relative hit slot of
   the track's j-th hit, in decreasing z.  trk_status[n] = 0 or VO_EV_OVERFLOW.
   Tracks of an event are ordered by decreasing key of their first hit. */
void velo_oracle_find_tracks(const float* x, const float* y, const uint32_t* key,
                             const uint32_t* layer_start, const uint32_t* layer_nhits,
                             const uint64_t* offsets, uint32_t n_events, const vo_params* p,
                             uint32_t* n_tracks, uint8_t* trk_nhits, uint32_t* hit_idx,
                             uint32_t* trk_status);

/* Fit of all tracks of events [0, n_events).  State outputs at track slots:
   x, y, z (beamline point of closest approach), tx, ty, cov_x[3*slot] =
   (var x, cov x-tx, var tx), cov_y likewise, chi2, ndof, accepted (plain cut). */
void velo_oracle_fit(const float* x, const float* y, const uint32_t* key,
                     const uint64_t* offsets, uint32_t n_events,
                     const uint32_t* n_tracks, const uint8_t* trk_nhits, const uint32_t* hit_idx,
                     const vo_params* p,
                     float* sx, float* sy, float* sz, float* stx, float* sty,
                     float* cov_x, float* cov_y, float* chi2, int32_t* ndof, uint8_t* accepted);

/* The fit with a measured momentum per track slot (p_mev[slot], MeV): the
   slope variance per plane crossed is 13.6^2 X/X0 / p^2, and the transport
   to the beamline point adds that noise at every plane between it and the
   last hit; a momentum that is not a positive finite number falls back to
   the constant pt0 fit.  With p_mev NULL this is velo_oracle_fit. */
void velo_oracle_fit_momentum(const float* x, const float* y, const uint32_t* key,
                              const uint64_t* offsets, uint32_t n_events,
                              const uint32_t* n_tracks, const uint8_t* trk_nhits,
                              const uint32_t* hit_idx, const float* p_mev, const vo_params* p,
                              float* sx, float* sy, float* sz, float* stx, float* sty,
                              float* cov_x, float* cov_y, float* chi2, int32_t* ndof,
                              uint8_t* accepted);
int32_t velo_oracle_fit_points_p(const float* hx, const float* hy, const float* hz,
                                 const int32_t* hlayer, int32_t n, float p_mev, const vo_params* p,
                                 float* out5, float* cov_x, float* cov_y, float* chi2);

/* Fit of one track given its hit coordinates directly (decreasing z).
   Used by the closed-form checks of the filter.  out[0..4] = x, y, z, tx, ty;
   cov_x[3], cov_y[3], *chi2, returns ndof. */
int32_t velo_oracle_fit_points(const float* hx, const float* hy, const float* hz,
                               const int32_t* hlayer, int32_t n, const vo_params* p,
                               float* out5, float* cov_x, float* cov_y, float* chi2);

/* float z of layer l */
float velo_oracle_layer_z(int32_t l);

/* Primary-vertex finding (velo_oracle_pv.c; Sec. 2.3.1, last paragraph):
   histogram of the tracks' beamline z, peaks as vertex candidates, every
   candidate fitted with every track under shared Tukey weights.  The
   readings are listed at the top of velo_oracle_pv.c. */
#define VO_MAX_PVS 64
#define VO_MAX_PV_TRACKS 2048
typedef struct {
    float z0;          /* mm, lower edge of the histogram */
    float bin_w;       /* mm, bin width */
    int32_t n_bins;
    float max_var;     /* mm^2, largest beamline-z variance of an admitted track */
    int32_t seed_min;  /* smallest histogram count of a candidate bin */
    int32_t nms;       /* bins on each side a candidate must dominate */
    float chi2_cut;    /* Tukey cut */
    int32_t n_iter;    /* fit rounds */
    float min_weight;  /* smallest weight sum of a PV */
} vo_pv_params;
void velo_oracle_pv_params_default(vo_pv_params* p);
/* PVs of events [0, n_events) from the fitted states of their tracks (track
   slots floor(offsets[e]/3) + t, t < n_tracks[e], clamped to the event's
   slots): n_pv[e]; pv_z, pv_var (variance of z), pv_w (weight sum) at
   e * VO_MAX_PVS + k (zero beyond n_pv); pv_status[e] 0 or VO_EV_PV_OVERFLOW. */
void velo_oracle_find_pvs(const uint64_t* offsets, uint32_t n_events, const uint32_t* n_tracks,
                          const float* sz, const float* stx, const float* sty,
                          const float* cov_x, const float* cov_y, const uint8_t* accepted,
                          const vo_pv_params* P, uint32_t* n_pv, float* pv_z, float* pv_var,
                          float* pv_w, uint32_t* pv_status);

/* Velo-to-UT search windows (velo_oracle_ut.c; Sec. 2.3.2): the UT hits of
   every event decoded and sorted into regions (plane, sensor row), then for
   every accepted track and UT plane the hits within the largest bending of
   a particle above p_min.  The readings are listed at the top of
   velo_oracle_ut.c.  Per event: sorted[ut_offsets[e] + i] (the event's words
   in ascending order), region[57 e + r] (first sorted index of region r,
   [56] = hits), ut_status[e]; per track slot (floor(offsets[e]/3) + t, counts
   clamped like the fit's, none when offsets[e+1] < offsets[e] or
   offsets[e+1] > n_pixels): win[8 slot + 2 k + i] = first | count << 16.    */
#define VO_UT_SECTORS 14
#define VO_UT_REGIONS 56
#define VO_UT_MAX_HITS 8192
#define VO_EV_UT_OVERFLOW 256u  /* more than VO_UT_MAX_HITS UT words in the event */
typedef struct {
    float p_min_mev;  /* smallest momentum the window admits */
    float kick_mev;   /* transverse-momentum kick of the field between the Velo and the UT */
    float z_kick;     /* mm, z of that kick */
    float tol_u;      /* mm, added to the half width along u */
    float tol_y;      /* mm, margin of the sensor rows in y */
} vo_ut_params;
void velo_oracle_ut_params_default(vo_ut_params* p);
float velo_oracle_ut_strip_u(uint32_t strip);
void velo_oracle_ut(const uint32_t* ut_words, const uint64_t* ut_offsets, uint32_t n_events,
                    uint64_t n_ut, const uint64_t* offsets, uint64_t n_pixels, const uint32_t* n_tracks,
                    const float* sx, const float* sy, const float* sz, const float* stx,
                    const float* sty, const uint8_t* accepted, const vo_ut_params* P,
                    uint32_t* sorted, uint32_t* region, uint32_t* ut_status, uint32_t* win);

/* Learned track-quality classifier (velo_oracle_mlp.c): 8 features,
   8-32-32-1 network, 1377 parameters W1[32][8], b1[32], W2[32][32], b2[32],
   w3[32], b3.  feat[8*slot]: chi2/ndof, n, missed planes, tx, ty, eta,
   z first plane, z last plane (double). */
int32_t velo_oracle_mlp_nparams(void);
void velo_oracle_features(const uint32_t* key, const uint64_t* offsets, uint32_t n_events,
                          const uint32_t* n_tracks, const uint8_t* trk_nhits, const uint32_t* hit_idx,
                          const float* stx, const float* sty, const float* chi2, const int32_t* ndof,
                          double* feat);
/* mean BCE-with-logits loss over n standardised samples g[8*n], labels y;
   grad[1377] receives its gradient (double) */
double velo_oracle_mlp_fwd_bwd(const double* p, const double* g, const double* y, int64_t n,
                               double* grad);
void velo_oracle_mlp_forward(const double* p, const double* g, int64_t n, double* z);
/* logits in the GPU inference precision (bfloat16 operands, binary32 sums)
   from raw binary32 features f[8*n] and binary32 parameters */
void velo_oracle_mlp_forward_bf16(const float* p, const float* mean, const float* stdv,
                                  const float* f, int64_t n, float* z);

#ifdef __cplusplus
}
#endif
#endif
