/*
 * velo_oracle_pv.c -- CPU oracle of primary-vertex finding on fitted Velo
 * tracks.  TEST INFRASTRUCTURE ONLY (see velo_oracle.h).
 *
 * The paper (Sec. 2.3.1, last paragraph) finds PVs as clusters in a
 * histogram of the tracks' points of closest approach to the beamline, and
 * fits every candidate with every track, each track weighted for each
 * vertex, so that the candidates do not depend on one another's fits and
 * run in parallel.  It gives no binning, thresholds or weight function; the
 * readings taken here:
 *
 *   admission   a track enters if it is accepted by the quality cut, its
 *               slope is not along the beam (tx^2 + ty^2 >= 1e-6), and the
 *               variance of its beamline z, var = (tx^2 var_x + ty^2 var_y)
 *               / (tx^2 + ty^2)^2 (var_x, var_y of the beamline state), is
 *               at most max_var; and its z falls inside the histogram.
 *   histogram   n_bins bins of width bin_w from z0; a track in bin b adds 2
 *               to bin b and 1 to each neighbour (integer counts).
 *   candidates  bin b with count >= seed_min that is larger than every bin
 *               up to nms bins before it and at least every bin up to nms
 *               bins after it; seeded at the bin centre, in bin order, at
 *               most VO_MAX_PVS (more: VO_EV_PV_OVERFLOW, the first kept).
 *   limit       an event with more than VO_MAX_PV_TRACKS admitted tracks gets
 *               VO_EV_PV_OVERFLOW and no PVs.
 *   fit         n_iter rounds, every candidate from the previous round's
 *               positions of all candidates: chi2 = (z_i - z_v)^2 / var_i;
 *               Tukey weight r = (1 - chi2/chi2_cut)^2 below the cut, else
 *               0; a track's weight for vertex v is r_v times its share
 *               r_v / sum_u r_u; z_v = sum(w z / var) / sum(w / var) (kept
 *               when no track has weight).
 *   output      from the weights at the final positions: var_v =
 *               1 / sum(w / var), weight sum W_v = sum(w); a candidate is a
 *               PV if W_v >= min_weight.  PVs in candidate (z) order.
 *
 * Sums run over tracks in their slot order and over candidates in candidate
 * order; binary32 throughout, in the order written.
 */
#include "velo_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

void velo_oracle_pv_params_default(vo_pv_params* p)
{
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

/* admitted tracks of one event, in slot order */
static int32_t admit(const uint64_t base, uint32_t nt, const float* sz, const float* stx,
                     const float* sty, const float* cov_x, const float* cov_y,
                     const uint8_t* accepted, const vo_pv_params* P, float* tz, float* tv)
{
    int32_t n = 0;
    float zhi = P->z0 + P->bin_w * (float)P->n_bins;
    for (uint32_t t = 0; t < nt; ++t) {
        uint64_t s = base + t;
        if (!accepted[s]) continue;
        float tx = stx[s], ty = sty[s];
        float t2 = tx * tx + ty * ty;
        if (!(t2 >= 1e-6f)) continue;
        float var = (tx * tx * cov_x[3 * s] + ty * ty * cov_y[3 * s]) / (t2 * t2);
        if (!(var <= P->max_var) || !(var > 0.0f)) continue;
        float z = sz[s];
        if (!(z >= P->z0 && z < zhi)) continue;
        tz[n] = z;
        tv[n] = var;
        n++;
    }
    return n;
}

static float tukey(float z, float var, float zv, float cut)
{
    float d = z - zv;
    float c = (d * d) / var;
    if (!(c < cut)) return 0.0f;
    float q = 1.0f - c / cut;
    return q * q;
}

/* one event: returns its status (0 or VO_EV_PV_OVERFLOW) */
static uint32_t pv_event(const float* tz, const float* tv, int32_t n, const vo_pv_params* P,
                         uint32_t* n_pv, float* oz, float* ovar, float* ow)
{
    uint32_t st = 0;
    int32_t nb = P->n_bins;
    uint32_t* H = (uint32_t*)calloc((size_t)nb, sizeof(uint32_t));
    for (int32_t i = 0; i < n; ++i) {
        int32_t b = (int32_t)floorf((tz[i] - P->z0) / P->bin_w);
        if (b < 0 || b >= nb) continue;
        H[b] += 2;
        if (b > 0) H[b - 1] += 1;
        if (b + 1 < nb) H[b + 1] += 1;
    }
    float cz[VO_MAX_PVS];
    int32_t nc = 0;
    for (int32_t b = 0; b < nb; ++b) {
        if (H[b] < (uint32_t)P->seed_min) continue;
        int peak = 1;
        for (int32_t c = b - P->nms; c < b && peak; ++c)
            if (c >= 0 && !(H[b] > H[c])) peak = 0;
        for (int32_t c = b + 1; c <= b + P->nms && peak; ++c)
            if (c < nb && !(H[b] >= H[c])) peak = 0;
        if (!peak) continue;
        if (nc == VO_MAX_PVS) { st = VO_EV_PV_OVERFLOW; break; }
        cz[nc++] = P->z0 + ((float)b + 0.5f) * P->bin_w;
    }
    free(H);

    float* S = (float*)malloc((size_t)(n ? n : 1) * sizeof(float));
    float nz[VO_MAX_PVS];
    for (int32_t it = 0; it <= P->n_iter; ++it) {
        /* shares of every track among the candidates at the current positions */
        for (int32_t i = 0; i < n; ++i) {
            float s = 0.0f;
            for (int32_t v = 0; v < nc; ++v) s = s + tukey(tz[i], tv[i], cz[v], P->chi2_cut);
            S[i] = s;
        }
        for (int32_t v = 0; v < nc; ++v) {
            float sa = 0.0f, saz = 0.0f, sw = 0.0f;
            for (int32_t i = 0; i < n; ++i) {
                float r = tukey(tz[i], tv[i], cz[v], P->chi2_cut);
                if (!(r > 0.0f)) continue;
                float w = r * (r / S[i]);
                float a = w / tv[i];
                sa = sa + a;
                saz = saz + a * tz[i];
                sw = sw + w;
            }
            if (it < P->n_iter) {
                nz[v] = sa > 0.0f ? saz / sa : cz[v];
            } else {
                /* after the last round: the outputs at the final positions */
                ovar[v] = sa > 0.0f ? 1.0f / sa : 0.0f;
                ow[v] = sw;
            }
        }
        if (it < P->n_iter)
            for (int32_t v = 0; v < nc; ++v) cz[v] = nz[v];
    }
    free(S);
    uint32_t k = 0;
    for (int32_t v = 0; v < nc; ++v) {
        if (!(ow[v] >= P->min_weight)) continue;
        oz[k] = cz[v];
        ovar[k] = ovar[v];
        ow[k] = ow[v];
        k++;
    }
    *n_pv = k;
    return st;
}

void velo_oracle_find_pvs(const uint64_t* offsets, uint32_t n_events, const uint32_t* n_tracks,
                          const float* sz, const float* stx, const float* sty,
                          const float* cov_x, const float* cov_y, const uint8_t* accepted,
                          const vo_pv_params* P, uint32_t* n_pv, float* pv_z, float* pv_var,
                          float* pv_w, uint32_t* pv_status)
{
    for (uint32_t e = 0; e < n_events; ++e) {
        uint64_t b = offsets[e], end = offsets[e + 1];
        uint32_t nt = n_tracks[e];
        uint32_t cap = end >= b ? (uint32_t)((end - b) / 3) : 0;
        if (nt > cap) nt = cap;
        float* tz = (float*)malloc((size_t)(nt ? nt : 1) * sizeof(float));
        float* tv = (float*)malloc((size_t)(nt ? nt : 1) * sizeof(float));
        int32_t n = admit(b / 3, nt, sz, stx, sty, cov_x, cov_y, accepted, P, tz, tv);
        float oz[VO_MAX_PVS], ov[VO_MAX_PVS], ow[VO_MAX_PVS];
        uint32_t k = 0;
        if (n > VO_MAX_PV_TRACKS)
            pv_status[e] = VO_EV_PV_OVERFLOW;   /* limit of the method's tables: no PVs */
        else
            pv_status[e] = pv_event(tz, tv, n, P, &k, oz, ov, ow);
        n_pv[e] = k;
        for (uint32_t j = 0; j < VO_MAX_PVS; ++j) {
            size_t o = (size_t)e * VO_MAX_PVS + j;
            pv_z[o] = j < k ? oz[j] : 0.0f;
            pv_var[o] = j < k ? ov[j] : 0.0f;
            pv_w[o] = j < k ? ow[j] : 0.0f;
        }
        free(tz);
        free(tv);
    }
}
