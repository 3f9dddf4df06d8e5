/*
 * velo_oracle.c -- plain, slow, obviously correct CPU oracle of the VELO
 * reconstruction path.  TEST INFRASTRUCTURE ONLY (see velo_oracle.h).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC
 * All floating point is binary32, evaluated in the order written.
 */
#include "velo_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Detector geometry (Sec. 2.3.1: 26 planes of pixel sensors).  The plane
   positions, pitch and hole are the detector model of this project: planes
   evenly spaced from z = -280 mm to +750 mm, 1536 x 1536 pixels of 55 um
   centred on the beam, pixels with centre radius < 5.1 mm inactive. */

float velo_oracle_layer_z(int32_t l)
{
    return (float)(-280.0 + 1030.0 * (double)l / 25.0);
}

static int in_hole(uint32_t col, uint32_t row)
{
    int64_t dc = 2 * (int64_t)col - 1535, dr = 2 * (int64_t)row - 1535;
    return dc * dc + dr * dr <= 34393;
}

/* ------------------------------------------------------------------ */
/* Clustering: connected-component labelling of the fired pixels of each
   plane (Sec. 2.3.1, first paragraph).  Reading: two pixels are connected
   when they touch by side or corner (8-connectivity).  Each component gives
   one hit: key = smallest pixel address, charge-weighted mean of the pixel
   centres from integer sums, size and charge in `aux`. */

typedef struct { uint32_t addr; uint32_t q; } opix;   /* addr = row << 11 | col */

static int cmp_opix(const void* a, const void* b)
{
    uint32_t x = ((const opix*)a)->addr, y = ((const opix*)b)->addr;
    return (x > y) - (x < y);
}

static int64_t find_addr(const opix* p, int64_t n, uint32_t addr)
{
    int64_t lo = 0, hi = n;           /* first index with p[i].addr >= addr */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (p[mid].addr < addr) lo = mid + 1; else hi = mid;
    }
    return (lo < n && p[lo].addr == addr) ? lo : -1;
}

static uint32_t cluster_event(const uint32_t* w, uint32_t n, uint64_t base,
                              float* x, float* y, uint32_t* key, uint32_t* aux,
                              uint32_t* lstart, uint32_t* lnh, uint32_t* nh)
{
    uint32_t st = 0;
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t col = w[i] & 0x7FFu, row = (w[i] >> 11) & 0x7FFu;
        uint32_t lay = (w[i] >> 22) & 31u, q = (w[i] >> 27) & 15u, top = w[i] >> 31;
        int valid = !top && lay < VO_N_LAYERS && row < 1536u && col < 1536u && q >= 1u;
        if (!valid) st |= VO_EV_BAD_WORD;
        else if (in_hole(col, row)) st |= VO_EV_HOLE;
        if (i > 0 && lay < ((w[i - 1] >> 22) & 31u)) st |= VO_EV_LAYER_ORDER;
    }
    memset(lstart, 0, 27 * sizeof(uint32_t));
    memset(lnh, 0, 26 * sizeof(uint32_t));
    *nh = 0;
    if (st) return st;

    /* words are grouped by ascending layer: layer l = [lstart[l], lstart[l+1]) */
    uint32_t cnt[27] = {0};
    for (uint32_t i = 0; i < n; ++i) cnt[((w[i] >> 22) & 31u) + 1]++;
    for (int l = 0; l < 26; ++l) cnt[l + 1] += cnt[l];
    uint32_t ls[27];
    for (int l = 0; l <= 26; ++l) ls[l] = cnt[l];

    opix* p = (opix*)malloc((n ? n : 1) * sizeof(opix));
    unsigned char* seen = (unsigned char*)malloc(n ? n : 1);
    int64_t* stack = (int64_t*)malloc((n ? n : 1) * sizeof(int64_t));
    for (uint32_t i = 0; i < n; ++i) {
        p[i].addr = w[i] & 0x3FFFFFu;
        p[i].q = (w[i] >> 27) & 15u;
    }
    /* sort each layer by address; equal neighbours are duplicated pixels */
    for (int l = 0; l < 26; ++l) {
        opix* s = p + ls[l];
        uint32_t m = ls[l + 1] - ls[l];
        qsort(s, m, sizeof(opix), cmp_opix);
        for (uint32_t i = 1; i < m; ++i)
            if (s[i].addr == s[i - 1].addr) st |= VO_EV_DUPLICATE;
    }
    if (st) { free(p); free(seen); free(stack); return st; }

    memset(seen, 0, n);
    uint32_t total = 0;
    for (int l = 0; l < 26; ++l) {
        opix* s = p + ls[l];
        int64_t m = (int64_t)(ls[l + 1] - ls[l]);
        uint32_t nc = 0;
        for (int64_t i = 0; i < m; ++i) {
            if (seen[ls[l] + i]) continue;
            /* new component; i is its smallest address since every smaller
               pixel already belongs to an earlier component */
            uint32_t Q = 0, SC = 0, SR = 0, N = 0;
            int64_t sp = 0;
            stack[sp++] = i;
            seen[ls[l] + i] = 1;
            while (sp) {
                int64_t k = stack[--sp];
                uint32_t col = s[k].addr & 0x7FFu, row = s[k].addr >> 11, q = s[k].q;
                Q += q; SC += q * col; SR += q * row; N += 1;
                for (int dr = -1; dr <= 1; ++dr)
                    for (int dc = -1; dc <= 1; ++dc) {
                        if (!dr && !dc) continue;
                        int64_t rr = (int64_t)row + dr, cc = (int64_t)col + dc;
                        if (rr < 0 || cc < 0 || rr >= 1536 || cc >= 1536) continue;
                        int64_t j = find_addr(s, m, (uint32_t)(rr << 11 | cc));
                        if (j >= 0 && !seen[ls[l] + j]) { seen[ls[l] + j] = 1; stack[sp++] = j; }
                    }
            }
            uint64_t slot = base + ls[l] + nc;
            x[slot] = ((float)SC / (float)Q - 767.5f) * 0.055f;
            y[slot] = ((float)SR / (float)Q - 767.5f) * 0.055f;
            key[slot] = ((uint32_t)l << 22) | s[i].addr;
            aux[slot] = ((N < 65535u ? N : 65535u) << 16) | (Q < 65535u ? Q : 65535u);
            nc++;
        }
        lstart[l] = ls[l];
        lnh[l] = nc;
        total += nc;
    }
    lstart[26] = ls[26];
    *nh = total;
    free(p); free(seen); free(stack);
    return 0;
}

/* Usable offsets (reading of the per-event error convention): event e owns
   words [offsets[e], offsets[e+1]) only if offsets[e] <= offsets[e+1] <=
   n_pixels and no earlier offset exceeds offsets[e]; the word ranges of
   usable events are then disjoint.  Any other event is flagged
   VO_EV_BAD_OFFSETS and has no hits. */
uint32_t velo_oracle_cluster(const uint32_t* pixels, const uint64_t* offsets, uint32_t e0,
                             uint32_t e1, uint64_t n_pixels,
                             float* x, float* y, uint32_t* key, uint32_t* aux,
                             uint32_t* layer_start, uint32_t* layer_nhits,
                             uint32_t* n_hits, uint32_t* status)
{
    uint32_t all = 0;
    uint64_t before = 0;   /* largest of offsets[0 .. e-1] */
    for (uint32_t e = 0; e < e0; ++e)
        if (offsets[e] > before) before = offsets[e];
    for (uint32_t e = e0; e < e1; ++e) {
        uint64_t b = offsets[e], end = offsets[e + 1];
        int usable = b <= end && end <= n_pixels && b >= before;
        if (b > before) before = b;
        if (!usable) {
            status[e] = VO_EV_BAD_OFFSETS;
            memset(layer_start + 27 * (size_t)e, 0, 27 * sizeof(uint32_t));
            memset(layer_nhits + 26 * (size_t)e, 0, 26 * sizeof(uint32_t));
            n_hits[e] = 0;
        } else {
            status[e] = cluster_event(pixels + b, (uint32_t)(end - b), b, x, y, key, aux,
                                      layer_start + 27 * (size_t)e, layer_nhits + 26 * (size_t)e,
                                      n_hits + e);
        }
        all |= status[e];
    }
    return all;
}

/* ------------------------------------------------------------------ */
/* Track finding (Sec. 2.3.1, second paragraph): seeds of three hits on
   consecutive planes, extended plane by plane along straight lines.
   Readings taken here:
   - planes are visited from the last (z = +750 mm) to the first; at plane l
     the active tracks are first extended into l, then new seeds are formed
     from planes (l+2, l+1, l) with hits not used by any track;
   - a seed doublet keeps both slopes within max_t and the two hits at the
     same azimuth within asin(sqrt(sin2_phi)) (prompt tracks keep constant
     azimuth), tested without trigonometry; the third hit lies within
     sqrt(s_seed) of the doublet line;
   - a track takes the closest unused hit within sqrt(s_fwd) of its line;
   - conflicts are resolved greedily in ascending priority: seeds by
     (s, key1, key0, key2), extensions by (s, key of the track's first hit,
     key of the hit); a hit belongs to at most one track;
   - a track that finds no hit on max_skip+1 consecutive planes is closed. */

typedef struct { float s; uint32_t k1, k0, k2; uint32_t h0, h1, h2; } oseed;
typedef struct { float s; uint32_t kf, kh; uint32_t t, h; } oext;
typedef struct { uint32_t hit[26]; int32_t n, skip; } otrack;

static int cmp_seed(const void* a, const void* b)
{
    const oseed* u = (const oseed*)a; const oseed* v = (const oseed*)b;
    if (u->s != v->s) return u->s < v->s ? -1 : 1;
    if (u->k1 != v->k1) return u->k1 < v->k1 ? -1 : 1;
    if (u->k0 != v->k0) return u->k0 < v->k0 ? -1 : 1;
    if (u->k2 != v->k2) return u->k2 < v->k2 ? -1 : 1;
    return 0;
}

static int cmp_ext(const void* a, const void* b)
{
    const oext* u = (const oext*)a; const oext* v = (const oext*)b;
    if (u->s != v->s) return u->s < v->s ? -1 : 1;
    if (u->kf != v->kf) return u->kf < v->kf ? -1 : 1;
    if (u->kh != v->kh) return u->kh < v->kh ? -1 : 1;
    return 0;
}

typedef struct {
    const float *x, *y; const uint32_t* key;   /* event-relative views */
    float z[26];
} ev_hits;

typedef struct { uint32_t k; uint32_t i; } okey;
static int cmp_okey_desc(const void* a, const void* b)
{
    uint32_t ka = ((const okey*)a)->k, kb = ((const okey*)b)->k;
    return (ka < kb) - (ka > kb);
}

static void push_track(otrack** v, size_t* n, size_t* cap, const otrack* t)
{
    if (*n == *cap) { *cap = *cap ? 2 * *cap : 64; *v = (otrack*)realloc(*v, *cap * sizeof(otrack)); }
    (*v)[(*n)++] = *t;
}

static uint32_t find_event(const ev_hits* H, const uint32_t* ls, const uint32_t* lnh,
                           const vo_params* P, otrack** out, size_t* n_out)
{
    uint32_t n_all = ls[26];
    unsigned char* used = (unsigned char*)calloc(n_all ? n_all : 1, 1);
    otrack *act = NULL, *fin = NULL, *nxt = NULL;
    size_t n_act = 0, c_act = 0, n_fin = 0, c_fin = 0, n_nxt = 0, c_nxt = 0;
    oseed* seeds = NULL; size_t c_seeds = 0;
    oext* exts = NULL; size_t c_exts = 0;
    unsigned char* matched = NULL; uint32_t* match_hit = NULL;
    uint32_t st = 0;

    for (int l = 25; l >= 0 && !st; --l) {
        const float zl = H->z[l];
        uint32_t h_lo = ls[l], h_n = lnh[l];

        /* 1. extend the active tracks into plane l */
        size_t n_ext = 0;
        for (size_t t = 0; t < n_act; ++t) {
            uint32_t a = act[t].hit[act[t].n - 1], b = act[t].hit[act[t].n - 2];
            float za = H->z[H->key[a] >> 22], zb = H->z[H->key[b] >> 22];
            float dza = za - zb;
            float txf = (H->x[a] - H->x[b]) / dza;
            float tyf = (H->y[a] - H->y[b]) / dza;
            float d = zl - za;
            float xp = H->x[a] + txf * d;
            float yp = H->y[a] + tyf * d;
            for (uint32_t i = 0; i < h_n; ++i) {
                uint32_t h = h_lo + i;
                if (used[h]) continue;
                float dx = H->x[h] - xp, dy = H->y[h] - yp;
                float s = dx * dx + dy * dy;
                if (!(s <= P->s_fwd)) continue;
                if (n_ext >= VO_MAX_CANDIDATES) { st = VO_EV_OVERFLOW; break; }
                if (n_ext == c_exts) { c_exts = c_exts ? 2 * c_exts : 256; exts = (oext*)realloc(exts, c_exts * sizeof(oext)); }
                exts[n_ext].s = s; exts[n_ext].kf = H->key[act[t].hit[0]]; exts[n_ext].kh = H->key[h];
                exts[n_ext].t = (uint32_t)t; exts[n_ext].h = h;
                n_ext++;
            }
            if (st) break;
        }
        if (st) break;
        qsort(exts, n_ext, sizeof(oext), cmp_ext);
        matched = (unsigned char*)realloc(matched, n_act ? n_act : 1);
        match_hit = (uint32_t*)realloc(match_hit, (n_act ? n_act : 1) * sizeof(uint32_t));
        memset(matched, 0, n_act ? n_act : 1);
        for (size_t k = 0; k < n_ext; ++k) {
            if (matched[exts[k].t] || used[exts[k].h]) continue;
            matched[exts[k].t] = 1; match_hit[exts[k].t] = exts[k].h; used[exts[k].h] = 1;
        }
        n_nxt = 0;
        for (size_t t = 0; t < n_act; ++t) {
            otrack tr = act[t];
            if (matched[t]) { tr.hit[tr.n++] = match_hit[t]; tr.skip = 0; }
            else tr.skip += 1;
            if (tr.skip > P->max_skip) push_track(&fin, &n_fin, &c_fin, &tr);
            else push_track(&nxt, &n_nxt, &c_nxt, &tr);
        }

        /* 2. seeds on planes (l+2, l+1, l) */
        if (l <= 23) {
            size_t n_seed = 0;
            uint32_t a0 = ls[l + 2], n0 = lnh[l + 2], a1 = ls[l + 1], n1 = lnh[l + 1];
            float z0 = H->z[l + 2], z1 = H->z[l + 1], z2 = zl;
            for (uint32_t j1 = 0; j1 < n1 && !st; ++j1) {
                uint32_t h1 = a1 + j1;
                if (used[h1]) continue;
                float x1 = H->x[h1], y1 = H->y[h1];
                for (uint32_t j0 = 0; j0 < n0 && !st; ++j0) {
                    uint32_t h0 = a0 + j0;
                    if (used[h0]) continue;
                    float x0 = H->x[h0], y0 = H->y[h0];
                    float dz = z1 - z0;
                    float tx = (x1 - x0) / dz;
                    float ty = (y1 - y0) / dz;
                    if (!(fabsf(tx) <= P->max_t && fabsf(ty) <= P->max_t)) continue;
                    float cr = x0 * y1 - y0 * x1;
                    float r0 = x0 * x0 + y0 * y0;
                    float r1 = x1 * x1 + y1 * y1;
                    if (!(cr * cr <= (P->sin2_phi * r0) * r1)) continue;
                    if (!(x0 * x1 + y0 * y1 > 0.0f)) continue;
                    float d = z2 - z1;
                    float xp = x1 + tx * d;
                    float yp = y1 + ty * d;
                    for (uint32_t i = 0; i < h_n; ++i) {
                        uint32_t h2 = h_lo + i;
                        if (used[h2]) continue;
                        float dx = H->x[h2] - xp, dy = H->y[h2] - yp;
                        float s = dx * dx + dy * dy;
                        if (!(s <= P->s_seed)) continue;
                        if (n_seed >= VO_MAX_CANDIDATES) { st = VO_EV_OVERFLOW; break; }
                        if (n_seed == c_seeds) { c_seeds = c_seeds ? 2 * c_seeds : 256; seeds = (oseed*)realloc(seeds, c_seeds * sizeof(oseed)); }
                        oseed* S = &seeds[n_seed++];
                        S->s = s; S->k1 = H->key[h1]; S->k0 = H->key[h0]; S->k2 = H->key[h2];
                        S->h0 = h0; S->h1 = h1; S->h2 = h2;
                    }
                }
            }
            if (st) break;
            qsort(seeds, n_seed, sizeof(oseed), cmp_seed);
            for (size_t k = 0; k < n_seed; ++k) {
                oseed* S = &seeds[k];
                if (used[S->h0] || used[S->h1] || used[S->h2]) continue;
                used[S->h0] = used[S->h1] = used[S->h2] = 1;
                otrack tr;
                tr.hit[0] = S->h0; tr.hit[1] = S->h1; tr.hit[2] = S->h2; tr.n = 3; tr.skip = 0;
                push_track(&nxt, &n_nxt, &c_nxt, &tr);
            }
        }
        otrack* tmp = act; act = nxt; nxt = tmp;
        size_t tc = c_act; c_act = c_nxt; c_nxt = tc;
        n_act = n_nxt;
    }
    if (!st) {
        for (size_t t = 0; t < n_act; ++t) push_track(&fin, &n_fin, &c_fin, &act[t]);
        /* output order: decreasing key of the first (highest-z) hit */
        okey* ord = (okey*)malloc((n_fin ? n_fin : 1) * sizeof(okey));
        for (size_t t = 0; t < n_fin; ++t) { ord[t].k = H->key[fin[t].hit[0]]; ord[t].i = (uint32_t)t; }
        qsort(ord, n_fin, sizeof(okey), cmp_okey_desc);
        otrack* sorted = (otrack*)malloc((n_fin ? n_fin : 1) * sizeof(otrack));
        for (size_t t = 0; t < n_fin; ++t) sorted[t] = fin[ord[t].i];
        free(ord); free(fin);
        *out = sorted; *n_out = n_fin;
    } else {
        free(fin); *out = NULL; *n_out = 0;
    }
    free(used); free(act); free(nxt); free(seeds); free(exts); free(matched); free(match_hit);
    return st;
}

void velo_oracle_find_tracks(const float* x, const float* y, const uint32_t* key,
                             const uint32_t* layer_start, const uint32_t* layer_nhits,
                             const uint64_t* offsets, uint32_t n_events, const vo_params* p,
                             uint32_t* n_tracks, uint8_t* trk_nhits, uint32_t* hit_idx,
                             uint32_t* trk_status)
{
    for (uint32_t e = 0; e < n_events; ++e) {
        uint64_t b = offsets[e];
        ev_hits H;
        H.x = x + b; H.y = y + b; H.key = key + b;
        for (int l = 0; l < 26; ++l) H.z[l] = velo_oracle_layer_z(l);
        otrack* tr = NULL; size_t nt = 0;
        trk_status[e] = find_event(&H, layer_start + 27 * (size_t)e, layer_nhits + 26 * (size_t)e,
                                   p, &tr, &nt);
        uint64_t base = b / 3;
        n_tracks[e] = (uint32_t)nt;
        for (size_t t = 0; t < nt; ++t) {
            trk_nhits[base + t] = (uint8_t)tr[t].n;
            for (int j = 0; j < 26; ++j)
                hit_idx[(base + t) * 26 + j] = j < tr[t].n ? tr[t].hit[j] : 0u;
        }
        free(tr);
    }
}

/* ------------------------------------------------------------------ */
/* Track fit (Sec. 2.3.1, third paragraph): a simple Kalman filter per
   projection, x and y independent, with multiple-scattering noise computed
   for a constant transverse momentum pt0 (400 MeV in the paper).  Readings:
   - state (u, t = du/dz) per projection, hits visited in decreasing z;
     initialised at the second hit from the first two hits;
   - scattering: slope variance grows by (dl planes) * 13.6^2 * X/X0 / p^2
     before each transport, with p = pt0 * sqrt(1+t2)/sqrt(t2), t2 the squared
     slope of the first two hits, i.e. 184.96 * X/X0 / pt0^2 * t2 / (1 + t2);
   - the final state (at the lowest-z hit) gets the slope noise of that one
     plane and is transported to the point of closest approach to the
     beamline, taken as the z axis (Sec. 2.3.1, fourth paragraph);
   - chi2 = sum of normalised residuals of both projections, ndof = 2n - 4;
   - plain track-quality cut: chi2/ndof <= qc4 (n >= 4) or <= qc3 (n = 3). */

typedef struct { float u, t, c00, c01, c11, chi2; } okf;

static okf kf_project(const float* m, const float* z, const int32_t* lay, int32_t n,
                      float sig2, float ms2)
{
    okf s;
    float d = z[1] - z[0];
    s.u = m[1];
    s.t = (m[1] - m[0]) / d;
    s.c00 = sig2;
    s.c01 = sig2 / d;
    s.c11 = (2.0f * sig2) / (d * d);
    s.chi2 = 0.0f;
    for (int32_t i = 2; i < n; ++i) {
        float dz = z[i] - z[i - 1];
        float dl = (float)(lay[i - 1] - lay[i]);
        s.c11 = s.c11 + dl * ms2;
        s.u = s.u + s.t * dz;
        s.c00 = s.c00 + 2.0f * dz * s.c01 + dz * dz * s.c11;
        s.c01 = s.c01 + dz * s.c11;
        float r = m[i] - s.u;
        float S = s.c00 + sig2;
        float k0 = s.c00 / S;
        float k1 = s.c01 / S;
        s.u = s.u + k0 * r;
        s.t = s.t + k1 * r;
        s.c11 = s.c11 - k1 * s.c01;
        s.c01 = s.c01 - k0 * s.c01;
        s.c00 = s.c00 - k0 * s.c00;
        s.chi2 = s.chi2 + (r * r) / S;
    }
    return s;
}

static void kf_transport(okf* s, float dz)
{
    s->u = s->u + s->t * dz;
    s->c00 = s->c00 + 2.0f * dz * s->c01 + dz * dz * s->c11;
    s->c01 = s->c01 + dz * s->c11;
}

/* the filter of both projections and the beamline transport, for a given
   slope variance added per plane crossed (ms2) */
static int32_t fit_points_ms2(const float* hx, const float* hy, const float* hz,
                              const int32_t* hlayer, int32_t n, float sig2, float ms2,
                              int through_planes,
                              float* out5, float* cov_x, float* cov_y, float* chi2)
{
    okf sx = kf_project(hx, hz, hlayer, n, sig2, ms2);
    okf sy = kf_project(hy, hz, hlayer, n, sig2, ms2);
    float zl = hz[n - 1];
    float num = sx.u * sx.t + sy.u * sy.t;
    float den = sx.t * sx.t + sy.t * sy.t;
    float dzb = den < 1e-12f ? 0.0f : -(num / den);
    /* the particle scattered in the plane of the last hit before reaching it
       from the beamline side: one plane of slope noise before the transport */
    sx.c11 = sx.c11 + ms2;
    sy.c11 = sy.c11 + ms2;
    if (through_planes) {
        /* and in every plane it crossed between the beamline point and the
           last hit: transport plane by plane towards lower z, one plane of
           slope noise at each, then the rest of the way */
        float zb = zl + dzb, zc = zl;
        for (int32_t l = hlayer[n - 1] - 1; l >= 0; --l) {
            float zp = velo_oracle_layer_z(l);
            if (!(zp > zb)) break;
            kf_transport(&sx, zp - zc);
            kf_transport(&sy, zp - zc);
            sx.c11 = sx.c11 + ms2;
            sy.c11 = sy.c11 + ms2;
            zc = zp;
        }
        kf_transport(&sx, zb - zc);
        kf_transport(&sy, zb - zc);
    } else {
        kf_transport(&sx, dzb);
        kf_transport(&sy, dzb);
    }
    out5[0] = sx.u; out5[1] = sy.u; out5[2] = zl + dzb; out5[3] = sx.t; out5[4] = sy.t;
    cov_x[0] = sx.c00; cov_x[1] = sx.c01; cov_x[2] = sx.c11;
    cov_y[0] = sy.c00; cov_y[1] = sy.c01; cov_y[2] = sy.c11;
    *chi2 = sx.chi2 + sy.chi2;
    return 2 * n - 4;
}

int32_t velo_oracle_fit_points(const float* hx, const float* hy, const float* hz,
                               const int32_t* hlayer, int32_t n, const vo_params* p,
                               float* out5, float* cov_x, float* cov_y, float* chi2)
{
    float sig2 = p->sigma_meas * p->sigma_meas;
    float d = hz[1] - hz[0];
    float tx0 = (hx[1] - hx[0]) / d;
    float ty0 = (hy[1] - hy[0]) / d;
    float t2 = tx0 * tx0 + ty0 * ty0;
    float kms = (184.96f * p->x_over_x0) / (p->pt0_mev * p->pt0_mev);
    float ms2 = (kms * t2) / (1.0f + t2);
    return fit_points_ms2(hx, hy, hz, hlayer, n, sig2, ms2, 0, out5, cov_x, cov_y, chi2);
}

/* Velo-only filter with a measured momentum (Sec. 2.3.5: the Velo segment
   fitted with the momentum estimated from the full track).  Reading: the
   same filter, with the slope variance per plane crossed from the track's
   own momentum, 13.6^2 X/X0 / p^2 (Highland without the logarithm), and the
   transport to the beamline point taken plane by plane through the planes
   between it and the last hit, with that noise at each (the impact
   parameter is made there); a momentum that is not a positive finite number
   falls back to the constant transverse-momentum fit. */
int32_t velo_oracle_fit_points_p(const float* hx, const float* hy, const float* hz,
                                 const int32_t* hlayer, int32_t n, float p_mev, const vo_params* p,
                                 float* out5, float* cov_x, float* cov_y, float* chi2)
{
    if (!(p_mev > 0.0f && p_mev <= 3.0e38f))
        return velo_oracle_fit_points(hx, hy, hz, hlayer, n, p, out5, cov_x, cov_y, chi2);
    float sig2 = p->sigma_meas * p->sigma_meas;
    float ms2 = (184.96f * p->x_over_x0) / (p_mev * p_mev);
    return fit_points_ms2(hx, hy, hz, hlayer, n, sig2, ms2, 1, out5, cov_x, cov_y, chi2);
}

void velo_oracle_fit(const float* x, const float* y, const uint32_t* key,
                     const uint64_t* offsets, uint32_t n_events,
                     const uint32_t* n_tracks, const uint8_t* trk_nhits, const uint32_t* hit_idx,
                     const vo_params* p,
                     float* sx, float* sy, float* sz, float* stx, float* sty,
                     float* cov_x, float* cov_y, float* chi2, int32_t* ndof, uint8_t* accepted)
{
    velo_oracle_fit_momentum(x, y, key, offsets, n_events, n_tracks, trk_nhits, hit_idx, NULL, p,
                             sx, sy, sz, stx, sty, cov_x, cov_y, chi2, ndof, accepted);
}

void velo_oracle_fit_momentum(const float* x, const float* y, const uint32_t* key,
                              const uint64_t* offsets, uint32_t n_events,
                              const uint32_t* n_tracks, const uint8_t* trk_nhits,
                              const uint32_t* hit_idx, const float* p_mev, const vo_params* p,
                              float* sx, float* sy, float* sz, float* stx, float* sty,
                              float* cov_x, float* cov_y, float* chi2, int32_t* ndof,
                              uint8_t* accepted)
{
    for (uint32_t e = 0; e < n_events; ++e) {
        uint64_t b = offsets[e], base = b / 3;
        for (uint32_t t = 0; t < n_tracks[e]; ++t) {
            uint64_t slot = base + t;
            int32_t n = trk_nhits[slot];
            float hx[26], hy[26], hz[26];
            int32_t hl[26];
            for (int32_t j = 0; j < n; ++j) {
                uint64_t h = b + hit_idx[slot * 26 + j];
                hx[j] = x[h]; hy[j] = y[h];
                hl[j] = (int32_t)(key[h] >> 22);
                hz[j] = velo_oracle_layer_z(hl[j]);
            }
            float o5[5], c;
            int32_t nd = p_mev
                ? velo_oracle_fit_points_p(hx, hy, hz, hl, n, p_mev[slot], p, o5, cov_x + 3 * slot,
                                           cov_y + 3 * slot, &c)
                : velo_oracle_fit_points(hx, hy, hz, hl, n, p, o5, cov_x + 3 * slot,
                                         cov_y + 3 * slot, &c);
            sx[slot] = o5[0]; sy[slot] = o5[1]; sz[slot] = o5[2];
            stx[slot] = o5[3]; sty[slot] = o5[4];
            chi2[slot] = c; ndof[slot] = nd;
            float r = c / (float)nd;
            accepted[slot] = (uint8_t)(n >= 4 ? (r <= p->qc4) : (r <= p->qc3));
        }
    }
}
