/*
 * velo_oracle_ut.c -- CPU oracle of the Velo-to-UT search windows.
 * TEST INFRASTRUCTURE ONLY (see velo_oracle.h).
 *
 * The paper (Sec. 2.3.2) describes the upstream tracker (UT) as four planes
 * of silicon strips, the outer two with vertical strips and the inner two
 * tilted by +5 and -5 degrees around z; most hits are single strips, so
 * there is no clustering; hits are decoded into regions and sorted so that
 * hits near an extrapolated Velo track are found quickly; Velo tracks are
 * extrapolated to the UT with the largest bending a particle of at least
 * 3 GeV can have between the Velo and the UT.  It gives no geometry,
 * format or window formula; the readings taken here:
 *
 *   geometry    planes k = 0..3 at z = 2327.5, 2372.5, 2597.5, 2642.5 mm,
 *               strip angles 0, +5, -5, 0 degrees; a strip measures
 *               u = x c_k + y s_k (c_k, s_k: the binary32 cosine and sine,
 *               0.9961947f and +-0.08715574f for the tilted planes);
 *               8192 strips of 0.1875 mm over u in [-768, 768): strip n has
 *               u = ((float)n + 0.5f) * 0.1875f - 768.0f (exact in binary32);
 *               every strip is cut into 14 sensors of 100 mm in y, sensor j
 *               covering y in [-700 + 100 j, -600 + 100 j).
 *   raw word    bits [0,13) strip, [13,17) sensor j (< 14), [17,19) plane,
 *               bits [19,32) zero; any order inside an event.
 *   regions     region r = 14 k + j; the hits of an event are sorted by
 *               the 19-bit word (plane, then sensor, then strip), so each
 *               region is a run sorted by u.  (The paper forms regions
 *               along x and sorts them along y; here the strips are long in
 *               y and the window is narrow in x, so regions follow y and
 *               are sorted along u.)
 *   status      a word with a sensor >= 14 or a high bit set: BAD_WORD; the
 *               same word twice: DUPLICATE (only when no other bit); more
 *               than VO_UT_MAX_HITS words: UT_OVERFLOW; offsets outside the
 *               usable-offsets rule of the pixel data: BAD_OFFSETS.  A
 *               flagged event has no UT hits and all its windows are empty.
 *   window      for every track accepted by the quality cut and every plane
 *               k, from the beamline state (x, y, z, tx, ty):
 *                 dz = z_k - z, xp = x + tx dz, yp = y + ty dz (straight: the
 *                 Velo is outside the field), up = xp c_k + yp s_k;
 *                 half width w_k = ((kick / p_min) (z_k - z_kick)) c_k + tol_u,
 *                 the largest x bending of a particle with p >= p_min for a
 *                 single transverse kick `kick` at z_kick, seen along u;
 *                 sensors j with yp + tol_y >= y_lo(j) and yp - tol_y < y_hi(j)
 *                 (at most two, in increasing j);
 *                 in each such region the hits with u - up within [-w_k, w_k],
 *                 i.e. lo = up - w_k <= u <= hi = up + w_k: the index of the
 *                 first one in the event's sorted hits and their number.
 *   output      win[8 slot + 2 k + i] = first | count << 16 for the i-th
 *               sensor of plane k (0 when there is none); tracks that are
 *               not accepted get zeros.
 *
 * Binary32 throughout, in the order written; the sort is a library sort of
 * distinct integers and the windows are linear scans of the regions.
 */
#include "velo_oracle.h"

#include <stdlib.h>
#include <string.h>

static const float UT_Z[4] = {2327.5f, 2372.5f, 2597.5f, 2642.5f};
static const float UT_C[4] = {1.0f, 0.9961947f, 0.9961947f, 1.0f};
static const float UT_S[4] = {0.0f, 0.08715574f, -0.08715574f, 0.0f};

void velo_oracle_ut_params_default(vo_ut_params* p)
{
    p->p_min_mev = 3000.0f;
    p->kick_mev = 45.0f;
    p->z_kick = 1000.0f;
    p->tol_u = 1.0f;
    p->tol_y = 10.0f;
}

float velo_oracle_ut_strip_u(uint32_t strip)
{
    return ((float)strip + 0.5f) * 0.1875f - 768.0f;
}

static int cmp_u32(const void* a, const void* b)
{
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return x < y ? -1 : x > y;
}

/* decode and sort one event's words into sorted[0..n); returns its status */
static uint32_t ut_event(const uint32_t* w, uint32_t n, uint32_t* sorted, uint32_t* region)
{
    memset(region, 0, 57 * sizeof(uint32_t));
    if (n > VO_UT_MAX_HITS) return VO_EV_UT_OVERFLOW;
    uint32_t st = 0;
    for (uint32_t i = 0; i < n; ++i)
        if ((w[i] >> 19) != 0u || ((w[i] >> 13) & 15u) >= VO_UT_SECTORS) st |= VO_EV_BAD_WORD;
    if (st) return st;
    uint32_t* tmp = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
    memcpy(tmp, w, n * sizeof(uint32_t));
    qsort(tmp, n, sizeof(uint32_t), cmp_u32);
    for (uint32_t i = 1; i < n && !st; ++i)
        if (tmp[i] == tmp[i - 1]) st = VO_EV_DUPLICATE;
    if (!st) {
        memcpy(sorted, tmp, n * sizeof(uint32_t));
        /* region r starts at the first word whose region index is >= r */
        for (uint32_t r = 0; r <= VO_UT_REGIONS; ++r) {
            uint32_t i = 0;
            while (i < n && ((tmp[i] >> 17) * VO_UT_SECTORS + ((tmp[i] >> 13) & 15u)) < r) ++i;
            region[r] = i;
        }
    }
    free(tmp);
    return st;
}

void velo_oracle_ut(const uint32_t* ut_words, const uint64_t* ut_offsets, uint32_t n_events,
                    uint64_t n_ut, const uint64_t* offsets, uint64_t n_pixels, const uint32_t* n_tracks,
                    const float* sx, const float* sy, const float* sz, const float* stx,
                    const float* sty, const uint8_t* accepted, const vo_ut_params* P,
                    uint32_t* sorted, uint32_t* region, uint32_t* ut_status, uint32_t* win)
{
    const float dtx = P->kick_mev / P->p_min_mev;
    float w[4];
    for (int k = 0; k < 4; ++k) w[k] = (dtx * (UT_Z[k] - P->z_kick)) * UT_C[k] + P->tol_u;
    uint64_t before = 0;
    for (uint32_t e = 0; e < n_events; ++e) {
        uint64_t ub = ut_offsets[e], ue = ut_offsets[e + 1];
        int usable = ub <= ue && ue <= n_ut && ub >= before;
        if (ub > before) before = ub;
        uint32_t* reg = region + 57 * (size_t)e;
        uint32_t st;
        if (!usable) {
            memset(reg, 0, 57 * sizeof(uint32_t));
            st = VO_EV_BAD_OFFSETS;
        } else {
            st = ut_event(ut_words + ub, (uint32_t)(ue - ub), sorted + ub, reg);
        }
        ut_status[e] = st;
        /* the event's track slots: none if its pixel offsets are inverted or
           run past the pixel buffer, else the count clamped to a third of
           its words (like the fit) */
        uint64_t b = offsets[e], end = offsets[e + 1];
        uint32_t nt = n_tracks[e];
        uint32_t cap = (end >= b && end <= n_pixels) ? (uint32_t)((end - b) / 3) : 0;
        if (nt > cap) nt = cap;
        const uint32_t* hs = sorted + ub;
        for (uint32_t t = 0; t < nt; ++t) {
            uint64_t s = b / 3 + t;
            uint32_t* o = win + 8 * s;
            memset(o, 0, 8 * sizeof(uint32_t));
            if (st || !accepted[s]) continue;
            for (int k = 0; k < 4; ++k) {
                float dz = UT_Z[k] - sz[s];
                float xp = sx[s] + stx[s] * dz;
                float yp = sy[s] + sty[s] * dz;
                float up = xp * UT_C[k] + yp * UT_S[k];
                float lo = up - w[k], hi = up + w[k];
                int i = 0;
                for (uint32_t j = 0; j < VO_UT_SECTORS && i < 2; ++j) {
                    float ylo = -700.0f + 100.0f * (float)j, yhi = ylo + 100.0f;
                    if (!(yp + P->tol_y >= ylo && yp - P->tol_y < yhi)) continue;
                    uint32_t r = (uint32_t)k * VO_UT_SECTORS + j;
                    uint32_t first = reg[r + 1], count = 0;
                    for (uint32_t h = reg[r]; h < reg[r + 1]; ++h) {
                        float u = velo_oracle_ut_strip_u(hs[h] & 8191u);
                        if (u >= lo && u <= hi) {
                            if (count == 0) first = h;
                            count++;
                        }
                    }
                    if (count == 0) first = 0;
                    o[2 * k + i] = first | count << 16;
                    i++;
                }
            }
        }
    }
}
