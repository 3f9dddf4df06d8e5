/*
 * velo_oracle_mlp.c -- CPU oracle of the learned track-quality classifier.
 * TEST INFRASTRUCTURE ONLY (see velo_oracle.h).
 *
 * The classifier is not part of the paper; it is this project's learned
 * replacement of the plain chi2/hit-count cut after the simple Kalman fit
 * (Sec. 2.3.1).  Definitions:
 *   features f (8): chi2/ndof, n hits, missed planes = (l_first - l_last + 1) - n,
 *                   tx, ty, eta = asinh(1/sqrt(tx^2+ty^2)), z of the first and
 *                   of the last hit plane
 *   standardised    g = (f - mean) / std
 *   network         h1 = relu(W1 g + b1) (32), h2 = relu(W2 h1 + b2) (32),
 *                   z = w3 . h2 + b3, p = sigmoid(z)
 *   loss            mean binary cross-entropy with logits:
 *                   max(z,0) - z y + log(1 + exp(-|z|))
 *   parameters      flat, 1377 values: W1[32][8], b1[32], W2[32][32], b2[32],
 *                   w3[32], b3
 * The double-precision forward/backward is the reference of the GPU's FP32
 * training kernels.  The bfloat16 forward emulates the GPU inference
 * precision (inputs, weights and hidden activations rounded to bfloat16
 * with round-to-nearest-even, products exact, sums in binary32), so the
 * accept decision z >= threshold is taken in the same precision on both
 * sides.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "velo_oracle.h"

#define NF 8
#define NH 32
#define O_W1 0
#define O_B1 (O_W1 + NH * NF)
#define O_W2 (O_B1 + NH)
#define O_B2 (O_W2 + NH * NH)
#define O_W3 (O_B2 + NH)
#define O_B3 (O_W3 + NH)
#define NPARAM (O_B3 + 1)

int32_t velo_oracle_mlp_nparams(void) { return NPARAM; }

/* Features of every track of events [0, n_events) at its slot (cap x 8). */
void velo_oracle_features(const uint32_t* key, const uint64_t* offsets, uint32_t n_events,
                          const uint32_t* n_tracks, const uint8_t* trk_nhits, const uint32_t* hit_idx,
                          const float* stx, const float* sty, const float* chi2, const int32_t* ndof,
                          double* feat)
{
    for (uint32_t e = 0; e < n_events; ++e) {
        uint64_t b = offsets[e], base = b / 3;
        for (uint32_t t = 0; t < n_tracks[e]; ++t) {
            uint64_t slot = base + t;
            int32_t n = trk_nhits[slot];
            int32_t lf = (int32_t)(key[b + hit_idx[slot * 26]] >> 22);
            int32_t ll = (int32_t)(key[b + hit_idx[slot * 26 + n - 1]] >> 22);
            double tx = stx[slot], ty = sty[slot];
            double t2 = tx * tx + ty * ty;
            if (t2 < 1e-12) t2 = 1e-12;
            double* f = feat + 8 * slot;
            f[0] = (double)chi2[slot] / (double)ndof[slot];
            f[1] = n;
            f[2] = (double)((lf - ll + 1) - n);
            f[3] = tx;
            f[4] = ty;
            f[5] = asinh(1.0 / sqrt(t2));
            f[6] = velo_oracle_layer_z(lf);
            f[7] = velo_oracle_layer_z(ll);
        }
    }
}

static double relu(double x) { return x > 0 ? x : 0; }

/* Mean loss and its gradient over n standardised samples (double). */
double velo_oracle_mlp_fwd_bwd(const double* p, const double* g, const double* y, int64_t n,
                               double* grad)
{
    memset(grad, 0, NPARAM * sizeof(double));
    double loss = 0;
    for (int64_t s = 0; s < n; ++s) {
        const double* x = g + NF * s;
        double h1[NH], h2[NH], z = p[O_B3];
        for (int i = 0; i < NH; ++i) {
            double a = p[O_B1 + i];
            for (int k = 0; k < NF; ++k) a += p[O_W1 + NF * i + k] * x[k];
            h1[i] = relu(a);
        }
        for (int i = 0; i < NH; ++i) {
            double a = p[O_B2 + i];
            for (int k = 0; k < NH; ++k) a += p[O_W2 + NH * i + k] * h1[k];
            h2[i] = relu(a);
        }
        for (int i = 0; i < NH; ++i) z += p[O_W3 + i] * h2[i];
        loss += (z > 0 ? z : 0) - z * y[s] + log1p(exp(-fabs(z)));
        double dz = (1.0 / (1.0 + exp(-z)) - y[s]) / (double)n;
        double dh2[NH], dh1[NH];
        grad[O_B3] += dz;
        for (int i = 0; i < NH; ++i) {
            grad[O_W3 + i] += dz * h2[i];
            dh2[i] = h2[i] > 0 ? dz * p[O_W3 + i] : 0;
        }
        for (int k = 0; k < NH; ++k) {
            double a = 0;
            for (int i = 0; i < NH; ++i) a += p[O_W2 + NH * i + k] * dh2[i];
            dh1[k] = h1[k] > 0 ? a : 0;
        }
        for (int i = 0; i < NH; ++i) {
            grad[O_B2 + i] += dh2[i];
            for (int k = 0; k < NH; ++k) grad[O_W2 + NH * i + k] += dh2[i] * h1[k];
            grad[O_B1 + i] += dh1[i];
            for (int k = 0; k < NF; ++k) grad[O_W1 + NF * i + k] += dh1[i] * x[k];
        }
    }
    return loss / (double)(n > 0 ? n : 1);
}

/* Logits in double of n standardised samples. */
void velo_oracle_mlp_forward(const double* p, const double* g, int64_t n, double* z)
{
    for (int64_t s = 0; s < n; ++s) {
        const double* x = g + NF * s;
        double h1[NH], h2[NH], o = p[O_B3];
        for (int i = 0; i < NH; ++i) {
            double a = p[O_B1 + i];
            for (int k = 0; k < NF; ++k) a += p[O_W1 + NF * i + k] * x[k];
            h1[i] = relu(a);
        }
        for (int i = 0; i < NH; ++i) {
            double a = p[O_B2 + i];
            for (int k = 0; k < NH; ++k) a += p[O_W2 + NH * i + k] * h1[k];
            h2[i] = relu(a);
        }
        for (int i = 0; i < NH; ++i) o += p[O_W3 + i] * h2[i];
        z[s] = o;
    }
}

/* round a binary32 value to bfloat16 (nearest, ties to even), returned as float */
static float bf16r(float v)
{
    uint32_t u;
    memcpy(&u, &v, 4);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

/* dot product of bfloat16 values: products are exact in binary32 and the sum
   is taken in double and rounded once (the GPU's binary32 accumulation differs
   from it by a few units in the last place) */
static float dot_bf16(const float* a, const float* b, int n)
{
    double s = 0;
    for (int i = 0; i < n; ++i) s += (double)(a[i] * b[i]);
    return (float)s;
}

/* Logits in the GPU inference precision from raw (unstandardised) binary32
   features: g = bf16((f - mean) / std) in binary32, weights bf16, hidden
   activations bf16 after bias and relu in binary32. */
void velo_oracle_mlp_forward_bf16(const float* p, const float* mean, const float* stdv,
                                  const float* f, int64_t n, float* z)
{
    float w1[NH * NF], w2[NH * NH], w3[NH];
    for (int i = 0; i < NH * NF; ++i) w1[i] = bf16r(p[O_W1 + i]);
    for (int i = 0; i < NH * NH; ++i) w2[i] = bf16r(p[O_W2 + i]);
    for (int i = 0; i < NH; ++i) w3[i] = bf16r(p[O_W3 + i]);
    for (int64_t s = 0; s < n; ++s) {
        float x[NF], h1[NH], h2[NH];
        for (int k = 0; k < NF; ++k) x[k] = bf16r((f[NF * s + k] - mean[k]) / stdv[k]);
        for (int i = 0; i < NH; ++i) {
            float a = dot_bf16(w1 + NF * i, x, NF) + p[O_B1 + i];
            h1[i] = bf16r(a > 0 ? a : 0);
        }
        for (int i = 0; i < NH; ++i) {
            float a = dot_bf16(w2 + NH * i, h1, NH) + p[O_B2 + i];
            h2[i] = bf16r(a > 0 ? a : 0);
        }
        z[s] = dot_bf16(w3, h2, NH) + p[O_B3];
    }
}
