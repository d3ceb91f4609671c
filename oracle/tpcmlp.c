/*
 * CPU ORACLE — test infrastructure only: the learned triplet pruning.
 *
 * A small MLP scores every accepted candidate triplet (down d, cluster i,
 * up u) of the neighbour finder; triplets scoring below a threshold are
 * dropped before the best pair is chosen, i.e. before the cellular
 * automaton runs. The paper describes no such network (it is this build's
 * extension of the tracker); the definitions here are the ones the GPU
 * kernels must reproduce:
 *
 *  - 12 features, each an FP32 expression evaluated in a fixed operation
 *    order with correctly rounded division and square root, then rounded to
 *    BF16 (round to nearest even): the normalised steps (u - i), (i - d) in y
 *    and t, the gap, the pad-row radius, the two pair-score residuals, the
 *    three-point curvature in (x, y), the (d, u) slopes in y and t, and the
 *    local candidate density;
 *  - 12 -> 64 -> 64 -> 1, ReLU, BF16 weights and activations, FP32 biases;
 *    here every product and sum is FP64 (the GPU accumulates in FP32);
 *  - loss: binary cross-entropy with logits, positive weight w_pos.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "tpcoracle.h"

float ora_bf16(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) { /* inf / nan: keep, quiet the nan */
        if (u & 0x007fffffu) u |= 0x00400000u;
        u &= 0xffff0000u;
    } else {
        u += 0x7fffu + ((u >> 16) & 1u);
        u &= 0xffff0000u;
    }
    float r;
    memcpy(&r, &u, 4);
    return r;
}

/* Features of one triplet, FP32 ops in this order, then BF16. wy, wt are
   the box half widths of the gap (g*win), c2s = sqrt(pair_c2). */
void ora_mlp_features(float yd, float td, float xd, float yi, float ti, float xi, float yu, float tu, float xu,
                      int32_t g, float wy, float wt, float w, float c2s, int32_t n_cand, float *f) {
    float dyu = yu - yi, dtu = tu - ti, dyd = yi - yd, dtd = ti - td;
    f[0] = dyu / wy;
    f[1] = dtu / wt;
    f[2] = dyd / wy;
    f[3] = dtd / wt;
    f[4] = (float)g;
    f[5] = xi / 245.0f;
    float by = yu - yd, bt = tu - td;
    float wby = w * by, wbt = w * bt;
    float ry = dyd - wby, rt = dtd - wbt;
    f[6] = ry / c2s;
    f[7] = rt / c2s;
    float ax = xi - xd, cx = xu - xd, ux = xu - xi;
    float cr1 = ax * by, cr2 = dyd * cx;
    float cr = cr1 - cr2;
    float ax2 = ax * ax, dyd2 = dyd * dyd;
    float dab = sqrtf(ax2 + dyd2);
    float cx2 = cx * cx, by2 = by * by;
    float dac = sqrtf(cx2 + by2);
    float ux2 = ux * ux, dyu2 = dyu * dyu;
    float dbc = sqrtf(ux2 + dyu2);
    float den1 = dab * dac;
    float den = den1 * dbc;
    float two_cr = 2.0f * cr;
    float kap = two_cr / den;
    f[8] = kap / 0.015f;
    f[9] = by / cx;
    f[10] = bt / cx;
    f[11] = (float)n_cand / 8.0f;
    for (int k = 0; k < MLP_IN; k++) f[k] = ora_bf16(f[k]);
    for (int k = MLP_IN; k < MLP_INP; k++) f[k] = 0.0f;
}

/* Forward pass: FP64 arithmetic, BF16 rounding of the hidden activations
   (through FP32, as the GPU stores them). Returns the logit; h1, h2 get the
   activations when not NULL. round_act = 0 keeps the activations in FP64
   (a smooth function, for derivative checks). */
static double ora_mlp_forward_d(const ora_mlp *m, const float *x, int32_t round_act, double *h1, double *h2) {
    for (int j = 0; j < MLP_H; j++) {
        double s = m->b1[j];
        for (int k = 0; k < MLP_INP; k++) s += (double)m->w1[j][k] * (double)x[k];
        if (s < 0) s = 0;
        h1[j] = round_act ? (double)ora_bf16((float)s) : s;
    }
    for (int j = 0; j < MLP_H; j++) {
        double s = m->b2[j];
        for (int k = 0; k < MLP_H; k++) s += (double)m->w2[j][k] * h1[k];
        if (s < 0) s = 0;
        h2[j] = round_act ? (double)ora_bf16((float)s) : s;
    }
    double z = m->b3;
    for (int k = 0; k < MLP_H; k++) z += (double)m->w3[k] * h2[k];
    return z;
}

double ora_mlp_forward(const ora_mlp *m, const float *x, int32_t round_act, float *h1o, float *h2o) {
    double h1[MLP_H], h2[MLP_H];
    double z = ora_mlp_forward_d(m, x, round_act, h1, h2);
    for (int j = 0; j < MLP_H; j++) {
        if (h1o) h1o[j] = (float)h1[j];
        if (h2o) h2o[j] = (float)h2[j];
    }
    return z;
}

void ora_mlp_forward_batch(const ora_mlp *m, int64_t n, const float *x, int32_t round_act, double *z) {
    for (int64_t i = 0; i < n; i++) z[i] = ora_mlp_forward(m, x + i * MLP_INP, round_act, NULL, NULL);
}

/* Mean BCE-with-logits loss over a batch and its gradient with respect to
   every weight and bias (FP64). The derivative of the BF16 rounding of an
   activation is taken as 1. Gradients are laid out like ora_mlp but in
   double: g1[64*16], gb1[64], g2[64*64], gb2[64], g3[64], gb3[1]. */
double ora_mlp_grad(const ora_mlp *m, int64_t n, const float *x, const float *label, double w_pos,
                    int32_t round_act, double *g1, double *gb1, double *g2, double *gb2, double *g3,
                    double *gb3) {
    memset(g1, 0, sizeof(double) * MLP_H * MLP_INP);
    memset(gb1, 0, sizeof(double) * MLP_H);
    memset(g2, 0, sizeof(double) * MLP_H * MLP_H);
    memset(gb2, 0, sizeof(double) * MLP_H);
    memset(g3, 0, sizeof(double) * MLP_H);
    *gb3 = 0.0;
    double loss = 0.0;
    for (int64_t i = 0; i < n; i++) {
        const float *xi = x + i * MLP_INP;
        double h1[MLP_H], h2[MLP_H];
        double z = ora_mlp_forward_d(m, xi, round_act, h1, h2);
        double yv = label[i];
        double wgt = yv > 0.5 ? w_pos : 1.0;
        /* loss = w * [log(1 + e^z) - y z], stable form */
        double lp = (z > 0 ? z + log1p(exp(-z)) : log1p(exp(z)));
        loss += wgt * (lp - yv * z);
        double sig = 1.0 / (1.0 + exp(-z));
        double dz = wgt * (sig - yv) / (double)n;
        *gb3 += dz;
        double dh2[MLP_H];
        for (int k = 0; k < MLP_H; k++) {
            g3[k] += dz * h2[k];
            dh2[k] = h2[k] > 0 ? dz * m->w3[k] : 0.0;
        }
        double dh1[MLP_H];
        for (int k = 0; k < MLP_H; k++) dh1[k] = 0.0;
        for (int j = 0; j < MLP_H; j++) {
            if (dh2[j] == 0.0) continue;
            gb2[j] += dh2[j];
            for (int k = 0; k < MLP_H; k++) {
                g2[j * MLP_H + k] += dh2[j] * h1[k];
                dh1[k] += dh2[j] * m->w2[j][k];
            }
        }
        for (int j = 0; j < MLP_H; j++) {
            if (!(h1[j] > 0)) continue;
            gb1[j] += dh1[j];
            for (int k = 0; k < MLP_INP; k++) g1[j * MLP_INP + k] += dh1[j] * xi[k];
        }
    }
    return loss / (double)n;
}

int32_t ora_mlp_sizeof(void) { return (int32_t)sizeof(ora_mlp); }

/* One AdamW step on a flat parameter vector, FP64 (Adam with bias-corrected
   first and second moments, Kingma & Ba; weight decay decoupled from the
   gradient, Loshchilov & Hutter, applied to the entries flagged in `decay`,
   i.e. the weights, never the biases). With k = step (1 for the first):
     p <- p - lr*wd*p                              (decay[i] != 0)
     m <- b1*m + (1 - b1)*g,   v <- b2*v + (1 - b2)*g*g
     p <- p - lr * (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps)
   The decay uses the parameter before this step's moment update. */
void ora_adamw_step(int64_t n, double *p, double *m, double *v, const double *g, const uint8_t *decay, double lr,
                    double b1, double b2, double eps, double wd, int32_t step) {
    double bc1 = 1.0 - pow(b1, (double)step), bc2 = 1.0 - pow(b2, (double)step);
    for (int64_t i = 0; i < n; i++) {
        double pi = p[i];
        if (decay[i]) pi -= lr * wd * pi;
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        pi -= lr * (m[i] / bc1) / (sqrt(v[i] / bc2) + eps);
        p[i] = pi;
    }
}
