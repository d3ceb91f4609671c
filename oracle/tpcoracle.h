/* CPU ORACLE — test infrastructure only. Declarations shared by the
   oracle's sources (tpcoracle.c: links, chains, fit; tpcmlp.c: the triplet
   network). */
#ifndef TPCORACLE_H
#define TPCORACLE_H
#include <stdint.h>

typedef struct {
    int32_t n_rows;
    const float *row_x;      /* [n_rows] pad-row x (cm) */
    float win_y, win_t;      /* box half widths per unit row gap (cm) */
    float pair_c2;           /* acceptance of the pair score (cm^2) */
    int32_t max_gap;         /* largest symmetric row gap tried */
    int32_t min_track_hits;  /* shortest chain that is a track */
    double bz;               /* field (T) */
    double sigma_y, sigma_t; /* cluster resolution (cm) */
    double ivar_s, ivar_tau, ivar_k; /* prior inverse variances (0 = prior off) */
    int32_t max_iter;        /* Gauss-Newton iterations */
    double s_max;            /* |sin phi| above which a propagation fails */
} ora_cfg;

#define MLP_IN 12
#define MLP_INP 16 /* padded input width */
#define MLP_H 64

/* network weights as FP32 values on the BF16 grid */
typedef struct {
    float w1[MLP_H][MLP_INP];
    float b1[MLP_H];
    float w2[MLP_H][MLP_H];
    float b2[MLP_H];
    float w3[MLP_H];
    float b3;
} ora_mlp;

float ora_bf16(float x);
void ora_mlp_features(float yd, float td, float xd, float yi, float ti, float xi, float yu, float tu, float xu,
                      int32_t g, float wy, float wt, float w, float c2s, int32_t n_cand, float *f);
double ora_mlp_forward(const ora_mlp *m, const float *x, int32_t round_act, float *h1o, float *h2o);

#endif
