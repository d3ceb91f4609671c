/*
 * CPU ORACLE — test infrastructure only.
 *
 * A plain, slow, obviously-correct CPU implementation of the TPC track-finding
 * hot path, used only by the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg to check and time the GPU library. It shares no code with
 * the GPU path and is never called by it.
 *
 * What it computes (the paper, Sec. 1, names the step: full TPC tracking of
 * whole continuous-readout time frames, derived from the Run 2 HLT cellular
 * automaton tracker, seeding with time in place of z; it prints no formulas,
 * so every rule below is the reading adopted for this build):
 *
 *  1. Neighbour links (FP32 decisions, exact): for a hit i on row r and gap
 *     g = 1, then 2, take the candidate sets on rows r-g and r+g inside a box
 *     of half widths g*WY (y) and g*WT (time) centred on the hit, score every
 *     (down, up) pair by the squared distance c of the hit from the straight
 *     line through the pair, in the (y, t) plane, interpolated at x_r, accept
 *     c <= C2, and keep the lexicographic minimum of (c, up index, down
 *     index). Rows 0 and n_rows-1 get no links.
 *  2. Cleaning: keep a link only if it is mutual (Jacobi update from the
 *     uncleaned arrays).
 *  3. Cellular-automaton chains: after cleaning every hit has at most one
 *     up and one down link, so the links form disjoint chains. A seed is a
 *     hit with no down link and an up link; a track is the chain of a seed
 *     with at least MIN_TRACK_HITS hits. Tracks are numbered in ascending
 *     seed input index; the assignment maps every member to its track.
 *  4. Track parameters (FP64): maximum a-posteriori helix fit, defined as
 *     the minimiser of the data chi2 of all clusters plus Gaussian priors on
 *     (sin phi, dt/darc, q/pT) centred on a three-point estimate; solved by
 *     Gauss-Newton to convergence and reported at the outermost cluster.
 *  5. Diagnostic: the same fit by an FP64 Kalman filter (extended pass, then
 *     passes linearised about the previous pass's helix), which converges to
 *     the estimate of step 4.
 *
 * Compiled with -ffp-contract=off and without fast-math, scalar SSE, so that
 * every FP32 operation of step 1 rounds exactly once, in the written order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "tpcoracle.h"

/* ---------------------------------------------------------------- links */

typedef struct {
    int32_t *start; /* [n_rows + 1] */
    int32_t *idx;   /* hits grouped by row, each row ordered by (t, index) */
} ora_rows;

typedef struct { float t; int32_t i; } ora_key;
static int ora_cmp_key(const void *a, const void *b) {
    const ora_key *p = (const ora_key *)a, *q = (const ora_key *)b;
    if (p->t < q->t) return -1;
    if (p->t > q->t) return 1;
    return (p->i > q->i) - (p->i < q->i);
}

static void ora_rows_build(const ora_cfg *cfg, int64_t n, const uint8_t *row, const float *t, ora_rows *R) {
    int nr = cfg->n_rows;
    R->start = (int32_t *)calloc((size_t)nr + 1, sizeof(int32_t));
    R->idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int64_t i = 0; i < n; i++) R->start[row[i] + 1]++;
    for (int r = 0; r < nr; r++) R->start[r + 1] += R->start[r];
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)nr);
    for (int r = 0; r < nr; r++) cur[r] = R->start[r];
    for (int64_t i = 0; i < n; i++) R->idx[cur[row[i]]++] = (int32_t)i;
    free(cur);
    /* sorting each row by time only narrows the search below; the candidate
       sets are still decided by the exact predicates */
    ora_key *keys = (ora_key *)malloc(sizeof(ora_key) * (size_t)(n ? n : 1));
    for (int64_t k = 0; k < n; k++) { keys[k].i = R->idx[k]; keys[k].t = t[R->idx[k]]; }
    for (int r = 0; r < nr; r++)
        qsort(keys + R->start[r], (size_t)(R->start[r + 1] - R->start[r]), sizeof(ora_key), ora_cmp_key);
    for (int64_t k = 0; k < n; k++) R->idx[k] = keys[k].i;
    free(keys);
}

static void ora_rows_free(ora_rows *R) { free(R->start); free(R->idx); }

/* first position in row r whose time is >= tmin (row ordered by time) */
static int32_t ora_lower(const ora_rows *R, const float *t, int r, double tmin) {
    int32_t lo = R->start[r], hi = R->start[r + 1];
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if ((double)t[R->idx[mid]] < tmin) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* Candidates of hit i on row rr (= r - g or r + g) inside the box of gap g,
   in time order; returns the count (list grows as needed). */
static int32_t ora_box(const ora_rows *R, const float *y, const float *t, int rr, float yi, float ti, float wy,
                       float wt, int is_down, int32_t **list, int32_t *cap) {
    /* conservative search range in time (a superset); the exact FP32
       predicates decide membership */
    double margin = (double)wt + 1.0;
    int32_t n = 0;
    for (int32_t p = ora_lower(R, t, rr, (double)ti - margin); p < R->start[rr + 1]; p++) {
        int32_t k = R->idx[p];
        if ((double)t[k] > (double)ti + margin) break;
        int in = is_down ? (fabsf(yi - y[k]) <= wy && fabsf(ti - t[k]) <= wt)
                         : (fabsf(y[k] - yi) <= wy && fabsf(t[k] - ti) <= wt);
        if (!in) continue;
        if (n == *cap) {
            *cap = *cap ? 2 * *cap : 64;
            *list = (int32_t *)realloc(*list, sizeof(int32_t) * (size_t)*cap);
        }
        (*list)[n++] = k;
    }
    return n;
}

/* Triplet network gate of the neighbour finder (NULL: none). */
typedef struct {
    const ora_mlp *m;
    double theta, tol;
    int32_t *near;      /* per hit: triplets with |logit - theta| < tol */
} ora_gate;

static void ora_links_one(const ora_cfg *cfg, const ora_rows *R, const uint8_t *row, const float *y,
                          const float *t, int32_t i, int32_t *up_i, int32_t *dn_i, int32_t *gap_i,
                          const ora_gate *gate) {
    int r = row[i];
    *up_i = -1; *dn_i = -1; *gap_i = 0;
    int32_t *D = NULL, *U = NULL, capd = 0, capu = 0;
    float c2s = sqrtf(cfg->pair_c2);
    for (int g = 1; g <= cfg->max_gap; g++) {
        if (r - g < 0 || r + g > cfg->n_rows - 1) continue;
        float xd = cfg->row_x[r - g], xi = cfg->row_x[r], xu = cfg->row_x[r + g];
        float num = xi - xd;
        float den = xu - xd;
        float w = num / den;
        float wy = (float)g * cfg->win_y;
        float wt = (float)g * cfg->win_t;
        float yi = y[i], ti = t[i];
        int32_t nd = ora_box(R, y, t, r - g, yi, ti, wy, wt, 1, &D, &capd);
        int32_t nu = ora_box(R, y, t, r + g, yi, ti, wy, wt, 0, &U, &capu);
        int found = 0;
        float bc = 0.f;
        int32_t bu = -1, bd = -1;
        for (int32_t a = 0; a < nd; a++) {
            int32_t d = D[a];
            float yd = y[d], td = t[d];
            for (int32_t b = 0; b < nu; b++) {
                int32_t u = U[b];
                float yu = y[u], tu = t[u];
                float ady = yi - yd;
                float adt = ti - td;
                float by = yu - yd;
                float bt = tu - td;
                float wby = w * by;
                float wbt = w * bt;
                float ry = ady - wby;
                float rt = adt - wbt;
                float ry2 = ry * ry;
                float rt2 = rt * rt;
                float c = ry2 + rt2;
                if (!(c <= cfg->pair_c2)) continue;
                if (gate && gate->m) {
                    float f[MLP_INP];
                    ora_mlp_features(yd, td, xd, yi, ti, xi, yu, tu, xu, g, wy, wt, w, c2s, nd + nu, f);
                    double z = ora_mlp_forward(gate->m, f, 1, NULL, NULL);
                    if (gate->near && fabs(z - gate->theta) < gate->tol) gate->near[i]++;
                    if (!(z >= gate->theta)) continue;
                }
                if (!found || c < bc || (c == bc && (u < bu || (u == bu && d < bd)))) {
                    found = 1; bc = c; bu = u; bd = d;
                }
            }
        }
        if (found) {
            *up_i = bu; *dn_i = bd; *gap_i = g;
            break;
        }
    }
    free(D);
    free(U);
}

/* Links of every hit of one sector (input-index space). */
void ora_links(const ora_cfg *cfg, int64_t n, const uint8_t *row, const float *y, const float *t,
               int32_t *up, int32_t *dn, int32_t *gap) {
    ora_rows R;
    ora_rows_build(cfg, n, row, t, &R);
    for (int64_t i = 0; i < n; i++) ora_links_one(cfg, &R, row, y, t, (int32_t)i, &up[i], &dn[i], &gap[i], NULL);
    ora_rows_free(&R);
}

/* Links of the listed hits only (for sampled checks on very large sectors);
   outputs are indexed like `query`. */
void ora_links_subset(const ora_cfg *cfg, int64_t n, const uint8_t *row, const float *y, const float *t,
                      int64_t nq, const int32_t *query, int32_t *up, int32_t *dn, int32_t *gap) {
    ora_rows R;
    ora_rows_build(cfg, n, row, t, &R);
    for (int64_t k = 0; k < nq; k++)
        ora_links_one(cfg, &R, row, y, t, query[k], &up[k], &dn[k], &gap[k], NULL);
    ora_rows_free(&R);
}

/* Links with the triplet network gate: a pair is accepted only if also its
   logit is >= theta; near[i] counts hit i's triplets within tol of theta
   (decisions there may legitimately differ from an FP32-accumulating
   implementation). */
void ora_links_pruned(const ora_cfg *cfg, int64_t n, const uint8_t *row, const float *y, const float *t,
                      const ora_mlp *m, double theta, double tol, int32_t *up, int32_t *dn, int32_t *gap,
                      int32_t *near) {
    ora_rows R;
    ora_rows_build(cfg, n, row, t, &R);
    ora_gate gt = {m, theta, tol, near};
    for (int64_t i = 0; i < n; i++) near[i] = 0;
    for (int64_t i = 0; i < n; i++) ora_links_one(cfg, &R, row, y, t, (int32_t)i, &up[i], &dn[i], &gap[i], &gt);
    ora_rows_free(&R);
}

/* Every accepted triplet (c <= pair_c2) of every hit for every gap
   g = 1..max_gap, with its features: tri[4k..4k+3] = (d, i, u, g),
   feat[16k..16k+15]. Returns the number found (entries beyond cap are
   counted, not stored). */
int64_t ora_triplets(const ora_cfg *cfg, int64_t n, const uint8_t *row, const float *y, const float *t,
                     int64_t cap, int32_t *tri, float *feat) {
    ora_rows R;
    ora_rows_build(cfg, n, row, t, &R);
    int32_t *D = NULL, *U = NULL, capd = 0, capu = 0;
    float c2s = sqrtf(cfg->pair_c2);
    int64_t cnt = 0;
    for (int64_t ii = 0; ii < n; ii++) {
        int32_t i = (int32_t)ii;
        int r = row[i];
        for (int g = 1; g <= cfg->max_gap; g++) {
            if (r - g < 0 || r + g > cfg->n_rows - 1) continue;
            float xd = cfg->row_x[r - g], xi = cfg->row_x[r], xu = cfg->row_x[r + g];
            float num = xi - xd;
            float den = xu - xd;
            float w = num / den;
            float wy = (float)g * cfg->win_y;
            float wt = (float)g * cfg->win_t;
            float yi = y[i], ti = t[i];
            int32_t nd = ora_box(&R, y, t, r - g, yi, ti, wy, wt, 1, &D, &capd);
            int32_t nu = ora_box(&R, y, t, r + g, yi, ti, wy, wt, 0, &U, &capu);
            for (int32_t a = 0; a < nd; a++) {
                int32_t d = D[a];
                float yd = y[d], td = t[d];
                for (int32_t b = 0; b < nu; b++) {
                    int32_t u = U[b];
                    float yu = y[u], tu = t[u];
                    float ady = yi - yd, adt = ti - td, by = yu - yd, bt = tu - td;
                    float wby = w * by, wbt = w * bt;
                    float ry = ady - wby, rt = adt - wbt;
                    float ry2 = ry * ry, rt2 = rt * rt;
                    float c = ry2 + rt2;
                    if (!(c <= cfg->pair_c2)) continue;
                    if (cnt < cap) {
                        tri[4 * cnt] = d; tri[4 * cnt + 1] = i; tri[4 * cnt + 2] = u; tri[4 * cnt + 3] = g;
                        ora_mlp_features(yd, td, xd, yi, ti, xi, yu, tu, xu, g, wy, wt, w, c2s, nd + nu,
                                         feat + 16 * cnt);
                    }
                    cnt++;
                }
            }
        }
    }
    free(D);
    free(U);
    ora_rows_free(&R);
    return cnt;
}

/* ------------------------------------------------------------- cleaning */

void ora_clean(int64_t n, const int32_t *up, const int32_t *dn, int32_t *upc, int32_t *dnc) {
    for (int64_t i = 0; i < n; i++) {
        int32_t u = up[i], d = dn[i];
        upc[i] = (u >= 0 && dn[u] == (int32_t)i) ? u : -1;
        dnc[i] = (d >= 0 && up[d] == (int32_t)i) ? d : -1;
    }
}

/* --------------------------------------------------------------- chains */

/* Tracks from cleaned links. Fills first[], len[] per track (capacity n),
   clusters[] (members, seed first, rows ascending; capacity n) and assign[]
   (track number or -1). Returns the number of tracks. */
int64_t ora_tracks(const ora_cfg *cfg, int64_t n, const int32_t *upc, const int32_t *dnc,
                   int64_t *first, int32_t *len, int32_t *clusters, int32_t *assign) {
    for (int64_t i = 0; i < n; i++) assign[i] = -1;
    int64_t nt = 0, nc = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!(dnc[i] < 0 && upc[i] >= 0)) continue;
        int32_t L = 0;
        for (int32_t p = (int32_t)i; p >= 0; p = upc[p]) L++;
        if (L < cfg->min_track_hits) continue;
        first[nt] = nc;
        len[nt] = L;
        for (int32_t p = (int32_t)i; p >= 0; p = upc[p]) {
            clusters[nc++] = p;
            assign[p] = (int32_t)nt;
        }
        nt++;
    }
    return nt;
}

/* chain length of every hit (number of hits of the chain it belongs to) */
void ora_chain_len(int64_t n, const int32_t *upc, const int32_t *dnc, int32_t *clen) {
    for (int64_t i = 0; i < n; i++) clen[i] = 0;
    for (int64_t i = 0; i < n; i++) {
        if (dnc[i] >= 0) continue;
        int32_t L = 0;
        for (int32_t p = (int32_t)i; p >= 0; p = upc[p]) L++;
        for (int32_t p = (int32_t)i; p >= 0; p = upc[p]) clen[p] = L;
    }
}

/* ------------------------------------------------------------ helix fit */

#define ORA_NP 5 /* state (y, t, sin phi, dt/darc, q/pT) */

/* asin(u)/u and its derivative, by their Maclaurin series near 0 */
static void ora_asin_ratio(double u, double *A, double *dA) {
    if (fabs(u) < 0.05) {
        /* a_n = C(2n,n)/4^n; asin(u)/u = sum a_n u^2n/(2n+1);
           d/du = sum a_n (2n/(2n+1)) u^(2n-1) */
        double an = 1.0, u2 = u * u, pw = 1.0, a = 0.0, da = 0.0;
        for (int k = 0; k <= 9; k++) {
            if (k > 0) an *= (double)(2 * k - 1) / (double)(2 * k);
            a += an * pw / (2.0 * k + 1.0);
            if (k > 0) da += an * (2.0 * k / (2.0 * k + 1.0)) * pw / u;
            pw *= u2;
        }
        *A = a;
        *dA = (u == 0.0) ? 0.0 : da;
    } else {
        double as = asin(u);
        *A = as / u;
        *dA = (1.0 / sqrt(1.0 - u * u) - *A) / u;
    }
}

/* Closed-form transport of the state q at x by dx along the helix, with the
   Jacobian F = d(q')/d(q). Returns 0 if |sin phi| leaves [0, s_max). */
static int ora_propagate(const ora_cfg *cfg, const double *q, double dx, double *qo, double F[5][5]) {
    double kB = 2.99792458e-3 * cfg->bz;
    double s = q[2], tau = q[3], k = q[4];
    double kap = -kB * k;
    double s1 = s + kap * dx;
    if (!(fabs(s) < cfg->s_max) || !(fabs(s1) < cfg->s_max)) return 0;
    double c = sqrt(1.0 - s * s), c1 = sqrt(1.0 - s1 * s1);
    double S = s + s1, C = c + c1;
    double dy = dx * S / C;
    double L = sqrt(dx * dx + dy * dy);
    double u = 0.5 * kap * L;
    if (!(fabs(u) < 1.0)) return 0;
    double A, dA;
    ora_asin_ratio(u, &A, &dA);
    double sgn = dx < 0 ? -1.0 : 1.0;
    double dl = sgn * L * A;
    qo[0] = q[0] + dy;
    qo[1] = q[1] + tau * dl;
    qo[2] = s1;
    qo[3] = tau;
    qo[4] = k;
    if (F) {
        memset(F, 0, sizeof(double) * 25);
        double dy_ds = dx * (2.0 / C + S * (s / c + s1 / c1) / (C * C));
        double dy_dk = -kB * dx * dx * (1.0 / C + S * s1 / (c1 * C * C));
        double dl_dL = sgn / sqrt(1.0 - u * u);
        double dl_ds = 0.0, dl_dk = 0.0;
        if (L > 0) {
            dl_ds = dl_dL * (dy / L) * dy_ds;
            dl_dk = dl_dL * (dy / L) * dy_dk + sgn * 0.5 * L * L * dA * (-kB);
        }
        F[0][0] = 1.0; F[0][2] = dy_ds; F[0][4] = dy_dk;
        F[1][1] = 1.0; F[1][2] = tau * dl_ds; F[1][3] = dl; F[1][4] = tau * dl_dk;
        F[2][2] = 1.0; F[2][4] = -kB * dx;
        F[3][3] = 1.0;
        F[4][4] = 1.0;
    }
    return 1;
}

/* Exposed for tests: one transport with Jacobian (F row-major 25). */
int32_t ora_propagate_c(const ora_cfg *cfg, const double *q, double dx, double *qo, double *F) {
    double Fm[5][5];
    int ok = ora_propagate(cfg, q, dx, qo, F ? Fm : NULL);
    if (ok && F) memcpy(F, Fm, sizeof(Fm));
    return ok;
}

/* Solve the symmetric positive-definite system H x = g (Cholesky); Hinv
   optional. Returns 0 if H is not positive definite. */
static int ora_chol_solve(double H[5][5], const double *g, double *x, double Hinv[5][5]) {
    double Lm[5][5];
    memset(Lm, 0, sizeof(Lm));
    for (int i = 0; i < 5; i++) {
        for (int j = 0; j <= i; j++) {
            double sum = H[i][j];
            for (int k = 0; k < j; k++) sum -= Lm[i][k] * Lm[j][k];
            if (i == j) {
                if (!(sum > 0)) return 0;
                Lm[i][i] = sqrt(sum);
            } else {
                Lm[i][j] = sum / Lm[j][j];
            }
        }
    }
    if (g && x) {
        double z[5];
        for (int i = 0; i < 5; i++) {
            double sum = g[i];
            for (int k = 0; k < i; k++) sum -= Lm[i][k] * z[k];
            z[i] = sum / Lm[i][i];
        }
        for (int i = 4; i >= 0; i--) {
            double sum = z[i];
            for (int k = i + 1; k < 5; k++) sum -= Lm[k][i] * x[k];
            x[i] = sum / Lm[i][i];
        }
    }
    if (Hinv) {
        for (int col = 0; col < 5; col++) {
            double e[5] = {0, 0, 0, 0, 0}, z[5], v[5];
            e[col] = 1.0;
            for (int i = 0; i < 5; i++) {
                double sum = e[i];
                for (int k = 0; k < i; k++) sum -= Lm[i][k] * z[k];
                z[i] = sum / Lm[i][i];
            }
            for (int i = 4; i >= 0; i--) {
                double sum = z[i];
                for (int k = i + 1; k < 5; k++) sum -= Lm[k][i] * v[k];
                v[i] = sum / Lm[i][i];
            }
            for (int i = 0; i < 5; i++) Hinv[i][col] = v[i];
        }
    }
    return 1;
}

/* Fit result. status: 0 ok, 2 = propagation/initialisation failure,
   4 = not converged. */
typedef struct {
    int32_t status, n_iter, ndf, pad;
    double x_ref, y, t, sinphi, tau, qpt, chi2;
    double cov[15]; /* lower triangle, row-major: (0,0),(1,0),(1,1),(2,0),... */
    double init[5]; /* three-point estimate at the first cluster */
} ora_fit;

/* Three-point estimate at the first cluster. */
static int ora_init3(const ora_cfg *cfg, int32_t L, const double *x, const double *y, const double *t,
                     double *q0) {
    double kB = 2.99792458e-3 * cfg->bz;
    int m = (L + 1) / 2 - 1; /* 0-based index of c_ceil(L/2) */
    double xa = x[0], ya = y[0], xb = x[m], yb = y[m], xc = x[L - 1], yc = y[L - 1];
    double abx = xb - xa, aby = yb - ya, acx = xc - xa, acy = yc - ya, bcx = xc - xb, bcy = yc - yb;
    double cr = abx * acy - aby * acx;
    double dab = sqrt(abx * abx + aby * aby), dac = sqrt(acx * acx + acy * acy),
           dbc = sqrt(bcx * bcx + bcy * bcy);
    if (!(dab > 0 && dac > 0 && dbc > 0)) return 0;
    double kap = 2.0 * cr / (dab * dac * dbc);
    double u = 0.5 * kap * dac;
    if (!(fabs(u) < 1.0)) return 0;
    double A, dA;
    ora_asin_ratio(u, &A, &dA);
    double phi = atan2(acy, acx) - asin(u);
    if (!(cos(phi) > 0)) return 0;
    q0[0] = ya;
    q0[1] = t[0];
    q0[2] = sin(phi);
    q0[3] = (t[L - 1] - t[0]) / (dac * A);
    q0[4] = (kB != 0.0) ? -kap / kB : 0.0;
    return 1;
}

/* data chi2 and normal equations of the MAP problem at q (state at x[0]) */
static int ora_normal(const ora_cfg *cfg, int32_t L, const double *x, const double *y, const double *t,
                      const double *q, const double *q0, double H[5][5], double *g, double *chi2_data,
                      double *cost) {
    double wy = 1.0 / (cfg->sigma_y * cfg->sigma_y), wt = 1.0 / (cfg->sigma_t * cfg->sigma_t);
    double P[5] = {0.0, 0.0, cfg->ivar_s, cfg->ivar_tau, cfg->ivar_k};
    if (H) memset(H, 0, sizeof(double) * 25);
    if (g) memset(g, 0, sizeof(double) * 5);
    double chi2 = 0.0;
    for (int j = 0; j < L; j++) {
        double qj[5], F[5][5];
        if (!ora_propagate(cfg, q, x[j] - x[0], qj, F)) return 0;
        double ry = y[j] - qj[0], rt = t[j] - qj[1];
        chi2 += ry * ry * wy + rt * rt * wt;
        if (H) {
            for (int a = 0; a < 5; a++) {
                g[a] += F[0][a] * wy * ry + F[1][a] * wt * rt;
                for (int b = 0; b < 5; b++) H[a][b] += F[0][a] * wy * F[0][b] + F[1][a] * wt * F[1][b];
            }
        }
    }
    double pr = 0.0;
    for (int a = 2; a < 5; a++) {
        double d = q0[a] - q[a];
        pr += P[a] * d * d;
        if (H) {
            H[a][a] += P[a];
            g[a] += P[a] * d;
        }
    }
    *chi2_data = chi2;
    *cost = chi2 + pr;
    return 1;
}

static void ora_pack_cov(double C[5][5], double *out15) {
    int k = 0;
    for (int i = 0; i < 5; i++)
        for (int j = 0; j <= i; j++) out15[k++] = C[i][j];
}

/* MAP fit of one track, clusters ordered by row (x ascending). */
void ora_fit_map(const ora_cfg *cfg, int32_t L, const double *x, const double *y, const double *t,
                 ora_fit *out) {
    memset(out, 0, sizeof(*out));
    out->ndf = 2 * L - 5;
    out->x_ref = x[L - 1];
    double q0[5], q[5];
    if (L < 3 || !ora_init3(cfg, L, x, y, t, q0)) { out->status = 2; return; }
    memcpy(out->init, q0, sizeof(q0));
    memcpy(q, q0, sizeof(q));
    double H[5][5], g[5], chi2, cost;
    if (!ora_normal(cfg, L, x, y, t, q, q0, H, g, &chi2, &cost)) { out->status = 2; return; }
    int conv = 0, it;
    for (it = 0; it < cfg->max_iter; it++) {
        double dq[5];
        if (!ora_chol_solve(H, g, dq, NULL)) { out->status = 2; return; }
        /* predicted decrease of the objective for the full step; once it is
           below what the objective's rounding can resolve, the full
           Gauss-Newton step is taken without a line search (the iteration is
           then in its quadratically convergent range) */
        double pred = 0.0;
        for (int a = 0; a < 5; a++) pred += g[a] * dq[a];
        int small = pred < 1e-9 * (1.0 + cost);
        double lam = 1.0;
        int acc = 0;
        double qn[5], Hn[5][5], gn[5], chi2n = 0, costn = 0;
        for (int h = 0; h < 40; h++) {
            for (int a = 0; a < 5; a++) qn[a] = q[a] + lam * dq[a];
            if (ora_normal(cfg, L, x, y, t, qn, q0, Hn, gn, &chi2n, &costn) && (small || costn <= cost)) {
                acc = 1;
                break;
            }
            lam *= 0.5;
        }
        if (!acc) break;
        double smax = 0.0;
        for (int a = 0; a < 5; a++) {
            double scale = fabs(q[a]) > 1.0 ? fabs(q[a]) : 1.0;
            double r = fabs(qn[a] - q[a]) / scale;
            if (r > smax) smax = r;
        }
        memcpy(q, qn, sizeof(q));
        memcpy(H, Hn, sizeof(H));
        memcpy(g, gn, sizeof(g));
        chi2 = chi2n;
        cost = costn;
        /* converged once a full step moves no parameter by more than 1e-10
           relative (floor 1): FP64 rounding of the predictions leaves steps of
           up to ~1e-11 relative in q/pT of short, poorly curved tracks, which
           never shrink further */
        if (smax < 1e-10) { conv = 1; it++; break; }
    }
    out->n_iter = it;
    double C1[5][5];
    if (!ora_chol_solve(H, NULL, NULL, C1)) { out->status = 2; return; }
    double qL[5], F[5][5];
    if (!ora_propagate(cfg, q, x[L - 1] - x[0], qL, F)) { out->status = 2; return; }
    double CL[5][5], T[5][5];
    for (int i = 0; i < 5; i++)
        for (int j = 0; j < 5; j++) {
            double s = 0;
            for (int k = 0; k < 5; k++) s += F[i][k] * C1[k][j];
            T[i][j] = s;
        }
    for (int i = 0; i < 5; i++)
        for (int j = 0; j < 5; j++) {
            double s = 0;
            for (int k = 0; k < 5; k++) s += T[i][k] * F[j][k];
            CL[i][j] = s;
        }
    out->y = qL[0]; out->t = qL[1]; out->sinphi = qL[2]; out->tau = qL[3]; out->qpt = qL[4];
    out->chi2 = chi2;
    ora_pack_cov(CL, out->cov);
    out->status = conv ? 0 : 4;
}

/* cost of the MAP objective at a state q at x[0] (tests: stationarity) */
double ora_map_cost(const ora_cfg *cfg, int32_t L, const double *x, const double *y, const double *t,
                    const double *q, const double *q0) {
    double chi2, cost;
    if (!ora_normal(cfg, L, x, y, t, q, q0, NULL, NULL, &chi2, &cost)) return INFINITY;
    return cost;
}

/* Diagnostic FP64 Kalman filter: pass 1 re-linearises at every step
   (extended filter); passes 2.. linearise about the helix of the previous
   pass's result, carried back to the first cluster. The prior is the same
   as in ora_fit_map; the first cluster is folded into the initial state. */
void ora_fit_kf(const ora_cfg *cfg, int32_t L, const double *x, const double *y, const double *t,
                int32_t passes, ora_fit *out) {
    memset(out, 0, sizeof(*out));
    out->ndf = 2 * L - 5;
    out->x_ref = x[L - 1];
    double q0[5];
    if (L < 3 || !ora_init3(cfg, L, x, y, t, q0)) { out->status = 2; return; }
    memcpy(out->init, q0, sizeof(q0));
    double vy = cfg->sigma_y * cfg->sigma_y, vt = cfg->sigma_t * cfg->sigma_t;
    double ref1[5]; /* reference state at x[0] */
    memcpy(ref1, q0, sizeof(ref1));
    double dev[5], C[5][5], ref[5], chi2 = 0;
    for (int pass = 0; pass < passes; pass++) {
        int ext = (pass == 0);
        memcpy(ref, ref1, sizeof(ref));
        /* deviation of the prior (first cluster, three-point centres) from the reference */
        dev[0] = y[0] - ref[0];
        dev[1] = t[0] - ref[1];
        dev[2] = q0[2] - ref[2];
        dev[3] = q0[3] - ref[3];
        dev[4] = q0[4] - ref[4];
        memset(C, 0, sizeof(C));
        C[0][0] = vy; C[1][1] = vt;
        C[2][2] = 1.0 / cfg->ivar_s; C[3][3] = 1.0 / cfg->ivar_tau; C[4][4] = 1.0 / cfg->ivar_k;
        chi2 = 0.0;
        for (int j = 1; j < L; j++) {
            double rn[5], F[5][5];
            if (!ora_propagate(cfg, ref, x[j] - x[j - 1], rn, F)) { out->status = 2; return; }
            double dn_[5], T[5][5], Cn[5][5];
            for (int a = 0; a < 5; a++) {
                double s = 0;
                for (int b = 0; b < 5; b++) s += F[a][b] * dev[b];
                dn_[a] = s;
            }
            for (int a = 0; a < 5; a++)
                for (int b = 0; b < 5; b++) {
                    double s = 0;
                    for (int k = 0; k < 5; k++) s += F[a][k] * C[k][b];
                    T[a][b] = s;
                }
            for (int a = 0; a < 5; a++)
                for (int b = 0; b < 5; b++) {
                    double s = 0;
                    for (int k = 0; k < 5; k++) s += T[a][k] * F[b][k];
                    Cn[a][b] = s;
                }
            memcpy(ref, rn, sizeof(ref));
            memcpy(dev, dn_, sizeof(dev));
            memcpy(C, Cn, sizeof(C));
            /* update with (y, t) at x[j] */
            double r0 = y[j] - (ref[0] + dev[0]);
            double r1 = t[j] - (ref[1] + dev[1]);
            double S00 = C[0][0] + vy, S01 = C[0][1], S11 = C[1][1] + vt;
            double det = S00 * S11 - S01 * S01;
            double i00 = S11 / det, i01 = -S01 / det, i11 = S00 / det;
            chi2 += r0 * (i00 * r0 + i01 * r1) + r1 * (i01 * r0 + i11 * r1);
            double K[5][2];
            for (int a = 0; a < 5; a++) {
                K[a][0] = C[a][0] * i00 + C[a][1] * i01;
                K[a][1] = C[a][0] * i01 + C[a][1] * i11;
            }
            for (int a = 0; a < 5; a++) dev[a] += K[a][0] * r0 + K[a][1] * r1;
            double Cu[5][5];
            for (int a = 0; a < 5; a++)
                for (int b = 0; b < 5; b++) Cu[a][b] = C[a][b] - (K[a][0] * C[0][b] + K[a][1] * C[1][b]);
            memcpy(C, Cu, sizeof(C));
            if (ext) {
                for (int a = 0; a < 5; a++) { ref[a] += dev[a]; dev[a] = 0.0; }
            }
        }
        /* estimate at the last cluster; carry it back for the next pass */
        double est[5];
        for (int a = 0; a < 5; a++) est[a] = ref[a] + dev[a];
        out->y = est[0]; out->t = est[1]; out->sinphi = est[2]; out->tau = est[3]; out->qpt = est[4];
        ora_pack_cov(C, out->cov);
        if (pass + 1 < passes) {
            double back[5];
            if (!ora_propagate(cfg, est, x[0] - x[L - 1], back, NULL)) { out->status = 2; return; }
            memcpy(ref1, back, sizeof(ref1));
        }
    }
    /* data chi2 of the final estimate's helix at every cluster */
    {
        double est[5] = {out->y, out->t, out->sinphi, out->tau, out->qpt};
        double wy = 1.0 / vy, wt = 1.0 / vt;
        chi2 = 0.0;
        for (int j = 0; j < L; j++) {
            double qj[5];
            if (!ora_propagate(cfg, est, x[j] - x[L - 1], qj, NULL)) { out->status = 2; return; }
            chi2 += (y[j] - qj[0]) * (y[j] - qj[0]) * wy + (t[j] - qj[1]) * (t[j] - qj[1]) * wt;
        }
    }
    out->chi2 = chi2;
    out->n_iter = passes;
    out->status = 0;
}

/* Fit all tracks of a sector from float clusters (row -> x). out[n_tracks]. */
void ora_fit_tracks(const ora_cfg *cfg, int64_t n_tracks, const int64_t *first, const int32_t *len,
                    const int32_t *clusters, const uint8_t *row, const float *y, const float *t,
                    int32_t kf_passes, ora_fit *out) {
    int32_t cap = 0;
    double *xb = NULL, *yb = NULL, *tb = NULL;
    for (int64_t k = 0; k < n_tracks; k++) {
        int32_t L = len[k];
        if (L > cap) {
            cap = L;
            xb = (double *)realloc(xb, sizeof(double) * (size_t)cap);
            yb = (double *)realloc(yb, sizeof(double) * (size_t)cap);
            tb = (double *)realloc(tb, sizeof(double) * (size_t)cap);
        }
        for (int32_t j = 0; j < L; j++) {
            int32_t c = clusters[first[k] + j];
            xb[j] = (double)cfg->row_x[row[c]];
            yb[j] = (double)y[c];
            tb[j] = (double)t[c];
        }
        if (kf_passes > 0) ora_fit_kf(cfg, L, xb, yb, tb, kf_passes, &out[k]);
        else ora_fit_map(cfg, L, xb, yb, tb, &out[k]);
    }
    free(xb); free(yb); free(tb);
}

int32_t ora_sizeof_fit(void) { return (int32_t)sizeof(ora_fit); }
int32_t ora_sizeof_cfg(void) { return (int32_t)sizeof(ora_cfg); }

/* ------------------------------------------------------------ following */
/* Track following and selection (the rest of an HLT-style tracklet
   constructor: the paper, Sec. 1, derives the tracker from the Run 2 HLT
   tracker and asks for more attached hits, Sec. 2; it prints no method, so
   this is the reading adopted for this build, with FP32 decisions):

   1. For every track of step 3, two linear Kalman filters in FP32, one for
      y(x) and one for t(x), each with state (value, slope) and covariance
      (p00, p01, p11), start at the innermost cluster with (value, 0) and
      diag(var, var_slope0), and take the chain's clusters in row order. A
      prediction by dx adds q_slope * |dx| to the slope variance:
        a = a + b*dx;  u = p01 + dx*p11;  p00 = (p00 + dx*p01) + dx*u;
        p01 = u;  p11 = p11 + q_slope*|dx|
      an update with measurement m of variance s2:
        S = p00 + s2;  iS = 1/S;  k0 = p00*iS;  k1 = p01*iS;  r = m - a;
        a = a + k0*r;  b = b + k1*r;
        p00 = p00 - k0*p00;  p01 = p01 - k0*p01;  p11 = p11 - k1*p01(old)
      (every operation one FP32 rounding, in this order).
   2. Outward extension: row by row beyond the last cluster, predict both
      filters to the row; among the row's clusters with |y - y_p| <= win_y
      and |t - t_p| <= win_t take the one with the smallest
      chi2 = (dy*dy)*(1/(p00y + var_y)) + (dt*dt)*(1/(p00t + var_t)), ties to the
      smaller input index; accept it if chi2 <= chi2_max and update both
      filters. max_miss consecutive rows without an accepted cluster, or the
      last row, end the extension. Inward extension: the same from the
      outermost cluster down (the filters restart there and take the chain
      in descending rows).
   3. Selection: a track's length is its chain plus both extensions; each
      cluster goes to the longest track containing it (ties: smaller seed
      input index); a track keeping fewer than min_track_hits clusters is
      dropped and its clusters are left unassigned. The kept tracks, in
      ascending seed input index, list their kept clusters in ascending
      rows. */

typedef struct {
    float win_y, win_t;  /* search box half widths around the prediction (cm) */
    float chi2_max;      /* gate */
    float q_slope;       /* slope variance added per cm of |dx| */
    float var_y, var_t;  /* measurement variances (cm^2) */
    float var_slope0;    /* initial slope variance */
    int32_t max_miss;    /* consecutive rows without a cluster that end an extension */
} ora_follow_cfg;

typedef struct { float a, b, p00, p01, p11; } ora_kf1;

static void ora_kf1_init(ora_kf1 *f, float m, float var, float var_slope0) {
    f->a = m; f->b = 0.0f; f->p00 = var; f->p01 = 0.0f; f->p11 = var_slope0;
}

static void ora_kf1_predict(ora_kf1 *f, float dx, float q) {
    float bdx = f->b * dx;
    f->a = f->a + bdx;
    float dp11 = dx * f->p11;
    float u = f->p01 + dp11;
    float dp01 = dx * f->p01;
    float s = f->p00 + dp01;
    float du = dx * u;
    f->p00 = s + du;
    f->p01 = u;
    float qa = q * fabsf(dx);
    f->p11 = f->p11 + qa;
}

static void ora_kf1_update(ora_kf1 *f, float m, float s2) {
    float S = f->p00 + s2;
    float iS = 1.0f / S;
    float k0 = f->p00 * iS;
    float k1 = f->p01 * iS;
    float r = m - f->a;
    float k0r = k0 * r, k1r = k1 * r;
    f->a = f->a + k0r;
    f->b = f->b + k1r;
    float k0p00 = k0 * f->p00, k0p01 = k0 * f->p01, k1p01 = k1 * f->p01;
    float n00 = f->p00 - k0p00;
    float n01 = f->p01 - k0p01;
    float n11 = f->p11 - k1p01;
    f->p00 = n00; f->p01 = n01; f->p11 = n11;
}

/* The filter of step 1 over n points (x[i], m[i]) taken in the given
   order, started at the first point; writes (a, b, p00, p01, p11). Exposed
   so that the filter can be checked on its own. */
void ora_kf1_run(int32_t n, const float *x, const float *m, float var, float var_slope0, float q,
                 float *out5) {
    ora_kf1 f;
    ora_kf1_init(&f, m[0], var, var_slope0);
    for (int32_t i = 1; i < n; i++) {
        ora_kf1_predict(&f, x[i] - x[i - 1], q);
        ora_kf1_update(&f, m[i], var);
    }
    out5[0] = f.a; out5[1] = f.b; out5[2] = f.p00; out5[3] = f.p01; out5[4] = f.p11;
}

/* One extension (dir = +1 outward, -1 inward) from row r_end, the filters
   already at x[r_end]; appends accepted clusters to ext (rows in the order
   visited), returns their count. */
static int32_t ora_extend(const ora_cfg *cfg, const ora_follow_cfg *fc, const ora_rows *R, const float *y,
                          const float *t, int r_end, int dir, ora_kf1 *fy, ora_kf1 *ft, int32_t *ext,
                          int32_t **list, int32_t *cap) {
    int32_t n = 0, miss = 0;
    float xp = cfg->row_x[r_end];
    for (int r = r_end + dir; r >= 0 && r < cfg->n_rows; r += dir) {
        float xr = cfg->row_x[r];
        float dx = xr - xp;
        ora_kf1_predict(fy, dx, fc->q_slope);
        ora_kf1_predict(ft, dx, fc->q_slope);
        xp = xr;
        float vy = fy->p00 + fc->var_y, vt = ft->p00 + fc->var_t;
        float ivy = 1.0f / vy, ivt = 1.0f / vt;
        int32_t nb = ora_box(R, y, t, r, fy->a, ft->a, fc->win_y, fc->win_t, 0, list, cap);
        int32_t best = -1;
        float bchi = 0.0f;
        for (int32_t k = 0; k < nb; k++) {
            int32_t c = (*list)[k];
            float dy = y[c] - fy->a, dt = t[c] - ft->a;
            float ey = dy * dy, et = dt * dt;
            float chi = ey * ivy + et * ivt;
            if (best < 0 || chi < bchi || (chi == bchi && c < best)) { best = c; bchi = chi; }
        }
        if (best >= 0 && bchi <= fc->chi2_max) {
            ora_kf1_update(fy, y[best], fc->var_y);
            ora_kf1_update(ft, t[best], fc->var_t);
            ext[n++] = best;
            miss = 0;
        } else if (++miss >= fc->max_miss) {
            break;
        }
    }
    return n;
}

/* Following and selection of the tracks (first, len, clusters) of one
   sector. Writes the kept tracks (out_first, out_len, out_clusters; same
   capacities as the inputs: at most n_tracks tracks and n clusters) and the
   assignment, and per input track the extension counts (ext_in, ext_out)
   and whether it was kept (kept: kept clusters, or -1 when dropped).
   Returns the number of kept tracks. */
int64_t ora_follow(const ora_cfg *cfg, const ora_follow_cfg *fc, int64_t n, const uint8_t *row, const float *y,
                   const float *t, int64_t n_tracks, const int64_t *first, const int32_t *len,
                   const int32_t *clusters, int64_t *out_first, int32_t *out_len, int32_t *out_clusters,
                   int32_t *assign, int32_t *ext_in, int32_t *ext_out, int32_t *kept) {
    ora_rows R;
    ora_rows_build(cfg, n, row, t, &R);
    int32_t *list = NULL, cap = 0;
    int32_t nr = cfg->n_rows;
    /* per track: inward extension (rows descending) and outward (ascending) */
    int64_t *eoff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_tracks + 1));
    int32_t *ebuf = NULL;
    int64_t ecap = 0, etot = 0;
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nr > 0 ? nr : 1));
    for (int64_t k = 0; k < n_tracks; k++) {
        const int32_t *c = clusters + first[k];
        int32_t L = len[k];
        eoff[k] = etot;
        if (etot + 2 * nr > ecap) {
            ecap = ecap ? 2 * ecap + 2 * nr : 4 * nr + 1024;
            ebuf = (int32_t *)realloc(ebuf, sizeof(int32_t) * (size_t)ecap);
        }
        ora_kf1 fy, ft;
        /* inward: start at the outermost cluster, chain in descending rows */
        ora_kf1_init(&fy, y[c[L - 1]], fc->var_y, fc->var_slope0);
        ora_kf1_init(&ft, t[c[L - 1]], fc->var_t, fc->var_slope0);
        for (int32_t j = L - 2; j >= 0; j--) {
            float dx = cfg->row_x[row[c[j]]] - cfg->row_x[row[c[j + 1]]];
            ora_kf1_predict(&fy, dx, fc->q_slope);
            ora_kf1_predict(&ft, dx, fc->q_slope);
            ora_kf1_update(&fy, y[c[j]], fc->var_y);
            ora_kf1_update(&ft, t[c[j]], fc->var_t);
        }
        ext_in[k] = ora_extend(cfg, fc, &R, y, t, row[c[0]], -1, &fy, &ft, ebuf + etot, &list, &cap);
        etot += ext_in[k];
        /* outward: start at the innermost cluster, chain in ascending rows */
        ora_kf1_init(&fy, y[c[0]], fc->var_y, fc->var_slope0);
        ora_kf1_init(&ft, t[c[0]], fc->var_t, fc->var_slope0);
        for (int32_t j = 1; j < L; j++) {
            float dx = cfg->row_x[row[c[j]]] - cfg->row_x[row[c[j - 1]]];
            ora_kf1_predict(&fy, dx, fc->q_slope);
            ora_kf1_predict(&ft, dx, fc->q_slope);
            ora_kf1_update(&fy, y[c[j]], fc->var_y);
            ora_kf1_update(&ft, t[c[j]], fc->var_t);
        }
        ext_out[k] = ora_extend(cfg, fc, &R, y, t, row[c[L - 1]], 1, &fy, &ft, ebuf + etot, &list, &cap);
        etot += ext_out[k];
    }
    eoff[n_tracks] = etot;
    /* claims: (length desc, seed input index asc) */
    int32_t *bT = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *bS = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int64_t i = 0; i < n; i++) { bT[i] = -1; bS[i] = INT32_MAX; }
#define ORA_CLAIM(cl, T_, S_)                                                   \
    do {                                                                       \
        int32_t cc_ = (cl);                                                    \
        if ((T_) > bT[cc_] || ((T_) == bT[cc_] && (S_) < bS[cc_])) {           \
            bT[cc_] = (T_); bS[cc_] = (S_);                                    \
        }                                                                      \
    } while (0)
    for (int64_t k = 0; k < n_tracks; k++) {
        const int32_t *c = clusters + first[k];
        int32_t T = len[k] + ext_in[k] + ext_out[k], S = c[0];
        for (int32_t j = 0; j < len[k]; j++) ORA_CLAIM(c[j], T, S);
        for (int64_t e = eoff[k]; e < eoff[k + 1]; e++) ORA_CLAIM(ebuf[e], T, S);
    }
#undef ORA_CLAIM
    for (int64_t i = 0; i < n; i++) assign[i] = -1;
    int64_t nt = 0, nc = 0;
    for (int64_t k = 0; k < n_tracks; k++) {
        const int32_t *c = clusters + first[k];
        int32_t T = len[k] + ext_in[k] + ext_out[k], S = c[0];
        /* the extended track in ascending rows: inward reversed, chain, outward */
        int32_t m = 0;
        for (int32_t e = ext_in[k] - 1; e >= 0; e--) tmp[m++] = ebuf[eoff[k] + e];
        for (int32_t j = 0; j < len[k]; j++) tmp[m++] = c[j];
        for (int32_t e = 0; e < ext_out[k]; e++) tmp[m++] = ebuf[eoff[k] + ext_in[k] + e];
        int32_t keep = 0;
        for (int32_t j = 0; j < m; j++) keep += (bT[tmp[j]] == T && bS[tmp[j]] == S);
        if (keep < cfg->min_track_hits) { kept[k] = -1; continue; }
        kept[k] = keep;
        out_first[nt] = nc;
        out_len[nt] = keep;
        for (int32_t j = 0; j < m; j++)
            if (bT[tmp[j]] == T && bS[tmp[j]] == S) {
                out_clusters[nc++] = tmp[j];
                assign[tmp[j]] = (int32_t)nt;
            }
        nt++;
    }
    free(bT); free(bS); free(tmp); free(eoff); free(ebuf); free(list);
    ora_rows_free(&R);
    return nt;
}
