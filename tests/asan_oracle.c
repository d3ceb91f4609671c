/* Driver that runs the oracle's C code under AddressSanitizer and
   UndefinedBehaviorSanitizer (host code only): one sector read from a
   binary file, then links, cleaning, chains, the MAP and Kalman fits, the
   track following and the triplet enumeration. Prints per step a few
   integer and floating-point sums, which the test compares with the same
   steps of the ordinary build.

   Input file (little endian): int64 n; int32 n_rows; float32 row_x[n_rows];
   float32 win_y, win_t, pair_c2; int32 max_gap, min_track_hits, max_iter;
   float64 bz, sigma_y, sigma_t, ivar_s, ivar_tau, ivar_k, s_max;
   float32 follow win_y, win_t, chi2_max, q_slope, var_y, var_t,
   var_slope0; int32 max_miss; uint8 row[n]; float32 y[n]; float32 t[n]. */
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/tpcoracle.c"

static void *rd(FILE *f, size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    if (!p || (bytes && fread(p, 1, bytes, f) != bytes)) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

int main(int argc, char **argv) {
    if (argc != 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t n;
    int32_t nr;
    if (fread(&n, 8, 1, f) != 1 || fread(&nr, 4, 1, f) != 1) return 2;
    float *row_x = rd(f, sizeof(float) * nr);
    ora_cfg c;
    c.n_rows = nr;
    c.row_x = row_x;
    float fw[3];
    int32_t iw[3];
    double dw[7];
    if (fread(fw, 4, 3, f) != 3 || fread(iw, 4, 3, f) != 3 || fread(dw, 8, 7, f) != 7) return 2;
    c.win_y = fw[0]; c.win_t = fw[1]; c.pair_c2 = fw[2];
    c.max_gap = iw[0]; c.min_track_hits = iw[1]; c.max_iter = iw[2];
    c.bz = dw[0]; c.sigma_y = dw[1]; c.sigma_t = dw[2];
    c.ivar_s = dw[3]; c.ivar_tau = dw[4]; c.ivar_k = dw[5]; c.s_max = dw[6];
    ora_follow_cfg fc;
    float ff[7];
    if (fread(ff, 4, 7, f) != 7 || fread(&fc.max_miss, 4, 1, f) != 1) return 2;
    fc.win_y = ff[0]; fc.win_t = ff[1]; fc.chi2_max = ff[2]; fc.q_slope = ff[3];
    fc.var_y = ff[4]; fc.var_t = ff[5]; fc.var_slope0 = ff[6];
    uint8_t *row = rd(f, n);
    float *y = rd(f, sizeof(float) * n), *t = rd(f, sizeof(float) * n);
    fclose(f);

    int32_t *up = malloc(4 * (n + 1)), *dn = malloc(4 * (n + 1)), *gap = malloc(4 * (n + 1));
    int32_t *upc = malloc(4 * (n + 1)), *dnc = malloc(4 * (n + 1));
    ora_links(&c, n, row, y, t, up, dn, gap);
    ora_clean(n, up, dn, upc, dnc);
    int64_t nl = 0, su = 0, nlc = 0;
    for (int64_t i = 0; i < n; i++) {
        nl += up[i] >= 0;
        su += up[i] + 2 * dn[i];
        nlc += upc[i] >= 0;
    }
    printf("links %lld %lld %lld\n", (long long)nl, (long long)su, (long long)nlc);

    int64_t *first = malloc(8 * (n + 1));
    int32_t *len = malloc(4 * (n + 1)), *cl = malloc(4 * (n + 1)), *asg = malloc(4 * (n + 1));
    const int64_t nt = ora_tracks(&c, n, upc, dnc, first, len, cl, asg);
    int64_t ntc = 0, sa = 0;
    for (int64_t k = 0; k < nt; k++) ntc += len[k];
    for (int64_t i = 0; i < n; i++) sa += asg[i];
    printf("tracks %lld %lld %lld\n", (long long)nt, (long long)ntc, (long long)sa);

    ora_fit *fit = malloc(sizeof(ora_fit) * (nt + 1));
    for (int kf = 0; kf <= 3; kf += 3) {
        ora_fit_tracks(&c, nt, first, len, cl, row, y, t, kf, fit);
        int64_t st = 0;
        double sq = 0.0, sc = 0.0;
        for (int64_t k = 0; k < nt; k++) {
            st += fit[k].status;
            if (fit[k].status == 0) {
                sq += fit[k].qpt;
                sc += fit[k].chi2;
            }
        }
        printf("fit%d %lld %.17g %.17g\n", kf, (long long)st, sq, sc);
    }

    int64_t *of = malloc(8 * (nt + 1));
    int32_t *ol = malloc(4 * (nt + 1)), *oc = malloc(4 * (n + 1)), *fa = malloc(4 * (n + 1));
    int32_t *ei = calloc(nt + 1, 4), *eo = calloc(nt + 1, 4), *kept = calloc(nt + 1, 4);
    const int64_t nk = ora_follow(&c, &fc, n, row, y, t, nt, first, len, cl, of, ol, oc, fa, ei, eo, kept);
    int64_t nkc = 0, se = 0;
    for (int64_t k = 0; k < nk; k++) nkc += ol[k];
    for (int64_t k = 0; k < nt; k++) se += ei[k] + 3 * eo[k] + 7 * kept[k];
    printf("follow %lld %lld %lld\n", (long long)nk, (long long)nkc, (long long)se);

    const int64_t ntr = ora_triplets(&c, n, row, y, t, 0, NULL, NULL);
    int32_t *tri = malloc(16 * (ntr + 1));
    float *feat = malloc(sizeof(float) * MLP_INP * (ntr + 1));
    ora_triplets(&c, n, row, y, t, ntr, tri, feat);
    int64_t stri = 0;
    double sf = 0.0;
    for (int64_t k = 0; k < ntr; k++) {
        stri += tri[4 * k] + tri[4 * k + 1] + tri[4 * k + 2] + tri[4 * k + 3];
        for (int j = 0; j < MLP_INP; j++) sf += feat[MLP_INP * k + j];
    }
    printf("triplets %lld %lld %.17g\n", (long long)ntr, (long long)stri, sf);

    free(row_x); free(row); free(y); free(t); free(up); free(dn); free(gap); free(upc); free(dnc);
    free(first); free(len); free(cl); free(asg); free(fit); free(of); free(ol); free(oc); free(fa);
    free(ei); free(eo); free(kept); free(tri); free(feat);
    return 0;
}
