// Track fit: FP32 helix fit of every track to the maximum-a-posteriori
// helix (data chi2 of all clusters plus Gaussian priors on sin phi, dt/darc
// and q/pT centred on a three-point estimate at the innermost cluster).
//
// The filter is the information form of the Kalman filter: each cluster's
// measurement update adds J^T W J to the information matrix and J^T W r to
// the information vector of the state at a reference point, so the updates
// of one pass are independent sums. Each pass linearises about the helix of
// the previous pass's result (one Gauss-Newton step of the MAP problem), so
// the passes converge to the MAP helix; the first pass linearises about the
// three-point estimate. The state (y, t, sin phi, dt/darc, q/pT) lives at
// the track's middle cluster x_c, with positions relative to that cluster,
// and every cluster's prediction is the closed-form helix transport from x_c
// (exact for a helix, no material): with kappa = -kB*q/pT,
//   s' = s + kappa*dx,  dy = dx*(s+s')/(c+c'),  chord L = sqrt(dx^2+dy^2),
//   darc = L*asin(kappa*L/2)/(kappa*L/2),  dt = tau*darc,
// so no rounding accumulates along the track and |dx| stays at most half
// the track's length. The prior on sin phi at the innermost cluster is a
// linear function of (sin phi, q/pT) at x_c and enters the normal equations
// exactly.
//
// Passes stop once a step moves no parameter by more than 3e-5 of
// max(|value|, floor, standard error) (floors 1 cm, 1 cm, 0.1, 0.1,
// 0.1 1/GeV; the standard error from the information matrix: FP32 rounding
// of the predictions leaves a few 1e-6 of a parameter's own uncertainty as
// noise, below which steps do not shrink), or after kf_passes passes
// (status 4). A pass whose objective rose by more than 1e-4 relative, or
// whose helix left the domain (|sin phi| >= s_max on the track), is undone
// and the step halved (at most 8 times in a row).
//
// Work layout: 4 lanes per track, 16 tracks per wave, taken from a queue in
// order of decreasing length (the tracks of a wave need about the same
// number of steps). Lane l of a track sums clusters l, l + 4, ... of the
// track's contiguous chain copy (4 consecutive records per track and load
// instruction; the copy stays in cache across the passes); the sums of a
// pass are reduced over the 4 lanes with cross-lane adds, and the 5x5 solve
// is repeated in the 4 lanes.
#include "tpcca_internal.h"

namespace tpcca {

constexpr int kFitG = 4;                              // lanes per track
constexpr int kFitPerWave = 64 / kFitG;               // tracks per wave
constexpr float kStepTol = 3e-5f;
constexpr float kCostTol = 1e-4f;
constexpr int kMaxHalvings = 8;
constexpr float kDriftLength = 250.f;   // cm: t = v_d t_coll + (drift length - |z|)

// Hardware reciprocal and reciprocal square root (about 1 ulp). In the
// Jacobian and the solve of the normal equations their errors change the
// size of a step, not the point where the steps vanish; in the predictions
// they add about an ulp to the FP32 rounding of each residual.
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// asin(u)/u and its derivative (Maclaurin series near 0)
__device__ inline float asin_ratio(float u) {
    if (fabsf(u) < 0.05f) {
        const float u2 = u * u;
        return 1.f + u2 * (1.f / 6.f + u2 * (3.f / 40.f + u2 * (5.f / 112.f)));
    }
    return asinf(u) / u;
}
__device__ inline float asin_ratio_d(float u) {
    if (fabsf(u) < 0.05f) {
        const float u2 = u * u;
        return u * (1.f / 3.f + u2 * (3.f / 10.f + u2 * (15.f / 56.f)));
    }
    const float iu = rcp(u);
    return (rsq(1.f - u * u) - asinf(u) * iu) * iu;
}

// Derivatives of the predicted (y, t) at x_c + dx with respect to the state
// at x_c: dy/dy0 = 1, dt/dt0 = 1 and these.
struct Jac {
    float ys, yk, ts, tt, tk;
};

// Helix transport of state q at x_c by dx (c0 = cos phi of q): predicted
// y, t and sin phi, and the Jacobian if J; false outside the domain.
__device__ inline bool transport(float kB, float smax, const float q[5], float c0, float dx, float &yo, float &to,
                                 float &so, Jac *J) {
    const float s = q[2], tau = q[3], k = q[4];
    const float kap = -kB * k;
    const float s1 = s + kap * dx;
    if (!(fabsf(s1) < smax)) return false;
    const float c1 = sqrtf(1.f - s1 * s1);
    const float S = s + s1, C = c0 + c1;
    const float dy = dx * S / C;
    const float L = sqrtf(dx * dx + dy * dy);
    const float u = 0.5f * kap * L;
    if (!(fabsf(u) < 1.f)) return false;
    const float sgn = dx < 0.f ? -1.f : 1.f;
    const float dl = sgn * L * asin_ratio(u);
    yo = q[0] + dy;
    to = q[1] + tau * dl;
    so = s1;
    if (J) {
        const float iC = rcp(C), ic = rcp(c0), ic1 = rcp(c1);
        J->ys = dx * (2.f * iC + S * (s * ic + s1 * ic1) * iC * iC);
        J->yk = -kB * dx * dx * (iC + S * s1 * ic1 * iC * iC);
        float dls = 0.f, dlk = 0.f;
        if (L > 0.f) {
            const float dldL = sgn * rsq(1.f - u * u);
            const float dyL = dy * rcp(L);
            dls = dldL * dyL * J->ys;
            dlk = dldL * dyL * J->yk - sgn * 0.5f * L * L * asin_ratio_d(u) * kB;
        }
        J->ts = tau * dls;
        J->tt = dl;
        J->tk = tau * dlk;
    }
    return true;
}

// asin(u)/u and its derivative for the passes: the Maclaurin series of
// asin (terms up to u^19, relative error below 1e-9 for |u| < 0.45), else
// asinf.
__device__ inline void asin_ratio_pair(float u, float &A, float &dA) {
    const float u2 = u * u;
    if (fabsf(u) < 0.45f) {
        // a_n = (2n)! / (4^n (n!)^2 (2n + 1)), n = 1..9
        constexpr float a1 = 1.f / 6.f, a2 = 3.f / 40.f, a3 = 15.f / 336.f, a4 = 35.f / 1152.f,
                        a5 = 63.f / 2816.f, a6 = 231.f / 13312.f, a7 = 143.f / 10240.f, a8 = 6435.f / 557056.f,
                        a9 = 12155.f / 1245184.f;
        A = 1.f + u2 * (a1 + u2 * (a2 + u2 * (a3 + u2 * (a4 + u2 * (a5 + u2 * (a6 + u2 * (a7 + u2 * (a8 + u2 * a9))))))));
        dA = u * (2.f * a1 + u2 * (4.f * a2 + u2 * (6.f * a3 + u2 * (8.f * a4 + u2 * (10.f * a5 + u2 * (12.f * a6 +
             u2 * (14.f * a7 + u2 * (16.f * a8 + u2 * (18.f * a9)))))))));
    } else {
        const float iu = rcp(u);
        A = asinf(u) * iu;
        dA = (rsq(1.f - u2) - A) * iu;
    }
}

// The transport of the passes (same formulas as transport): hardware square
// root and reciprocal (about 1 ulp each, below the FP32 rounding noise that
// the passes settle at), no early exit; ok is false outside the domain.
__device__ inline void transport_pass(float kB, float smax, const float q[5], float c0, float ic0, float dx,
                                      float &yo, float &to, Jac &J, bool &ok) {
    const float s = q[2], tau = q[3], k = q[4];
    const float kap = -kB * k;
    const float s1 = s + kap * dx;
    ok = ok && fabsf(s1) < smax;
    const float c1 = __builtin_amdgcn_sqrtf(fmaxf(1.f - s1 * s1, 0.f));
    const float S = s + s1, C = c0 + c1;
    const float iC = rcp(C);
    const float dy = dx * S * iC;
    const float L = __builtin_amdgcn_sqrtf(dx * dx + dy * dy);
    const float u = 0.5f * kap * L;
    ok = ok && fabsf(u) < 1.f;
    float A, dA;
    asin_ratio_pair(u, A, dA);
    const float sgn = dx < 0.f ? -1.f : 1.f;
    const float dl = sgn * L * A;
    yo = q[0] + dy;
    to = q[1] + tau * dl;
    const float ic1 = rcp(c1);
    J.ys = dx * (2.f * iC + S * (s * ic0 + s1 * ic1) * iC * iC);
    J.yk = -kB * dx * dx * (iC + S * s1 * ic1 * iC * iC);
    const float dldL = sgn * rsq(1.f - u * u);
    const float dyL = L > 0.f ? dy * rcp(L) : 0.f;
    J.ts = tau * (dldL * dyL * J.ys);
    J.tt = dl;
    J.tk = tau * (dldL * dyL * J.yk - sgn * 0.5f * L * L * dA * kB);
}

// Sums of one pass over a lane's clusters (reduced over the track's lanes).
//   information matrix: ys, yk, ys2, ysyk, yk2, ts, tt, tk, ts2, tstt, tstk,
//   tt2, tttk, tk2 (the y0/t0 diagonal is the cluster count);
//   information vector: ry, rt, ys*ry + .., tt*rt, ..; chi2
enum { kSys, kSyk, kSys2, kSysyk, kSyk2, kSts, kStt, kStk, kSts2, kStstt, kStstk, kStt2, kStttk, kStk2,
       kSry, kSrt, kSysry, kSykry, kStsrt, kSttrt, kStkrt, kSchi, kNSum };

// In-place Cholesky factorisation of a symmetric 5x5 matrix (lower
// triangle); false if not positive definite.
__device__ inline bool chol5(float A[5][5]) {
#pragma unroll
    for (int j = 0; j < 5; j++) {
        float d = A[j][j];
#pragma unroll
        for (int k = 0; k < j; k++) d -= A[j][k] * A[j][k];
        if (!(d > 0.f)) return false;
        const float il = rsq(d);
        A[j][j] = d * il;
#pragma unroll
        for (int i = j + 1; i < 5; i++) {
            float v = A[i][j];
#pragma unroll
            for (int k = 0; k < j; k++) v -= A[i][k] * A[j][k];
            A[i][j] = v * il;
        }
    }
    return true;
}

// Solve L L^T x = b with the factor from chol5.
__device__ inline void chol5_solve(const float Lm[5][5], const float b[5], float x[5]) {
    float z[5];
#pragma unroll
    for (int i = 0; i < 5; i++) {
        float v = b[i];
#pragma unroll
        for (int k = 0; k < i; k++) v -= Lm[i][k] * z[k];
        z[i] = v * rcp(Lm[i][i]);
    }
#pragma unroll
    for (int i = 4; i >= 0; i--) {
        float v = z[i];
#pragma unroll
        for (int k = i + 1; k < 5; k++) v -= Lm[k][i] * x[k];
        x[i] = v * rcp(Lm[i][i]);
    }
}

// Diagonal of H^-1 from the Cholesky factor L of H (H^-1 = L^-T L^-1).
__device__ inline void chol5_inv_diag(const float Lm[5][5], float dg[5]) {
    float Li[5][5];
#pragma unroll
    for (int i = 0; i < 5; i++) {
        const float ii = rcp(Lm[i][i]);
        Li[i][i] = ii;
#pragma unroll
        for (int j = 0; j < i; j++) {
            float v = 0.f;
#pragma unroll
            for (int k = j; k < i; k++) v += Lm[i][k] * Li[k][j];
            Li[i][j] = -v * ii;
        }
    }
#pragma unroll
    for (int i = 0; i < 5; i++) {
        float v = 0.f;
#pragma unroll
        for (int k = i; k < 5; k++) v += Li[k][i] * Li[k][i];
        dg[i] = v;
    }
}

// Sum of v over each aligned group of G lanes (G = 1, 2, 4, 8 or 16), in
// every lane of the group (cross-lane adds: swap neighbours, pairs, quads of
// a row, halves of a row).
template <int G>
__device__ inline float group_sum(float v) {
    static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group of 1, 2, 4, 8 or 16 lanes");
    if (G >= 2) v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
    if (G >= 4) v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
    if (G >= 8) v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
    if (G >= 16) v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));
    return v;
}

// A finished fit, parked in LDS until the wave writes its tracks out.
struct FitDone {
    float q[5], chi2;
    int32_t status, has_cov;
    float Hf[5][5];   // Cholesky factor of the information matrix at x_c (lower triangle)
};

// Output of a finished track at its outermost cluster (every lane of the
// track computes it, lane 0 writes): the state at x_c carried to x_L, the
// covariance from the Cholesky factor Hf of the information matrix at x_c
// (null: zero), C' = F H^-1 F^T.
// x of a cluster: the pad row's x, or (for refits of merged tracks, whose
// clusters come from two sectors) the x the record carries in its id field.
template <bool kX>
__device__ inline float xof(const float *sx, const Rec &e) {
    return kX ? __int_as_float(e.id) : sx[e.sr & 255];
}

template <bool kX>
__device__ inline void fit_emit(const KArgs &a, const float *sx, int g, int L, const Rec &e0, const Rec &cm, const Rec &cL,
                                float xc, const float q[5], float chi2, int status, const float (*Hf)[5],
                                bool writer) {
    const float kB = a.bz_kb, smax = a.s_max;
    const int si = e0.sr >> 8;
    tpcca_track o;
    o.frame = a.si[si].frame;
    o.sector = a.si[si].sector;
    o.n_clusters = L;
    o.first = (int64_t)(a.cl_off[g] - a.st[si].cl_base);
    o.seed = (kX || a.follow) ? a.trk_seed[g] : e0.id;   // with following (or a refit): the chain's seed
    o.ndf = 2 * L - 5;
    const float XL = xof<kX>(sx, cL) - xc;
    o.x_ref = xof<kX>(sx, cL);
    o.t_base = cL.t;
    float yo = 0.f, to = 0.f, so = 0.f;
    Jac J{};
    const bool fin = status != 2 && fabsf(q[2]) < smax &&
                     transport(kB, smax, q, sqrtf(1.f - q[2] * q[2]), XL, yo, to, so, &J);
    o.status = fin ? status : 2;
#pragma unroll
    for (int i = 0; i < 15; i++) o.cov[i] = 0.f;
    if (fin) {
        o.y = cm.y + yo;
        o.dt = to - (cL.t - cm.t);
        o.sinphi = so;
        o.tau = q[3];
        o.qpt = q[4];
        o.chi2 = chi2;
        if (Hf) {
            const float F[5][5] = {{1.f, 0.f, J.ys, 0.f, J.yk},
                                   {0.f, 1.f, J.ts, J.tt, J.tk},
                                   {0.f, 0.f, 1.f, 0.f, -kB * XL},
                                   {0.f, 0.f, 0.f, 1.f, 0.f},
                                   {0.f, 0.f, 0.f, 0.f, 1.f}};
            // columns of H^-1 F^T, one per row of F
            float W[5][5];
#pragma unroll
            for (int r = 0; r < 5; r++) chol5_solve(Hf, F[r], W[r]);
            int k = 0;
#pragma unroll
            for (int i = 0; i < 5; i++)
#pragma unroll
                for (int j = 0; j <= i; j++) {
                    float v = 0.f;
#pragma unroll
                    for (int m = 0; m < 5; m++) v += F[i][m] * W[j][m];
                    o.cov[k++] = v;
                }
        }
    } else {
        o.y = o.dt = o.sinphi = o.tau = o.qpt = o.chi2 = 0.f;
    }
    // collision time: the drift time at the helix's closest approach to the
    // beam line in the transverse plane, minus the drift length; the arc s
    // back to it solves tan(kappa s) = -a kappa / (1 + b kappa) with a, b the
    // position along and across the direction at x_ref
    float t0 = __builtin_nanf("");
    if (fin) {
        const float kap = -kB * o.qpt;
        const float cph = sqrtf(1.f - o.sinphi * o.sinphi);
        const float pa = o.x_ref * cph + o.y * o.sinphi, pb = o.y * cph - o.x_ref * o.sinphi;
        const float sd = kap != 0.f ? atan2f(-pa * kap, 1.f + pb * kap) / kap : -pa;
        t0 = (o.t_base + o.dt) + o.tau * sd - kDriftLength;
    }
    if (writer) {
        a.trk[g] = o;
        a.trk_t0[g] = t0;
    }
}

// Fit of the tracks at queue positions [base, base + 64 / G), G lanes each.
template <int G, bool kX>
__device__ void fit_wave(const KArgs &a, const float *sx, int32_t *hist, FitDone *done, int base, int nt) {
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);        // lane within the track's group
    const float kB = a.bz_kb, smax = a.s_max;
    const float wy = 1.f / a.sigma_y2, wt = 1.f / a.sigma_t2;
    const float ivs = 1.f / a.var_s, ivtau = 1.f / a.var_tau, ivk = 1.f / a.var_k;
    const float floor_[5] = {1.f, 1.f, 0.1f, 0.1f, 0.1f};
    const int qi = base + lane / G;
    const bool have = qi < nt;
    const int g = have ? a.perm[qi] : 0;
    const int L = have ? a.trk_len[g] : 0;
    const Rec *ch = a.chain + (have ? a.choff[g] : 0);
    // reference cluster (middle) and the clusters of this lane, relative
    const int mi = (L + 1) / 2 - 1;
    Rec cm = {}, c1 = {}, cL = {};
    if (have) {
        cm = ch[mi];
        c1 = ch[0];
        cL = ch[L - 1];
    }
    const float xc = xof<kX>(sx, cm);
    // three-point estimate at the innermost cluster (positions relative to it)
    const float X1 = xof<kX>(sx, c1) - xc;
    bool ok = have;
    float q0s = 0.f, q0tau = 0.f, q0k = 0.f;
    float q[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if (ok) {
        const float x1 = xof<kX>(sx, c1);
        const float Xm = xc - x1, Ym = cm.y - c1.y;
        const float XL = xof<kX>(sx, cL) - x1, YL = cL.y - c1.y, TL = cL.t - c1.t;
        const float bcx = XL - Xm, bcy = YL - Ym;
        const float cr = Xm * YL - Ym * XL;
        const float dab = sqrtf(Xm * Xm + Ym * Ym), dac = sqrtf(XL * XL + YL * YL),
                    dbc = sqrtf(bcx * bcx + bcy * bcy);
        if (!(dab > 0.f && dac > 0.f && dbc > 0.f)) ok = false;
        const float kap = 2.f * cr / (dab * dac * dbc);
        const float u = 0.5f * kap * dac;
        if (!(fabsf(u) < 1.f)) ok = false;
        if (ok) {
            const float phi = atan2f(YL, XL) - asinf(u);
            if (!(cosf(phi) > 0.f)) ok = false;
            q0s = sinf(phi);
            q0tau = TL / (dac * asin_ratio(u));
            q0k = (kB != 0.f) ? -kap / kB : 0.f;
        }
        // the three-point helix carried from the innermost cluster to x_c
        if (ok && !(fabsf(q0s) < smax)) ok = false;
        if (ok) {
            const float q1[5] = {c1.y - cm.y, c1.t - cm.t, q0s, q0tau, q0k};
            float yo, to, so;
            ok = transport(kB, smax, q1, sqrtf(1.f - q0s * q0s), -X1, yo, to, so, nullptr);
            q[0] = yo;
            q[1] = to;
            q[2] = so;
            q[3] = q0tau;
            q[4] = q0k;
        }
    }
    // running until the track's result is parked in done[] (lane 0 of the
    // track writes it)
    FitDone &D = done[lane / G];
    auto park = [&](const float *qf, float chi2, int st, const float (*Hf)[5]) {
        if (gl == 0) {
#pragma unroll
            for (int i = 0; i < 5; i++) D.q[i] = qf[i];
            D.chi2 = chi2;
            D.status = st;
            D.has_cov = Hf != nullptr;
            if (Hf)
#pragma unroll
                for (int i = 0; i < 5; i++)
#pragma unroll
                    for (int j = 0; j <= i; j++) D.Hf[i][j] = Hf[i][j];
        }
    };
    bool run = ok;
    if (have && !ok) {
        park(q, 0.f, 2, nullptr);
        if (gl == 0) atomicAdd(&hist[0], 1);
    }
    float best[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, best_chi = 0.f, best_cost = 0.f;
    bool have_best = false;
    int passes = 0, halv = 0, halv_total = 0;
    while (__any(run)) {
        // one pass: sums of this lane's clusters
        float sm[kNSum];
#pragma unroll
        for (int i = 0; i < kNSum; i++) sm[i] = 0.f;
        bool dom = run && fabsf(q[2]) < smax;
        if (dom) {
            const float c0 = sqrtf(1.f - q[2] * q[2]), ic0 = rcp(c0);
            for (int j = gl; j < L; j += G) {
                const Rec e = ch[j];
                float yo, to;
                Jac J;
                transport_pass(kB, smax, q, c0, ic0, xof<kX>(sx, e) - xc, yo, to, J, dom);
                const float ry = (e.y - cm.y) - yo, rt = (e.t - cm.t) - to;
                sm[kSys] += J.ys;
                sm[kSyk] += J.yk;
                sm[kSys2] += J.ys * J.ys;
                sm[kSysyk] += J.ys * J.yk;
                sm[kSyk2] += J.yk * J.yk;
                sm[kSts] += J.ts;
                sm[kStt] += J.tt;
                sm[kStk] += J.tk;
                sm[kSts2] += J.ts * J.ts;
                sm[kStstt] += J.ts * J.tt;
                sm[kStstk] += J.ts * J.tk;
                sm[kStt2] += J.tt * J.tt;
                sm[kStttk] += J.tt * J.tk;
                sm[kStk2] += J.tk * J.tk;
                sm[kSry] += ry;
                sm[kSrt] += rt;
                sm[kSysry] += J.ys * ry;
                sm[kSykry] += J.yk * ry;
                sm[kStsrt] += J.ts * rt;
                sm[kSttrt] += J.tt * rt;
                sm[kStkrt] += J.tk * rt;
                sm[kSchi] += ry * ry * wy + rt * rt * wt;
            }
        }
        // reduce over the G lanes of the track
#pragma unroll
        for (int i = 0; i < kNSum; i++) sm[i] = group_sum<G>(sm[i]);
        const uint64_t bad = __ballot(run && !dom);
        const uint64_t gmask = ((1ull << G) - 1ull) << (lane & ~(G - 1));
        dom = (bad & gmask) == 0ull;
        if (!run) continue;
        passes++;
        // objective: data chi2 plus the prior terms (sin phi at the
        // innermost cluster is s - kB*k*X1)
        const float ps = q0s - (q[2] - kB * q[4] * X1), pt = q0tau - q[3], pk = q0k - q[4];
        const float cost = sm[kSchi] + ps * ps * ivs + pt * pt * ivtau + pk * pk * ivk;
        if (!dom || (have_best && !(cost <= best_cost * (1.f + kCostTol)))) {
            // undo: halve the step from the best state
            int st = -1;
            if (!have_best) st = 2;
            else if (++halv > kMaxHalvings) st = 4;
            if (st >= 0) {
                park(have_best ? best : q, best_chi, st, nullptr);
                run = false;
            } else {
                halv_total++;
#pragma unroll
                for (int i = 0; i < 5; i++) q[i] = best[i] + 0.5f * (q[i] - best[i]);
            }
            continue;
        }
        halv = 0;
        have_best = true;
        best_cost = cost;
        best_chi = sm[kSchi];
#pragma unroll
        for (int i = 0; i < 5; i++) best[i] = q[i];
        const float nL = (float)L;
        const float a4 = -kB * X1;   // d(sin phi at the innermost cluster)/d(q/pT)
        float H[5][5];
        H[0][0] = wy * nL;
        H[1][0] = 0.f;
        H[1][1] = wt * nL;
        H[2][0] = wy * sm[kSys];
        H[2][1] = wt * sm[kSts];
        H[2][2] = wy * sm[kSys2] + wt * sm[kSts2] + ivs;
        H[3][0] = 0.f;
        H[3][1] = wt * sm[kStt];
        H[3][2] = wt * sm[kStstt];
        H[3][3] = wt * sm[kStt2] + ivtau;
        H[4][0] = wy * sm[kSyk];
        H[4][1] = wt * sm[kStk];
        H[4][2] = wy * sm[kSysyk] + wt * sm[kStstk] + ivs * a4;
        H[4][3] = wt * sm[kStttk];
        H[4][4] = wy * sm[kSyk2] + wt * sm[kStk2] + ivs * a4 * a4 + ivk;
        float gv[5];
        gv[0] = wy * sm[kSry];
        gv[1] = wt * sm[kSrt];
        gv[2] = wy * sm[kSysry] + wt * sm[kStsrt] + ivs * ps;
        gv[3] = wt * sm[kSttrt] + ivtau * pt;
        gv[4] = wy * sm[kSykry] + wt * sm[kStkrt] + ivs * a4 * ps + ivk * pk;
        if (!chol5(H)) {
            park(q, best_chi, 2, nullptr);
            run = false;
            continue;
        }
        float dq[5], var[5];
        chol5_solve(H, gv, dq);
        chol5_inv_diag(H, var);
        bool conv = true;
#pragma unroll
        for (int i = 0; i < 5; i++) {
            // the step is negligible against the value (or its floor) or
            // against the parameter's own standard error
            const float scale = fmaxf(fmaxf(fabsf(q[i]), floor_[i]), sqrtf(fmaxf(var[i], 0.f)));
            conv = conv && fabsf(dq[i]) <= kStepTol * scale;
            q[i] += dq[i];
        }
        if (conv || passes >= a.kf_passes) {
            // the covariance is that of the last linearisation
            park(q, best_chi, conv ? 0 : 4, H);
            run = false;
        }
    }
    if (ok && gl == 0) {
        atomicAdd(&hist[min(passes, kPassBins - 1)], 1);
        if (halv_total) atomicAdd(&hist[kPassBins], 1);
    }
    // the wave's LDS writes above are read by the other lanes of the track
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (have) {
        float qf[5];
#pragma unroll
        for (int i = 0; i < 5; i++) qf[i] = D.q[i];
        fit_emit<kX>(a, sx, g, L, c1, cm, cL, xc, qf, D.chi2, D.status, D.has_cov ? D.Hf : nullptr, gl == 0);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Every wave takes kFitPerWave tracks at a time from the queue (track slots
// in order of decreasing length, so the tracks of a wave have about the same
// length).
template <bool kX>
__global__ __launch_bounds__(256) void k_fit(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    __shared__ float sx[kMaxRows];
    __shared__ int32_t hist[kPassBins + 1];   // tracks by passes; [kPassBins]: fits with halved steps
    __shared__ FitDone done[256 / kFitG];
    FitDone *wd = done + (threadIdx.x >> 6) * kFitPerWave;
    for (int r = threadIdx.x; r < a.n_rows; r += blockDim.x) sx[r] = a.row_x[r];
    for (int i = threadIdx.x; i <= kPassBins; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const int nt = min(a.cnt->n_tracks, a.trk_cap);
    const int lane = threadIdx.x & 63;
    for (;;) {
        int base = 0;
        if (lane == 0) base = atomicAdd(&a.cnt->fit_next, kFitPerWave);
        base = __shfl(base, 0);
        if (base >= nt) break;
        fit_wave<kFitG, kX>(a, sx, hist, wd, base, nt);
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= kPassBins; i += blockDim.x)
        if (hist[i]) atomicAdd(&a.cnt->fit_passes[i], hist[i]);
}

void launch_fit(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL(k_fit<false>, dim3(l.grid), dim3(256), 0, s, a);
}

void launch_fit_x(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL(k_fit<true>, dim3(l.grid), dim3(256), 0, s, a);
}

}  // namespace tpcca
