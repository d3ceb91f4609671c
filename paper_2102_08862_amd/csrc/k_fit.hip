// Track fit: one lane per track, FP32 Kalman filter with the state
// (y, t, sin phi, dt/darc, q/pT) and its 5x5 covariance in registers.
//
// The helix is transported between pad rows in closed form (exact for a
// helix, no material): with kappa = -kB*q/pT,
//   s' = s + kappa*dx,  dy = dx*(s+s')/(c+c'),  chord L = sqrt(dx^2+dy^2),
//   darc = L*asin(kappa*L/2)/(kappa*L/2),  dt = tau*darc.
// The filter starts at the innermost cluster from a three-point estimate
// (circle through the first, middle and last cluster) which also centres
// Gaussian priors on (sin phi, tau, q/pT). Pass 1 is an extended Kalman
// filter; every further pass is a Kalman filter linearised about the helix of
// the previous pass's result carried back to the first cluster, i.e. one
// Gauss-Newton step of the maximum-a-posteriori problem, so the passes
// converge to the MAP helix. Passes stop when one changes no parameter by
// more than 1e-5 relative, or after kf_passes passes (status 4). Positions are kept relative to the first
// cluster so that FP32 resolves the sagitta of short tracks.
#include "tpcca_internal.h"

namespace tpcca {

// Hardware reciprocal and reciprocal square root (about 1 ulp), used only
// for the transport Jacobian and the Kalman gain: errors there change how
// fast the passes converge, not the helix they converge to. The reference
// trajectory itself (positions, arc lengths) keeps correctly rounded
// division and square root.
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
    return (rsq(1.f - u * u) - asinf(u) * rcp(u)) * rcp(u);
}

struct Jac {
    float ys, yk, ts, tt, tk, sk;
};

// transport q by dx; Jacobian if J != nullptr; false on |sin phi| >= smax.
// cs: cos phi of q if known (>= 0; a chain of transports hands each
// step's final cosine to the next), else -1; receives cos phi of qo.
__device__ inline bool transport(float kB, float smax, const float q[5], float dx, float qo[5], Jac *J,
                                 float &cs) {
    const float s = q[2], tau = q[3], k = q[4];
    const float kap = -kB * k;
    const float s1 = s + kap * dx;
    if (!(fabsf(s) < smax) || !(fabsf(s1) < smax)) return false;
    const float c = cs >= 0.f ? cs : sqrtf(1.f - s * s), c1 = sqrtf(1.f - s1 * s1);
    cs = c1;
    const float S = s + s1, C = c + c1;
    const float dy = dx * S / C;
    const float L = sqrtf(dx * dx + dy * dy);
    const float u = 0.5f * kap * L;
    if (!(fabsf(u) < 1.f)) return false;
    const float sgn = dx < 0.f ? -1.f : 1.f;
    const float dl = sgn * L * asin_ratio(u);
    qo[0] = q[0] + dy;
    qo[1] = q[1] + tau * dl;
    qo[2] = s1;
    qo[3] = tau;
    qo[4] = k;
    if (J) {
        const float iC = rcp(C), ic = rcp(c), ic1 = rcp(c1);
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
        J->sk = -kB * dx;
    }
    return true;
}

// d' = F d, C' = F C F^T for the sparse transport Jacobian
__device__ inline void apply_jac(const Jac &J, float d[5], float C[5][5]) {
    d[0] += J.ys * d[2] + J.yk * d[4];
    d[1] += J.ts * d[2] + J.tt * d[3] + J.tk * d[4];
    d[2] += J.sk * d[4];
    float T[5][5];
#pragma unroll
    for (int b = 0; b < 5; b++) {
        T[0][b] = C[0][b] + J.ys * C[2][b] + J.yk * C[4][b];
        T[1][b] = C[1][b] + J.ts * C[2][b] + J.tt * C[3][b] + J.tk * C[4][b];
        T[2][b] = C[2][b] + J.sk * C[4][b];
        T[3][b] = C[3][b];
        T[4][b] = C[4][b];
    }
#pragma unroll
    for (int a = 0; a < 5; a++) {
        C[a][0] = T[a][0] + J.ys * T[a][2] + J.yk * T[a][4];
        C[a][1] = T[a][1] + J.ts * T[a][2] + J.tt * T[a][3] + J.tk * T[a][4];
        C[a][2] = T[a][2] + J.sk * T[a][4];
        C[a][3] = T[a][3];
        C[a][4] = T[a][4];
    }
}

// measurement update with (ry, rt) = measurement - prediction
__device__ inline void kf_update(float d[5], float C[5][5], float ry, float rt, float vy, float vt) {
    const float S00 = C[0][0] + vy, S01 = C[0][1], S11 = C[1][1] + vt;
    const float idet = rcp(S00 * S11 - S01 * S01);
    const float i00 = S11 * idet, i01 = -S01 * idet, i11 = S00 * idet;
    float K0[5], K1[5];
#pragma unroll
    for (int a = 0; a < 5; a++) {
        K0[a] = C[a][0] * i00 + C[a][1] * i01;
        K1[a] = C[a][0] * i01 + C[a][1] * i11;
    }
#pragma unroll
    for (int a = 0; a < 5; a++) d[a] += K0[a] * ry + K1[a] * rt;
    float R0[5], R1[5];
#pragma unroll
    for (int b = 0; b < 5; b++) {
        R0[b] = C[0][b];
        R1[b] = C[1][b];
    }
#pragma unroll
    for (int a = 0; a < 5; a++)
#pragma unroll
        for (int b = 0; b <= a; b++) {
            const float v = C[a][b] - (K0[a] * R0[b] + K1[a] * R1[b]);
            C[a][b] = v;
            C[b][a] = v;
        }
}

constexpr float kConvTol = 1e-5f;

// State of one lane's track between passes.
struct FitLane {
    int g;                 // track slot; -1: none, -2: the queue is empty
    int pass, L;
    const Rec *ch;
    float x1, y1, t1, TL;
    float q0[5], ref1[5], est[5], prev[5];
    bool ok, conv;
};

// Three-point estimate at the first cluster of track g (circle through the
// first, middle and last cluster).
__device__ inline void fit_init(const KArgs &a, const float *sx, int g, FitLane &F) {
    const float kB = a.bz_kb;
    F.g = g;
    F.pass = 0;
    F.L = a.trk_len[g];
    F.ch = a.chain + a.off8[g];
    const Rec c1 = F.ch[0];
    const int m = (F.L + 1) / 2 - 1;
    const Rec cm = F.ch[m], cL = F.ch[F.L - 1];
    F.x1 = sx[c1.sr];
    F.y1 = c1.y;
    F.t1 = c1.t;
    const float Xm = sx[cm.sr] - F.x1, Ym = cm.y - F.y1;
    const float XL = sx[cL.sr] - F.x1;
    const float YL = cL.y - F.y1;
    F.TL = cL.t - F.t1;
    F.ok = true;
    F.conv = false;
#pragma unroll
    for (int i = 0; i < 5; i++) F.q0[i] = F.est[i] = F.prev[i] = 0.f;
    const float bcx = XL - Xm, bcy = YL - Ym;
    const float cr = Xm * YL - Ym * XL;
    const float dab = sqrtf(Xm * Xm + Ym * Ym), dac = sqrtf(XL * XL + YL * YL),
                dbc = sqrtf(bcx * bcx + bcy * bcy);
    if (!(dab > 0.f && dac > 0.f && dbc > 0.f)) F.ok = false;
    const float kap = 2.f * cr / (dab * dac * dbc);
    const float u = 0.5f * kap * dac;
    if (!(fabsf(u) < 1.f)) F.ok = false;
    if (F.ok) {
        const float phi = atan2f(YL, XL) - asinf(u);
        if (!(cosf(phi) > 0.f)) F.ok = false;
        F.q0[2] = sinf(phi);
        F.q0[3] = F.TL / (dac * asin_ratio(u));
        F.q0[4] = (kB != 0.f) ? -kap / kB : 0.f;
    }
#pragma unroll
    for (int i = 0; i < 5; i++) F.ref1[i] = F.q0[i];
}

__device__ inline void fit_output(const KArgs &a, const float *sx, const FitLane &F, const float (&C)[5][5],
                                  float chi2) {
    const int g = F.g;
    const Rec e0 = a.rec[a.trk_seed[g]];
    const int si = e0.sr >> 8;
    const Rec cL = F.ch[F.L - 1];
    tpcca_track o;
    o.frame = a.si[si].frame;
    o.sector = a.si[si].sector;
    o.n_clusters = F.L;
    o.status = F.ok ? (F.conv ? 0 : 4) : 2;
    o.first = (int64_t)(a.cl_off[g] - a.st[si].cl_base);
    o.seed = e0.id;
    o.ndf = 2 * F.L - 5;
    o.x_ref = sx[cL.sr];
    o.t_base = cL.t;
    if (F.ok) {
        o.y = F.y1 + F.est[0];
        o.dt = F.est[1] - F.TL;
        o.sinphi = F.est[2];
        o.tau = F.est[3];
        o.qpt = F.est[4];
        o.chi2 = chi2;
        int k = 0;
#pragma unroll
        for (int i = 0; i < 5; i++)
#pragma unroll
            for (int j = 0; j <= i; j++) o.cov[k++] = C[i][j];
    } else {
        o.y = o.dt = o.sinphi = o.tau = o.qpt = o.chi2 = 0.f;
#pragma unroll
        for (int i = 0; i < 15; i++) o.cov[i] = 0.f;
    }
    a.trk[g] = o;
}

// One pass over the chain; when the track is finished (converged, failed,
// or out of passes) its record is written and true returned.
__device__ inline bool fit_pass(const KArgs &a, const float *sx, FitLane &F) {
    const float kB = a.bz_kb, smax = a.s_max;
    const float vy = a.sigma_y2, vt = a.sigma_t2;
    const float ivy = 1.f / vy, ivt = 1.f / vt;
    const bool ext = (F.pass == 0);
    float ref[5], dev[5], C[5][5];
#pragma unroll
    for (int i = 0; i < 5; i++) {
        ref[i] = F.ref1[i];
        dev[i] = F.q0[i] - F.ref1[i];
    }
#pragma unroll
    for (int i = 0; i < 5; i++)
#pragma unroll
        for (int j = 0; j < 5; j++) C[i][j] = 0.f;
    C[0][0] = vy;
    C[1][1] = vt;
    C[2][2] = a.var_s;
    C[3][3] = a.var_tau;
    C[4][4] = a.var_k;
    float chi = ref[0] * ref[0] * ivy + ref[1] * ref[1] * ivt;
    float Xp = 0.f;
    float cs = -1.f;   // cos phi of ref (the extended filter moves ref: recomputed)
    for (int j = 1; j < F.L; j++) {
        const Rec cj = F.ch[j];
        const float Xj = sx[cj.sr] - F.x1;
        float rn[5];
        Jac J;
        if (ext) cs = -1.f;
        if (!transport(kB, smax, ref, Xj - Xp, rn, &J, cs)) {
            F.ok = false;
            fit_output(a, sx, F, C, 0.f);
            return true;
        }
        Xp = Xj;
        apply_jac(J, dev, C);
#pragma unroll
        for (int i = 0; i < 5; i++) ref[i] = rn[i];
        const float Yj = cj.y - F.y1, Tj = cj.t - F.t1;
        const float ey = Yj - ref[0], et = Tj - ref[1];
        chi += ey * ey * ivy + et * et * ivt;
        kf_update(dev, C, ey - dev[0], et - dev[1], vy, vt);
        if (ext) {
#pragma unroll
            for (int i = 0; i < 5; i++) {
                ref[i] += dev[i];
                dev[i] = 0.f;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 5; i++) F.est[i] = ref[i] + dev[i];
    // converged once a re-linearised pass moves no parameter by more than
    // kConvTol relative (floor 1 in every unit)
    if (F.pass > 0) {
        bool conv = true;
#pragma unroll
        for (int i = 0; i < 5; i++) conv = conv && fabsf(F.est[i] - F.prev[i]) <= kConvTol * fmaxf(fabsf(F.est[i]), 1.f);
        F.conv = conv;
    }
#pragma unroll
    for (int i = 0; i < 5; i++) F.prev[i] = F.est[i];
    bool done = F.conv || F.pass + 1 >= a.kf_passes;
    float cs0 = -1.f;
    if (!done && !transport(kB, smax, F.est, -Xp, F.ref1, nullptr, cs0)) {
        F.ok = false;
        done = true;
    }
    if (done) {
        fit_output(a, sx, F, C, chi);
        return true;
    }
    F.pass++;
    return false;
}

// Tracks come from a queue in order of decreasing length (so the lanes of a
// wave carry chains of nearly equal length), and a lane takes its next track
// as soon as its current one is finished: a wave runs one pass per step for
// every lane, so a track that needs more passes does not hold the other
// lanes of its wave idle.
__global__ __launch_bounds__(256) void k_fit(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    __shared__ float sx[kMaxRows];
    for (int r = threadIdx.x; r < a.n_rows; r += blockDim.x) sx[r] = a.row_x[r];
    __syncthreads();
    const int nt = min(a.cnt->n_tracks, a.trk_cap);
    const int lane = threadIdx.x & 63;
    FitLane F;
    F.g = -1;
    for (;;) {
        const bool need = F.g == -1;
        const uint64_t m = __ballot(need);
        if (m) {
            const int first = __ffsll((unsigned long long)m) - 1;
            int base = 0;
            if (lane == first) base = atomicAdd(&a.cnt->fit_next, __popcll(m));
            base = __shfl(base, first);
            if (need) {
                const int i = base + __popcll(m & ((1ull << lane) - 1ull));
                if (i < nt) {
                    fit_init(a, sx, a.perm[i], F);
                    if (!F.ok) {
                        const float Z[5][5] = {};
                        fit_output(a, sx, F, Z, 0.f);
                        F.g = -1;
                    }
                } else {
                    F.g = -2;
                }
            }
        }
        if (__all(F.g == -2)) break;
        if (F.g >= 0 && fit_pass(a, sx, F)) F.g = -1;
    }
}

void launch_fit(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL(k_fit, dim3(l.grid), dim3(256), 0, s, a);
}

}  // namespace tpcca
