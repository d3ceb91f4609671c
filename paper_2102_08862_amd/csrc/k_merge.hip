// Sector merging (after a run): a particle that crosses the border between
// two adjacent sectors of one side leaves a track in each. Time is the
// seeding coordinate, so this joining is deferred to after the tracking
// (Sec. 1); the tracks' collision times make the search local.
//
// Eligible tracks: fit ok, at least min_len clusters, finite collision time.
// A pair (A in sector s, B in the next sector of the same side, 360/(n/2)
// degrees further) with |t0_A - t0_B| <= window is scored from A's helix:
// B's reference point and direction rotated into A's frame, at (a, b)
// along and across A's direction; on A's circle (curvature kappa = -kB q/pT)
// the nearest point lies at the turning angle th = atan2(kappa a,
// 1 - kappa b), arc th / kappa (a if kappa = 0); the residuals are the
// transverse miss (2b - kappa (a^2 + b^2)) / (1 + sqrt((kappa a)^2 +
// (1 - kappa b)^2)), B's direction minus A's there, A's time there minus
// B's and tau_A - tau_B, and D2 = sum (residual / scale)^2 with scales 0.5
// cm, 0.02, 0.5 cm, 0.01. A pair is a candidate if D2 <= d2_cut and merged
// if each track is the other's best candidate (least D2, then least index).
//
// Membrane merging (a particle crossing z = 0 leaves a track in sector k of
// the A side and one in sector k + n/2 of the C side, at the same azimuth)
// runs the same kernels with pairs (k, k + n/2), no rotation, the time
// residual replaced by a test that the two time lines t0 + tau s meet
// between the pieces, and tau_A + tau_B in place of tau_A - tau_B (the
// drift time runs against z on the A side and with it on the C side).
//
//   k_mg_range   smallest and largest eligible t0 (block-reduced)
//   k_mg_count   eligible tracks per (sector instance, time bin)
//   (scan)       bin starts
//   k_mg_place   tracks grouped by bin, with a compact copy of their states
//   k_mg_best    per eligible track, in bin order (neighbouring threads read
//                overlapping candidate ranges): best candidate in the next
//                and in the previous sector, over the bins of
//                [t0 - 1.001 window, t0 + 1.001 window] (the bin index is
//                monotone in t0, so no candidate within the window is
//                missed)
//   k_mg_mutual  mutual bests -> partners
//   k_rf_*       refit of the merged pairs: pair list in the order of the
//                first track's slot, virtual tracks (clusters of both in the
//                first track's frame, ordered by x), then the fit kernel
//                with the x each record carries
#include "merge_internal.h"

namespace tpcca {

namespace {

constexpr float kSigR = 0.5f, kSigPhi = 0.02f, kSigT = 0.5f, kSigTau = 0.01f;

__device__ inline int si_of(const KArgs &a, const MergeArgs &m, int g) {
    const tpcca_track &T = a.trk[g];
    return T.frame * m.n_sectors + T.sector;
}

__device__ inline bool eligible(const KArgs &a, const MergeArgs &m, int g) {
    const float t0 = a.trk_t0[g];
    return a.trk[g].status == 0 && a.trk_len[g] >= m.min_len && __builtin_isfinite(t0);
}

struct MState {
    float x, y, t, s, tau, q, t0, phi;
};

__device__ inline MState mstate(const MergeArgs &m, int p) {
    const float4 u = m.mst[2 * p], v = m.mst[2 * p + 1];
    return MState{u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
}

__device__ inline int bin_of(const MergeArgs &m, float t0) {
    const int b = (int)floorf((t0 - m.lo) * m.inv_w);
    return min(max(b, 0), m.nb - 1);
}

// D2 of the pair (A, B) with B's sector dal further in azimuth; infinite
// once the tau term alone exceeds the cut (D2 is a sum of squares, and an
// FP32 sum of non-negative terms is at least each of them, so no candidate
// is lost).
__device__ inline float pair_d2(const MState &A, const MState &B, float kB, float cdal, float sdal, float dal,
                                float cut) {
    const float r3 = (A.tau - B.tau) / kSigTau;
    if (!(r3 * r3 <= cut)) return __builtin_inff();
    const float ca = sqrtf(fmaxf(1.f - A.s * A.s, 0.f));
    const float xb = B.x * cdal - B.y * sdal, yb = B.x * sdal + B.y * cdal;
    const float vx = xb - A.x, vy = yb - A.y;
    const float a = vx * ca + vy * A.s, b = -vx * A.s + vy * ca;
    const float k = -kB * A.q;
    const float th = atan2f(k * a, 1.f - k * b);
    const float arc = k != 0.f ? th / k : a;
    const float h = sqrtf((k * a) * (k * a) + (1.f - k * b) * (1.f - k * b));
    const float dr = (2.f * b - k * (a * a + b * b)) / (1.f + h);
    // direction difference wrapped to (-pi, pi]
    float dphi = B.phi + dal - (A.phi + th);
    const float pi = 3.14159265358979f;
    while (dphi > pi) dphi -= 2.f * pi;
    while (dphi <= -pi) dphi += 2.f * pi;
    const float dt = A.t + A.tau * arc - B.t;
    const float r0 = dr / kSigR, r1 = dphi / kSigPhi, r2 = dt / kSigT;
    return r0 * r0 + r1 * r1 + r2 * r2 + r3 * r3;
}

// Membrane pairs: A in sector k (A side), B in sector k + n/2, the same
// azimuth. D2 of the transverse miss, the direction difference and
// tau_A + tau_B; infinite unless the time lines t0 + tau s of the two meet
// (within kMemSTol of time) at an arc s between the two states' arcs from
// the beam line, widened by kMemSMargin: a particle crossing z = 0 ends one
// piece and starts the other there.
constexpr float kMemSMargin = 5.f, kMemSTol = 1.f;

// Transverse arc from the beam line's closest approach to the state.
__device__ inline float ref_arc(const MState &X, float kB) {
    const float c = sqrtf(fmaxf(1.f - X.s * X.s, 0.f));
    const float a = X.x * c + X.y * X.s, b = -X.x * X.s + X.y * c;
    const float k = -kB * X.q;
    return k != 0.f ? -atan2f(-a * k, 1.f + b * k) / k : a;
}

__device__ inline float pair_d2_mem(const MState &A, const MState &B, float kB, float cut) {
    const float r3 = (A.tau + B.tau) / kSigTau;   // as in pair_d2: the cheap term first
    if (!(r3 * r3 <= cut)) return __builtin_inff();
    const float D = A.tau - B.tau, dT = B.t0 - A.t0;
    const float sa = ref_arc(A, kB), sb = ref_arc(B, kB);
    const float e0 = D * (fminf(sa, sb) - kMemSMargin), e1 = D * (fmaxf(sa, sb) + kMemSMargin);
    if (!(dT >= fminf(e0, e1) - kMemSTol && dT <= fmaxf(e0, e1) + kMemSTol)) return __builtin_inff();
    const float ca = sqrtf(fmaxf(1.f - A.s * A.s, 0.f));
    const float vx = B.x - A.x, vy = B.y - A.y;
    const float a = vx * ca + vy * A.s, b = -vx * A.s + vy * ca;
    const float k = -kB * A.q;
    const float th = atan2f(k * a, 1.f - k * b);
    const float h = sqrtf((k * a) * (k * a) + (1.f - k * b) * (1.f - k * b));
    const float dr = (2.f * b - k * (a * a + b * b)) / (1.f + h);
    float dphi = B.phi - (A.phi + th);
    const float pi = 3.14159265358979f;
    while (dphi > pi) dphi -= 2.f * pi;
    while (dphi <= -pi) dphi += 2.f * pi;
    const float r0 = dr / kSigR, r1 = dphi / kSigPhi;
    return r0 * r0 + r1 * r1 + r3 * r3;
}

}  // namespace

__global__ __launch_bounds__(256) void k_mg_range(KArgs a, MergeArgs m) {
    __shared__ uint32_t smin, smax;
    for (int si = blockIdx.x; si < a.n_si; si += gridDim.x) {
        const SiState S = a.st[si];
        if (threadIdx.x == 0) {
            smin = 0xffffffffu;
            smax = 0u;
        }
        __syncthreads();
        uint32_t lmin = 0xffffffffu, lmax = 0u;
        for (int k = threadIdx.x; k < S.n_tracks; k += blockDim.x) {
            const int g = S.trk_base + k;
            if (!eligible(a, m, g)) continue;
            lmin = min(lmin, fkey(a.trk_t0[g]));
            lmax = max(lmax, fkey(a.trk_t0[g]));
        }
        for (int off = 32; off > 0; off >>= 1) {
            lmin = min(lmin, (uint32_t)__shfl_xor((int)lmin, off));
            lmax = max(lmax, (uint32_t)__shfl_xor((int)lmax, off));
        }
        if ((threadIdx.x & 63) == 0) {
            atomicMin(&smin, lmin);
            atomicMax(&smax, lmax);
        }
        __syncthreads();
        if (threadIdx.x == 0 && smin <= smax) {
            atomicMin(&m.range[0], smin);
            atomicMax(&m.range[1], smax);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_mg_count(KArgs a, MergeArgs m) {
    for (int si = blockIdx.x; si < a.n_si; si += gridDim.x) {
        const SiState S = a.st[si];
        for (int k = threadIdx.x; k < S.n_tracks; k += blockDim.x) {
            const int g = S.trk_base + k;
            if (eligible(a, m, g)) atomicAdd(&m.start[(int64_t)si * m.nb + bin_of(m, a.trk_t0[g])], 1);
        }
    }
}

__global__ __launch_bounds__(256) void k_mg_place(KArgs a, MergeArgs m) {
    for (int si = blockIdx.x; si < a.n_si; si += gridDim.x) {
        const SiState S = a.st[si];
        for (int k = threadIdx.x; k < S.n_tracks; k += blockDim.x) {
            const int g = S.trk_base + k;
            if (!eligible(a, m, g)) continue;
            const int64_t c = (int64_t)si * m.nb + bin_of(m, a.trk_t0[g]);
            const int p = m.start[c] + atomicAdd(&m.cur[c], 1);
            const tpcca_track &T = a.trk[g];
            m.list[p] = g;
            m.mst[2 * p] = make_float4(T.x_ref, T.y, T.t_base + T.dt, T.sinphi);
            m.mst[2 * p + 1] = make_float4(T.tau, T.qpt, a.trk_t0[g], asinf(T.sinphi));
        }
    }
}

// One thread per eligible track, in list order (grid-stride over the list):
// its best candidate in the next sector (it is A) and in the previous sector
// (it is B); across the membrane, an A-side track's best in the C-side
// sector of its azimuth, a C-side track's best in the A-side one.
__global__ __launch_bounds__(256) void k_mg_best(KArgs a, MergeArgs m) {
    const int half = m.n_sectors / 2;
    const float dal = 6.283185307179586f / (float)half;
    const float cdal = cosf(dal), sdal = sinf(dal);
    const float kB = a.bz_kb;
    const int ne = *m.n_elig;
    const float wide = m.window * 1.001f;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < ne; p += gridDim.x * blockDim.x) {
        const int g = m.list[p];
        const MState X = mstate(m, p);
        const int si = si_of(a, m, g);
        const int fr = si / m.n_sectors, sec = si - fr * m.n_sectors;
        const int side = sec / half, k = sec - side * half;
        const int si_next = m.membrane ? (side == 0 ? fr * m.n_sectors + half + k : -1)
                                       : fr * m.n_sectors + side * half + (k + 1) % half;
        const int si_prev = m.membrane ? (side == 1 ? fr * m.n_sectors + k : -1)
                                       : fr * m.n_sectors + side * half + (k + half - 1) % half;
        const int b0 = bin_of(m, X.t0 - wide), b1 = bin_of(m, X.t0 + wide);
        int bn = -1, bp = -1;
        float dn = 0.f, dp = 0.f;
        for (int dir = 0; dir < 2; dir++) {
            const int sj = dir == 0 ? si_next : si_prev;
            if (sj < 0) continue;
            const int64_t base = (int64_t)sj * m.nb;
            const int j0 = m.start[base + b0], j1 = m.start[base + b1 + 1];
            for (int j = j0; j < j1; j++) {
                const MState Y = mstate(m, j);
                if (!(fabsf(X.t0 - Y.t0) <= m.window)) continue;
                const float d2 = m.membrane ? (dir == 0 ? pair_d2_mem(X, Y, kB, m.d2_cut) : pair_d2_mem(Y, X, kB, m.d2_cut))
                                            : (dir == 0 ? pair_d2(X, Y, kB, cdal, sdal, dal, m.d2_cut)
                                                        : pair_d2(Y, X, kB, cdal, sdal, dal, m.d2_cut));
                if (!(d2 <= m.d2_cut)) continue;
                const int h = m.list[j];
                if (dir == 0) {
                    if (bn < 0 || d2 < dn || (d2 == dn && h < bn)) {
                        bn = h;
                        dn = d2;
                    }
                } else if (bp < 0 || d2 < dp || (d2 == dp && h < bp)) {
                    bp = h;
                    dp = d2;
                }
            }
        }
        m.best_next[g] = bn;
        m.best_prev[g] = bp;
    }
}

__global__ __launch_bounds__(256) void k_mg_mutual(KArgs a, MergeArgs m) {
    const int nt = min(a.cnt->n_tracks, a.trk_cap);
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nt; g += gridDim.x * blockDim.x) {
        const int h = m.best_next[g];
        if (h >= 0 && m.best_prev[h] == g) {
            m.partner_next[g] = h;
            m.partner_prev[h] = g;
            atomicAdd(m.n_pairs, 1);
        }
    }
}

// ------------------------------------------------------------ refit
constexpr int kRfMax = 2 * kMaxRows + 2;   // clusters of a virtual track

__global__ __launch_bounds__(256) void k_rf_flags(KArgs a, MergeArgs m, RefitArgs r, int nt) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nt; g += gridDim.x * blockDim.x)
        r.flags[g] = m.partner_next[g] >= 0 ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_rf_pairs(KArgs a, MergeArgs m, RefitArgs r, int nt) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nt; g += gridDim.x * blockDim.x) {
        const int h = m.partner_next[g];
        if (h < 0) continue;
        const int i = r.pidx[g];
        r.pa[i] = g;
        r.pb[i] = h;
        r.vlen[i] = min(a.trk_len[g] + a.trk_len[h], kRfMax);
        r.vseed[i] = (int32_t)a.trk[g].seed;   // the first track's seed as reported
        r.vperm[i] = i;
    }
}

// One wave per pair: the clusters of both tracks in the first track's frame
// (the partner's rotated by the sector angle), each placed at its rank by x
// (ties in the order first track, then partner, each in its own order).

__global__ __launch_bounds__(256) void k_rf_build(KArgs a, RefitArgs r, int np) {
    __shared__ float xs_all[4][kRfMax];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float *xs = xs_all[w];
    const int half = r.n_sectors / 2;
    const float dal = 6.283185307179586f / (float)half;
    const float cd = cosf(dal), sd = sinf(dal);
    const int nw = gridDim.x * (blockDim.x >> 6);
    for (int i = blockIdx.x * (blockDim.x >> 6) + w; i < np; i += nw) {
        const int g = r.pa[i], h = r.pb[i];
        const int LA = a.trk_len[g], LB = a.trk_len[h], L = min(LA + LB, kRfMax);
        const Rec *ca = a.chain + a.choff[g], *cb = a.chain + a.choff[h];
        const int si = ca[0].sr >> 8;
        constexpr int kPer = (kRfMax + 63) / 64;
        float xx[kPer], yy[kPer], tt[kPer];
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            const int j = lane + 64 * u;
            xx[u] = yy[u] = tt[u] = 0.f;
            if (j < L) {
                const Rec e = j < LA ? ca[j] : cb[j - LA];
                const float x = a.row_x[e.sr & 255];
                if (j < LA) {
                    xx[u] = x;
                    yy[u] = e.y;
                } else {
                    xx[u] = x * cd - e.y * sd;
                    yy[u] = x * sd + e.y * cd;
                }
                tt[u] = e.t;
                xs[j] = xx[u];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        Rec *dst = r.vchain + r.voff[i];
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            const int j = lane + 64 * u;
            if (j < L) {
                int rank = 0;
                for (int k = 0; k < L; k++) rank += (xs[k] < xx[u] || (xs[k] == xx[u] && k < j)) ? 1 : 0;
                dst[rank] = Rec{yy[u], tt[u], __float_as_int(xx[u]), si << 8};
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

void launch_refit_flags(const KArgs &a, const MergeArgs &m, const RefitArgs &r, int n_tracks, hipStream_t s) {
    if (n_tracks > 0)
        hipLaunchKernelGGL(k_rf_flags, dim3(min((n_tracks + 255) / 256, 65535)), dim3(256), 0, s, a, m, r, n_tracks);
}

void launch_refit_pairs(const KArgs &a, const MergeArgs &m, const RefitArgs &r, int n_tracks, hipStream_t s) {
    if (n_tracks > 0)
        hipLaunchKernelGGL(k_rf_pairs, dim3(min((n_tracks + 255) / 256, 65535)), dim3(256), 0, s, a, m, r, n_tracks);
}

void launch_refit_build(const KArgs &a, const RefitArgs &r, int n_pairs, hipStream_t s) {
    if (n_pairs > 0) hipLaunchKernelGGL(k_rf_build, dim3(min((n_pairs + 3) / 4, 65535)), dim3(256), 0, s, a, r, n_pairs);
}

void launch_merge_range(const KArgs &a, const MergeArgs &m, hipStream_t s) {
    if (a.n_si > 0) hipLaunchKernelGGL(k_mg_range, dim3(min(a.n_si, 4096)), dim3(256), 0, s, a, m);
}

void launch_merge_count(const KArgs &a, const MergeArgs &m, hipStream_t s) {
    if (a.n_si > 0) hipLaunchKernelGGL(k_mg_count, dim3(min(a.n_si, 4096)), dim3(256), 0, s, a, m);
}

void launch_merge_place(const KArgs &a, const MergeArgs &m, hipStream_t s) {
    if (a.n_si > 0) hipLaunchKernelGGL(k_mg_place, dim3(min(a.n_si, 4096)), dim3(256), 0, s, a, m);
}

void launch_merge_pairs(const KArgs &a, const MergeArgs &m, int n_tracks, int n_elig, hipStream_t s) {
    if (n_elig > 0) hipLaunchKernelGGL(k_mg_best, dim3(min((n_elig + 255) / 256, 65535)), dim3(256), 0, s, a, m);
    if (n_tracks > 0) hipLaunchKernelGGL(k_mg_mutual, dim3(min((n_tracks + 255) / 256, 65535)), dim3(256), 0, s, a, m);
}

}  // namespace tpcca
