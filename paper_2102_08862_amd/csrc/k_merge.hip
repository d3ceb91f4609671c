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
//   k_mg_range   smallest and largest eligible t0 (block-reduced)
//   k_mg_count   eligible tracks per (sector instance, time bin)
//   (scan)       bin starts
//   k_mg_place   tracks grouped by bin
//   k_mg_best    per eligible track: best candidate in the next and in the
//                previous sector (bins within one of its own: the bin width
//                is a power of two >= window from a multiple of it, so bin
//                indices are exact and a pair within the window is at most
//                one bin apart)
//   k_mg_mutual  mutual bests -> partners
#include "merge_internal.h"

namespace tpcca {

namespace {

constexpr float kSigR = 0.5f, kSigPhi = 0.02f, kSigT = 0.5f, kSigTau = 0.01f;

struct TrkState {
    float x, y, t, s, tau, q, t0;
};

__device__ inline int si_of(const KArgs &a, const MergeArgs &m, int g) {
    const tpcca_track &T = a.trk[g];
    return T.frame * m.n_sectors + T.sector;
}

__device__ inline bool eligible(const KArgs &a, const MergeArgs &m, int g) {
    const float t0 = a.trk_t0[g];
    return a.trk[g].status == 0 && a.trk_len[g] >= m.min_len && __builtin_isfinite(t0);
}

__device__ inline TrkState state_of(const KArgs &a, int g) {
    const tpcca_track &T = a.trk[g];
    return TrkState{T.x_ref, T.y, T.t_base + T.dt, T.sinphi, T.tau, T.qpt, a.trk_t0[g]};
}

__device__ inline int bin_of(const MergeArgs &m, float t0) {
    const int b = (int)floorf((t0 - m.lo) * m.inv_w);
    return min(max(b, 0), m.nb - 1);
}

// D2 of the pair (A, B) with B's sector dal further in azimuth.
__device__ inline float pair_d2(const TrkState &A, const TrkState &B, float kB, float cdal, float sdal, float dal) {
    const float ca = sqrtf(fmaxf(1.f - A.s * A.s, 0.f));
    const float xb = B.x * cdal - B.y * sdal, yb = B.x * sdal + B.y * cdal;
    const float vx = xb - A.x, vy = yb - A.y;
    const float a = vx * ca + vy * A.s, b = -vx * A.s + vy * ca;
    const float k = -kB * A.q;
    const float th = atan2f(k * a, 1.f - k * b);
    const float arc = k != 0.f ? th / k : a;
    const float h = sqrtf((k * a) * (k * a) + (1.f - k * b) * (1.f - k * b));
    const float dr = (2.f * b - k * (a * a + b * b)) / (1.f + h);
    float dphi = asinf(B.s) + dal - (asinf(A.s) + th);
    dphi = atan2f(sinf(dphi), cosf(dphi));
    const float dt = A.t + A.tau * arc - B.t;
    const float dtau = A.tau - B.tau;
    const float r0 = dr / kSigR, r1 = dphi / kSigPhi, r2 = dt / kSigT, r3 = dtau / kSigTau;
    return r0 * r0 + r1 * r1 + r2 * r2 + r3 * r3;
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
            m.list[m.start[c] + atomicAdd(&m.cur[c], 1)] = g;
        }
    }
}

// One thread per eligible track (grid-stride over the track slots): its
// best candidate in the next sector (it is A) and in the previous sector
// (it is B).
__global__ __launch_bounds__(256) void k_mg_best(KArgs a, MergeArgs m) {
    const int half = m.n_sectors / 2;
    const float dal = 6.283185307179586f / (float)half;
    const float cdal = cosf(dal), sdal = sinf(dal);
    const float kB = a.bz_kb;
    const int nt = min(a.cnt->n_tracks, a.trk_cap);
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nt; g += gridDim.x * blockDim.x) {
        int bn = -1, bp = -1;
        if (eligible(a, m, g)) {
            const int si = si_of(a, m, g);
            const int fr = si / m.n_sectors, sec = si - fr * m.n_sectors;
            const int side = sec / half, k = sec - side * half;
            const int si_next = fr * m.n_sectors + side * half + (k + 1) % half;
            const int si_prev = fr * m.n_sectors + side * half + (k + half - 1) % half;
            const TrkState X = state_of(a, g);
            const int b = bin_of(m, X.t0);
            const int b0 = max(b - 1, 0), b1 = min(b + 1, m.nb - 1);
            float dn = 0.f, dp = 0.f;
            for (int dir = 0; dir < 2; dir++) {
                const int64_t base = (int64_t)(dir == 0 ? si_next : si_prev) * m.nb;
                const int j0 = m.start[base + b0], j1 = m.start[base + b1 + 1];
                for (int j = j0; j < j1; j++) {
                    const int h = m.list[j];
                    const TrkState Y = state_of(a, h);
                    if (!(fabsf(X.t0 - Y.t0) <= m.window)) continue;
                    const float d2 = dir == 0 ? pair_d2(X, Y, kB, cdal, sdal, dal) : pair_d2(Y, X, kB, cdal, sdal, dal);
                    if (!(d2 <= m.d2_cut)) continue;
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

void launch_merge_range(const KArgs &a, const MergeArgs &m, hipStream_t s) {
    if (a.n_si > 0) hipLaunchKernelGGL(k_mg_range, dim3(min(a.n_si, 4096)), dim3(256), 0, s, a, m);
}

void launch_merge_count(const KArgs &a, const MergeArgs &m, hipStream_t s) {
    if (a.n_si > 0) hipLaunchKernelGGL(k_mg_count, dim3(min(a.n_si, 4096)), dim3(256), 0, s, a, m);
}

void launch_merge_place(const KArgs &a, const MergeArgs &m, hipStream_t s) {
    if (a.n_si > 0) hipLaunchKernelGGL(k_mg_place, dim3(min(a.n_si, 4096)), dim3(256), 0, s, a, m);
}

void launch_merge_pairs(const KArgs &a, const MergeArgs &m, int n_tracks, hipStream_t s) {
    if (n_tracks <= 0) return;
    const int blocks = min((n_tracks + 255) / 256, 65535);
    hipLaunchKernelGGL(k_mg_best, dim3(blocks), dim3(256), 0, s, a, m);
    hipLaunchKernelGGL(k_mg_mutual, dim3(blocks), dim3(256), 0, s, a, m);
}

}  // namespace tpcca
