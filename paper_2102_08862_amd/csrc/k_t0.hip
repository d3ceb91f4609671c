// Collision candidates from the tracks' collision times (after a run).
//
// Time is the seeding coordinate, so collisions are separated only after
// tracking (Sec. 1). Each fitted track carries its collision time t0 (the
// drift time of its helix at the closest approach to the beam line minus the
// drift length, computed by the fit's output step). Per frame and side (A:
// sectors 0 .. n/2-1, C: the rest) the anchors (tracks of at least min_len
// clusters with a finite t0: short tracks extrapolate too far to time the
// collision well) in ascending t0 form a new group wherever t0 jumps by more
// than a gap. No sort is needed: with bins of half the gap, two values of one
// bin never differ by more than the gap, so the groups follow from the
// smallest and largest t0 of each non-empty bin. A group's time is the mean
// t0 of its anchors; every other track with a finite t0 then joins the group
// of nearest time (the earlier on a tie) if it lies within a window.
//
//   k_t0_range   per (frame, side): smallest and largest anchor t0
//   k_t0_bins    per anchor: count, smallest and largest t0 of its bin
//   k_t0_scan    one workgroup per (frame, side): group number of every bin
//   k_t0_group   per anchor: group number; per group: sum of t0 and count
//   k_t0_mean    per group: mean t0 of its anchors
//   k_t0_attach  per other track: nearest group time by binary search
#include "tpcca_internal.h"

namespace tpcca {

namespace {

__device__ inline int side_of(const KArgs &a, int si, int n_sectors) {
    const int s = a.si[si].sector;
    return 2 * a.si[si].frame + (s >= n_sectors / 2 ? 1 : 0);
}

__device__ inline bool anchor(const KArgs &a, const CollArgs &c, int g, float t0) {
    return __builtin_isfinite(t0) && a.trk_len[g] >= c.min_len;
}

__device__ inline int bin_of(float t0, float lo, float inv_w) {
    return (int)floorf(__fmul_rn(__fsub_rn(t0, lo), inv_w));
}

}  // namespace

// One block per sector instance: the block's smallest and largest anchor
// t0, then one atomic each.
__global__ __launch_bounds__(256) void k_t0_range(KArgs a, CollArgs c) {
    __shared__ uint32_t smin, smax;
    for (int si = blockIdx.x; si < a.n_si; si += gridDim.x) {
        const SiState S = a.st[si];
        const int h = side_of(a, si, c.n_sectors);
        if (threadIdx.x == 0) {
            smin = 0xffffffffu;
            smax = 0u;
        }
        __syncthreads();
        uint32_t lmin = 0xffffffffu, lmax = 0u;
        for (int k = threadIdx.x; k < S.n_tracks; k += blockDim.x) {
            const float t0 = a.trk_t0[S.trk_base + k];
            if (!anchor(a, c, S.trk_base + k, t0)) continue;
            lmin = min(lmin, fkey(t0));
            lmax = max(lmax, fkey(t0));
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
            atomicMin(&c.range[2 * h], smin);
            atomicMax(&c.range[2 * h + 1], smax);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_t0_bins(KArgs a, CollArgs c) {
    for (int si = blockIdx.x; si < a.n_si; si += gridDim.x) {
        const SiState S = a.st[si];
        const int h = side_of(a, si, c.n_sectors);
        const int nb = c.nbins[h];
        if (nb <= 0) continue;
        const float lo = fkey_inv(c.range[2 * h]);
        uint32_t *cnt = c.bin_cnt + c.bin_base[h];
        uint32_t *bmin = c.bin_min + c.bin_base[h];
        uint32_t *bmax = c.bin_max + c.bin_base[h];
        for (int k = threadIdx.x; k < S.n_tracks; k += blockDim.x) {
            const float t0 = a.trk_t0[S.trk_base + k];
            if (!anchor(a, c, S.trk_base + k, t0)) continue;
            const int b = min(max(bin_of(t0, lo, c.inv_w), 0), nb - 1);
            atomicAdd(&cnt[b], 1u);
            atomicMin(&bmin[b], fkey(t0));
            atomicMax(&bmax[b], fkey(t0));
        }
    }
}

// One workgroup of kScanWaves waves per (frame, side), each wave a
// contiguous share of the bins, 64 at a time: a non-empty bin opens a group
// if the largest t0 of the previous non-empty bin lies more than the gap
// below its smallest t0. Three passes over a share: its last non-empty
// bin's largest t0; the opens, given the carry from the shares before; the
// group numbers, offset by the opens of the shares before.
// bin_grp[b] = group number (-1: empty bin).
constexpr int kScanWaves = 16;

__global__ __launch_bounds__(64 * kScanWaves) void k_t0_scan(CollArgs c) {
    __shared__ float s_last[kScanWaves];
    __shared__ int s_any[kScanWaves], s_opens[kScanWaves];
    const int h = blockIdx.x;
    const int nb = c.nbins[h];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t *cnt = c.bin_cnt + c.bin_base[h];
    const uint32_t *bmin = c.bin_min + c.bin_base[h];
    const uint32_t *bmax = c.bin_max + c.bin_base[h];
    int32_t *grp = c.bin_grp + c.bin_base[h];
    const int share = ((nb + kScanWaves - 1) / kScanWaves + 63) & ~63;
    const int b0 = min(w * share, nb), b1 = min(b0 + share, nb);
    // pass 1: the share's last non-empty bin
    float last = 0.f;
    bool any = false;
    for (int k0 = b0; k0 < b1; k0 += 64) {
        const int b = k0 + lane;
        const bool ne = b < b1 && cnt[b] > 0u;
        const uint64_t m = __ballot(ne);
        if (m) {
            const float mx = ne ? fkey_inv(bmax[b]) : 0.f;
            last = __shfl(mx, 63 - __builtin_clzll(m));
            any = true;
        }
    }
    if (lane == 0) {
        s_last[w] = last;
        s_any[w] = any;
    }
    __syncthreads();
    // carry: the last non-empty bin of the shares before
    bool have = false;
    float carry = 0.f;
    for (int v = w - 1; v >= 0; v--)
        if (s_any[v]) {
            have = true;
            carry = s_last[v];
            break;
        }
    // pass 2 counts the opens, pass 3 numbers the groups
    int opens = 0;
    for (int pass = 0; pass < 2; pass++) {
        int base = 0;
        if (pass == 1) {
            for (int v = 0; v < w; v++) base += s_opens[v];
        }
        bool hv = have;
        float pm_carry = carry;
        int groups = base;
        for (int k0 = b0; k0 < b1; k0 += 64) {
            const int b = k0 + lane;
            const bool ne = b < b1 && cnt[b] > 0u;
            const float mn = ne ? fkey_inv(bmin[b]) : 0.f, mx = ne ? fkey_inv(bmax[b]) : 0.f;
            const uint64_t m = __ballot(ne);
            const uint64_t below = m & ((1ull << lane) - 1ull);
            const int src = below ? 63 - __builtin_clzll(below) : 0;
            const float pm_lane = __shfl(mx, src);
            const bool has_prev = below != 0ull || hv;
            const float pm = below ? pm_lane : pm_carry;
            const bool op = ne && (!has_prev || __fsub_rn(mn, pm) > c.gap);
            const uint64_t om = __ballot(op);
            if (pass == 1 && b < b1) grp[b] = ne ? groups + __popcll(om & ((2ull << lane) - 1ull)) - 1 : -1;
            if (m) {
                pm_carry = __shfl(mx, 63 - __builtin_clzll(m));
                hv = true;
            }
            groups += __popcll(om);
        }
        if (pass == 0) {
            opens = groups;
            if (lane == 0) s_opens[w] = opens;
            __syncthreads();
        } else if (w == kScanWaves - 1 && lane == 0) {
            c.n_groups[h] = groups;
        }
    }
}

// Mean t0 of every group (after the group sums).
__global__ __launch_bounds__(256) void k_t0_mean(CollArgs c, int n_groups_total) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n_groups_total; g += gridDim.x * blockDim.x)
        c.grp_mean[g] = c.grp_cnt[g] > 0 ? c.grp_sum[g] / (double)c.grp_cnt[g] : 0.0;
}

__global__ __launch_bounds__(256) void k_t0_group(KArgs a, CollArgs c) {
    for (int si = blockIdx.x; si < a.n_si; si += gridDim.x) {
        const SiState S = a.st[si];
        const int h = side_of(a, si, c.n_sectors);
        const int nb = c.nbins[h];
        const float lo = nb > 0 ? fkey_inv(c.range[2 * h]) : 0.f;
        for (int k = threadIdx.x; k < S.n_tracks; k += blockDim.x) {
            const float t0 = a.trk_t0[S.trk_base + k];
            int g = -1;
            if (nb > 0 && anchor(a, c, S.trk_base + k, t0)) {
                const int b = min(max(bin_of(t0, lo, c.inv_w), 0), nb - 1);
                g = c.bin_grp[c.bin_base[h] + b];
                if (g >= 0 && c.grp_sum) {
                    atomicAdd(&c.grp_sum[c.grp_base[h] + g], (double)t0);
                    atomicAdd(&c.grp_cnt[c.grp_base[h] + g], 1);
                }
            }
            c.trk_group[S.trk_base + k] = g;
        }
    }
}

// Tracks that are not anchors: the group of nearest mean time, if within
// the window. Group times ascend within a side (groups are disjoint t0
// intervals in order), so a binary search finds the first group not earlier
// than t0; the candidates are it and the one before. FP64 as the group sums.
__global__ __launch_bounds__(256) void k_t0_attach(KArgs a, CollArgs c) {
    for (int si = blockIdx.x; si < a.n_si; si += gridDim.x) {
        const SiState S = a.st[si];
        const int h = side_of(a, si, c.n_sectors);
        const int ng = c.n_groups[h];
        if (ng <= 0) continue;
        const double *mean = c.grp_mean + c.grp_base[h];
        for (int k = threadIdx.x; k < S.n_tracks; k += blockDim.x) {
            const int g = S.trk_base + k;
            const float t0f = a.trk_t0[g];
            if (!__builtin_isfinite(t0f) || a.trk_len[g] >= c.min_len) continue;
            const double v = (double)t0f;
            int lo = 0, hi = ng;   // first group of mean >= v in [lo, hi]
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (mean[mid] < v) lo = mid + 1;
                else hi = mid;
            }
            const int j0 = max(lo - 1, 0), j1 = min(lo, ng - 1);
            const double d0 = fabs(v - mean[j0]), d1 = fabs(v - mean[j1]);
            const int near = d0 <= d1 ? j0 : j1;
            const double d = d0 <= d1 ? d0 : d1;
            if (d <= (double)c.window) {
                c.trk_group[g] = near;
                atomicAdd(&c.grp_att[c.grp_base[h] + near], 1);
            }
        }
    }
}

void launch_t0_range(const KArgs &a, const CollArgs &c, hipStream_t s) {
    if (a.n_si > 0) hipLaunchKernelGGL(k_t0_range, dim3(min(a.n_si, 4096)), dim3(256), 0, s, a, c);
}

void launch_t0_bins(const KArgs &a, const CollArgs &c, int n_sides, hipStream_t s) {
    if (a.n_si > 0) hipLaunchKernelGGL(k_t0_bins, dim3(min(a.n_si, 4096)), dim3(256), 0, s, a, c);
    if (n_sides > 0) hipLaunchKernelGGL(k_t0_scan, dim3(n_sides), dim3(64 * kScanWaves), 0, s, c);
}

void launch_t0_group(const KArgs &a, const CollArgs &c, hipStream_t s) {
    if (a.n_si > 0) hipLaunchKernelGGL(k_t0_group, dim3(min(a.n_si, 4096)), dim3(256), 0, s, a, c);
}

void launch_t0_attach(const KArgs &a, const CollArgs &c, int n_groups_total, hipStream_t s) {
    if (n_groups_total > 0)
        hipLaunchKernelGGL(k_t0_mean, dim3(min((n_groups_total + 255) / 256, 4096)), dim3(256), 0, s, c, n_groups_total);
    if (a.n_si > 0) hipLaunchKernelGGL(k_t0_attach, dim3(min(a.n_si, 4096)), dim3(256), 0, s, a, c);
}

}  // namespace tpcca
