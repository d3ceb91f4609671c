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
//   k_t0_scan    one wave per (frame, side): group number of every bin
//   k_t0_group   per anchor: group number; per group: sum of t0 and count
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

// One block per sector instance.
__global__ __launch_bounds__(256) void k_t0_range(KArgs a, CollArgs c) {
    for (int si = blockIdx.x; si < a.n_si; si += gridDim.x) {
        const SiState S = a.st[si];
        const int h = side_of(a, si, c.n_sectors);
        for (int k = threadIdx.x; k < S.n_tracks; k += blockDim.x) {
            const float t0 = a.trk_t0[S.trk_base + k];
            if (!anchor(a, c, S.trk_base + k, t0)) continue;
            atomicMin(&c.range[2 * h], fkey(t0));
            atomicMax(&c.range[2 * h + 1], fkey(t0));
        }
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

// One wave per (frame, side), 64 bins at a time: a non-empty bin opens a
// group if the largest t0 of the previous non-empty bin lies more than the
// gap below its smallest t0. bin_grp[b] = group number (-1: empty bin).
__global__ __launch_bounds__(64) void k_t0_scan(CollArgs c) {
    const int h = blockIdx.x;
    const int nb = c.nbins[h];
    const int lane = threadIdx.x;
    const uint32_t *cnt = c.bin_cnt + c.bin_base[h];
    const uint32_t *bmin = c.bin_min + c.bin_base[h];
    const uint32_t *bmax = c.bin_max + c.bin_base[h];
    int32_t *grp = c.bin_grp + c.bin_base[h];
    float prev_max = 0.f;   // largest t0 of the last non-empty bin so far (wave-uniform)
    bool any = false;       // a non-empty bin has been seen
    int groups = 0;         // groups opened so far
    for (int b0 = 0; b0 < nb; b0 += 64) {
        const int b = b0 + lane;
        const bool ne = b < nb && cnt[b] > 0u;
        const float mn = ne ? fkey_inv(bmin[b]) : 0.f, mx = ne ? fkey_inv(bmax[b]) : 0.f;
        const uint64_t m = __ballot(ne);
        // the previous non-empty bin of this lane: the highest set lane below,
        // else the carry from earlier chunks
        const uint64_t below = m & ((1ull << lane) - 1ull);
        const int src = below ? 63 - __builtin_clzll(below) : 0;
        const float pm_lane = __shfl(mx, src);
        const bool has_prev = below != 0ull || any;
        const float pm = below ? pm_lane : prev_max;
        const bool opens = ne && (!has_prev || __fsub_rn(mn, pm) > c.gap);
        const uint64_t om = __ballot(opens);
        const int g = groups + __popcll(om & ((2ull << lane) - 1ull)) - 1;
        if (b < nb) grp[b] = ne ? g : -1;
        if (m) {
            const int last = 63 - __builtin_clzll(m);
            prev_max = __shfl(mx, last);
            any = true;
        }
        groups += __popcll(om);
    }
    if (lane == 0) c.n_groups[h] = groups;
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
        const double *sum = c.grp_sum + c.grp_base[h];
        const int32_t *cnt = c.grp_cnt + c.grp_base[h];
        for (int k = threadIdx.x; k < S.n_tracks; k += blockDim.x) {
            const int g = S.trk_base + k;
            const float t0f = a.trk_t0[g];
            if (!__builtin_isfinite(t0f) || a.trk_len[g] >= c.min_len) continue;
            const double v = (double)t0f;
            int lo = 0, hi = ng;   // first group of mean >= v in [lo, hi]
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (sum[mid] / (double)cnt[mid] < v) lo = mid + 1;
                else hi = mid;
            }
            const int j0 = max(lo - 1, 0), j1 = min(lo, ng - 1);
            const double d0 = fabs(v - sum[j0] / (double)cnt[j0]), d1 = fabs(v - sum[j1] / (double)cnt[j1]);
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
    if (n_sides > 0) hipLaunchKernelGGL(k_t0_scan, dim3(n_sides), dim3(64), 0, s, c);
}

void launch_t0_group(const KArgs &a, const CollArgs &c, hipStream_t s) {
    if (a.n_si > 0) hipLaunchKernelGGL(k_t0_group, dim3(min(a.n_si, 4096)), dim3(256), 0, s, a, c);
}

void launch_t0_attach(const KArgs &a, const CollArgs &c, hipStream_t s) {
    if (a.n_si > 0) hipLaunchKernelGGL(k_t0_attach, dim3(min(a.n_si, 4096)), dim3(256), 0, s, a, c);
}

}  // namespace tpcca
