// Cellular-automaton stage and track output.
//
//   k_seeds      one lane per cluster: mutual-link test of its up and down
//                links (cleaning), seed = mutual up link and no mutual down
//                link; seeds compacted with wave ballots
//   k_chainlen   one lane per seed: walk the chain of mutual links to its
//                end; chains with >= min_track_hits clusters are tracks; set
//                the seed's bit in the sector's input-index bitmap
//   (scan)       prefix popcounts of the bitmap give every track its number:
//                tracks are numbered in ascending seed input index
//   k_track_slot track slot, length and seed of every track
//   (scan)       prefix of lengths -> offsets of the cluster lists
//   k_emit       one lane per track: walk the chain again, write the
//                cluster list (input indices, rows ascending), the
//                assignment of every member, and the chain's (y, t, row)
//                contiguously for the fit
#include "tpcca_internal.h"

namespace tpcca {

// wave-level stream compaction: returns the output slot of lanes with pred
__device__ inline int wave_compact(bool pred, int32_t *counter) {
    const unsigned long long m = __ballot(pred);
    const int lane = __lane_id();
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    int base = 0;
    if (lane == 0 && m) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, 0);
    return base + before;
}

__global__ __launch_bounds__(256) void k_seeds(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    const int n = min(a.cnt->n_valid_total, a.n_in);
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const int p = base + threadIdx.x;
        bool seed = false;
        if (p < n) {
            const int2 l = a.link[p];
            const bool mu = l.x >= 0 && l.x < n && a.link[l.x].y == p;
            const bool md = l.y >= 0 && l.y < n && a.link[l.y].x == p;
            seed = mu && !md;
        }
        const int slot = wave_compact(seed, &a.cnt->n_seeds);
        if (seed && slot < a.seed_cap) a.seeds[slot] = p;
    }
}

void launch_seeds(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL(k_seeds, dim3(l.grid), dim3(256), 0, s, a);
}

__global__ __launch_bounds__(256) void k_chainlen(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    const int ns = min(a.cnt->n_seeds, a.seed_cap);
    const int nv = min(a.cnt->n_valid_total, a.n_in);
    const int stride = gridDim.x * blockDim.x;
    const int R = a.n_rows;
    for (int base = blockIdx.x * blockDim.x; base < ns; base += stride) {
        const int k = base + threadIdx.x;
        int p = 0, L = 0;
        if (k < ns) {
            p = a.seeds[k];
            int q = p;
            L = 1;
            for (int step = 0; step < R; step++) {
                const int u = a.link[q].x;
                if (u < 0 || u >= nv) break;
                if (a.link[u].y != q) break;
                q = u;
                L++;
            }
        }
        const bool trk = (k < ns) && L >= a.min_track_hits;
        const int slot = wave_compact(trk, &a.cnt->n_tseeds);
        if (trk && slot < a.tseed_cap) {
            a.tseed[slot] = p;
            a.tlen[slot] = L;
            const Rec e = a.rec[p];
            const int si = e.sr >> 8;
            atomicOr(&a.bits[a.si[si].word_base + (e.id >> 5)], 1u << (e.id & 31));
        }
    }
}

void launch_chainlen(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL(k_chainlen, dim3(l.grid), dim3(256), 0, s, a);
}

__global__ __launch_bounds__(256) void k_track_slot(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    const int nt = min(a.cnt->n_tseeds, a.tseed_cap);
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nt; k += gridDim.x * blockDim.x) {
        const int p = a.tseed[k];
        const Rec e = a.rec[p];
        const int si = e.sr >> 8;
        const int w = a.si[si].word_base + (e.id >> 5);
        const uint32_t below = a.bits[w] & ((1u << (e.id & 31)) - 1u);
        const int g = a.wpre[w] + __popc(below);
        a.tslot[k] = g;
        if (g < a.trk_cap) {
            a.trk_len[g] = a.tlen[k];
            a.trk_seed[g] = p;
        }
    }
}

void launch_track_slots(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL(k_track_slot, dim3(l.grid), dim3(256), 0, s, a);
}

__global__ void k_si_tracks(KArgs a) {
    for (int si = blockIdx.x * blockDim.x + threadIdx.x; si < a.n_si; si += gridDim.x * blockDim.x) {
        const SiDesc d = a.si[si];
        const int b = a.wpre[d.word_base];
        a.st[si].trk_base = b;
        a.st[si].n_tracks = a.wpre[d.word_base + d.nwords] - b;
    }
}

void launch_si_tracks(const KArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_si_tracks, dim3((a.n_si + 255) / 256), dim3(256), 0, s, a);
}

__global__ void k_si_clusters(KArgs a) {
    for (int si = blockIdx.x * blockDim.x + threadIdx.x; si < a.n_si; si += gridDim.x * blockDim.x) {
        const int b = a.st[si].trk_base, n = a.st[si].n_tracks;
        const int c0 = a.cl_off[b];
        a.st[si].cl_base = c0;
        a.st[si].n_cl = a.cl_off[b + n] - c0;
    }
}

void launch_si_clusters(const KArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_si_clusters, dim3((a.n_si + 255) / 256), dim3(256), 0, s, a);
}

__global__ __launch_bounds__(256) void k_emit(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    const int nt = min(a.cnt->n_tseeds, a.tseed_cap);
    const int R = a.n_rows;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nt; k += gridDim.x * blockDim.x) {
        const int g = a.tslot[k];
        if (g >= a.trk_cap) continue;
        int q = a.tseed[k];
        const int off = a.cl_off[g];
        const int L = a.trk_len[g];
        Rec e = a.rec[q];
        const int si = e.sr >> 8;
        const int tn = g - a.st[si].trk_base;
        const int inb = a.si[si].in_base;
        for (int j = 0; j < L && j <= R; j++) {
            a.clusters[off + j] = e.id;
            a.assign[inb + e.id] = tn;
            a.chain_yt[off + j] = make_float2(e.y, e.t);
            a.chain_row[off + j] = (uint8_t)(e.sr & 255);
            if (j + 1 < L) {
                q = a.link[q].x;
                e = a.rec[q];
            }
        }
    }
}

void launch_emit(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL(k_emit, dim3(l.grid), dim3(256), 0, s, a);
}

// ------------------------------------------------------------------ scans
// Three-phase exclusive scan over n elements (n possibly read from device
// memory): per-block sums, a single-block scan of the sums, block-local
// scans plus offsets. out[n] receives the total.

constexpr int kScanBlock = 256;
constexpr int kPerThread = kScanItems / kScanBlock;

struct PopcIn {
    const uint32_t *p;
    __device__ int operator()(int i) const { return __popc(p[i]); }
};
struct I32In {
    const int32_t *p;
    __device__ int operator()(int i) const { return p[i]; }
};

__device__ inline int block_excl_scan(int v, int *sh, int &total) {
    const int tid = threadIdx.x, n = blockDim.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < n; off <<= 1) {
        const int x = (tid >= off) ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += x;
        __syncthreads();
    }
    total = sh[n - 1];
    const int r = sh[tid] - v;
    __syncthreads();
    return r;
}

template <class F>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(F f, const int32_t *n_dev, int32_t n_host, int32_t n_cap,
                                                           int32_t *bsum) {
    __shared__ int sh[kScanBlock];
    const int n = n_dev ? min(*n_dev, n_cap) : n_host;
    const int nb = (n + kScanItems - 1) / kScanItems;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        int s = 0;
        const int base = b * kScanItems;
        for (int k = threadIdx.x; k < kScanItems; k += kScanBlock) {
            const int i = base + k;
            if (i < n) s += f(i);
        }
        int tot;
        block_excl_scan(s, sh, tot);
        if (threadIdx.x == 0) bsum[b] = tot;
    }
}

__global__ __launch_bounds__(1024) void k_scan_top(const int32_t *n_dev, int32_t n_host, int32_t n_cap,
                                                  int32_t *bsum) {
    __shared__ int sh[1024];
    const int n = n_dev ? min(*n_dev, n_cap) : n_host;
    const int nb = (n + kScanItems - 1) / kScanItems;
    int carry = 0;
    for (int base = 0; base < nb; base += blockDim.x) {
        const int i = base + threadIdx.x;
        const int v = (i < nb) ? bsum[i] : 0;
        int tot;
        const int e = block_excl_scan(v, sh, tot);
        if (i < nb) bsum[i] = carry + e;
        carry += tot;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

template <class F>
__global__ __launch_bounds__(kScanBlock) void k_scan_down(F f, const int32_t *n_dev, int32_t n_host, int32_t n_cap,
                                                         const int32_t *bsum, int32_t *out, int32_t *total_dst) {
    __shared__ int sh[kScanBlock];
    const int n = n_dev ? min(*n_dev, n_cap) : n_host;
    const int nb = (n + kScanItems - 1) / kScanItems;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const int base = b * kScanItems + threadIdx.x * kPerThread;
        int v[kPerThread];
        int s = 0;
#pragma unroll
        for (int k = 0; k < kPerThread; k++) {
            const int i = base + k;
            v[k] = (i < n) ? f(i) : 0;
            s += v[k];
        }
        int tot;
        int run = block_excl_scan(s, sh, tot) + bsum[b];
#pragma unroll
        for (int k = 0; k < kPerThread; k++) {
            const int i = base + k;
            if (i < n) out[i] = run;
            run += v[k];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        out[n] = bsum[nb];
        if (total_dst) *total_dst = bsum[nb];
    }
}

template <class F>
static void scan_impl(F f, const int32_t *n_dev, int32_t n_host, int32_t n_cap, int32_t *out, int32_t *total_dst,
                      int32_t *tmp, hipStream_t s) {
    const int nb_max = (n_cap + kScanItems - 1) / kScanItems;
    const int grid = max(1, min(nb_max, 2048));
    hipLaunchKernelGGL(k_scan_reduce<F>, dim3(grid), dim3(kScanBlock), 0, s, f, n_dev, n_host, n_cap, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, n_dev, n_host, n_cap, tmp);
    hipLaunchKernelGGL(k_scan_down<F>, dim3(grid), dim3(kScanBlock), 0, s, f, n_dev, n_host, n_cap, tmp, out,
                       total_dst);
}

void launch_scan_popc(const uint32_t *in, int32_t n, int32_t *out, int32_t *total_dst, int32_t *tmp,
                      hipStream_t s) {
    scan_impl(PopcIn{in}, nullptr, n, n, out, total_dst, tmp, s);
}

void launch_scan_i32_dev(const int32_t *in, const int32_t *n_dev, int32_t n_cap, int32_t *out, int32_t *total_dst,
                         int32_t *tmp, hipStream_t s) {
    scan_impl(I32In{in}, n_dev, 0, n_cap, out, total_dst, tmp, s);
}

}  // namespace tpcca
