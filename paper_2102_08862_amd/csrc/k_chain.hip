// Cellular-automaton stage and track output.
//
//   k_seeds      one lane per cluster: mutual-link test of its up and down
//                links (cleaning), kept up links written out (one 4-byte
//                gather per chain step afterwards); seed = mutual up link
//                and no mutual down link; seeds compacted with wave ballots
//   k_walk       one lane per seed: walk the chain of mutual links to its
//                end; chains with >= min_track_hits clusters are tracks: set
//                the seed's bit in the sector's input-index bitmap and copy
//                the chain's clusters {y, t, id, sector/row} to a reserved
//                run of the chain copies (walked again, links in cache)
//   (scan)       prefix popcounts of the bitmap give every track its number:
//                tracks are numbered in ascending seed input index
//   k_track_slot track slot, length and seed of every track
//   (scan)       prefix of lengths -> offsets of the cluster lists
//   k_lists      cluster lists (input indices, rows ascending) and the
//                assignment, through per-bucket runs
//   k_asg_fill   the assignment, one bucket of input indices at a time
#include "tpcca_internal.h"

namespace tpcca {

// block-wide exclusive scan of one int per thread (blockDim <= 1024)
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


// Compaction of a block's flags: one global atomic per chunk of kCompactChunk
// positions, so that the single output counter is not contended. Inside a
// chunk the seeds are listed in position order (sub-chunk k of 256
// positions, then wave, then lane), so that neighbouring lanes of the chain
// walk start from neighbouring clusters of one pad row and their walks
// gather from the same cache lines.
constexpr int kCompactPer = 32;
constexpr int kCompactChunk = 256 * kCompactPer;

__global__ __launch_bounds__(256) void k_seeds(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    __shared__ int s_cnt[kCompactPer * 4 + 1];
    __shared__ int s_base;
    const int n = min(a.cnt->n_valid_total, a.n_in);
    const int nch = (n + kCompactChunk - 1) / kCompactChunk;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int c = blockIdx.x; c < nch; c += gridDim.x) {
        const int base = c * kCompactChunk;
        uint32_t mask = 0;
#pragma unroll 4
        for (int k = 0; k < kCompactPer; k++) {
            const int p = base + k * 256 + tid;
            bool seed = false;
            if (p < n) {
                const int2 l = a.link[p];
                const bool mu = l.x >= 0 && l.x < n && a.link[l.x].y == p;
                const bool md = l.y >= 0 && l.y < n && a.link[l.y].x == p;
                a.upc[p] = mu ? l.x : -1;
                seed = mu && !md;
                if (seed) mask |= 1u << k;
            }
            const uint64_t b = __ballot(seed);
            if (lane == 0) s_cnt[k * 4 + wv] = __popcll(b);
        }
        __syncthreads();
        // exclusive prefix over the (sub-chunk, wave) counts in position order
        if (tid < 64) {
            int carry = 0;
            for (int i0 = 0; i0 < kCompactPer * 4; i0 += 64) {
                const int v = s_cnt[i0 + tid];
                int x = v;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int y = __shfl_up(x, o);
                    if (tid >= o) x += y;
                }
                s_cnt[i0 + tid] = carry + x - v;
                carry += __shfl(x, 63);
            }
            if (tid == 0) {
                s_base = carry ? atomicAdd(&a.cnt->n_seeds, carry) : 0;
                s_cnt[kCompactPer * 4] = carry;
            }
        }
        __syncthreads();
        const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll 4
        for (int k = 0; k < kCompactPer; k++) {
            const bool seed = (mask >> k) & 1u;
            const uint64_t b = __ballot(seed);
            if (seed) {
                const int o = s_base + s_cnt[k * 4 + wv] + __popcll(b & below);
                if (o < a.seed_cap) a.seeds[o] = base + k * 256 + tid;
            }
        }
        __syncthreads();
    }
}

void launch_seeds(const KArgs &a, Launch l, hipStream_t s) {
    const int nch = (a.n_in + kCompactChunk - 1) / kCompactChunk;
    hipLaunchKernelGGL(k_seeds, dim3(max(1, min(l.grid, nch))), dim3(256), 0, s, a);
}

// One lane per seed: walk the chain of mutual links to its end (one 4-byte
// cleaned-link gather per step); a chain of >= min_track_hits clusters is a
// track: its seed bit is set in the sector's input-index bitmap, and a second
// walk of the same chain (its links now in cache) copies its clusters
// {y, t, input index, (sector instance << 8) | row} to a run of the chain
// copies that the wave reserves with one atomic (runs of a multiple of 4
// entries, so the fit's loads of 4 consecutive records are 64-byte aligned).
constexpr int kWalkBatch = 4;
// positions of a chain's first clusters kept in registers by the first walk,
// so that the second walk gathers their records without chasing the links
constexpr int kWalkKeep = 32;

__device__ inline int wave_excl_sum(int v, int &total) {
    const int lane = threadIdx.x & 63;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    total = __shfl(x, 63);
    return x - v;
}

__global__ __launch_bounds__(256) void k_walk(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    const int ns = min(a.cnt->n_seeds, a.seed_cap);
    const int R = a.n_rows;
    const int lane = threadIdx.x & 63;
    const int stride = gridDim.x * blockDim.x;
    // uniform per wave: every lane of a wave runs the same iterations
    for (int base = blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < ns; base += stride) {
        const int k = base + lane;
        int p = 0, L = 0;
        int pos[kWalkKeep];
        if (k < ns) {
            p = a.seeds[k];
            int q = p;
            L = 1;
            pos[0] = p;
            // L - 1 steps taken so far, at most R in all
#pragma unroll
            for (int j = 1; j < kWalkKeep; j++) {
                if (L == j && j <= R) {
                    const int u = a.upc[q];   // mutual up link (cleaned)
                    if (u >= 0) {
                        q = u;
                        L++;
                    }
                }
                pos[j] = q;
            }
            if (L == kWalkKeep) {
                for (int step = kWalkKeep - 1; step < R; step++) {
                    const int u = a.upc[q];
                    if (u < 0) break;
                    q = u;
                    L++;
                }
            }
        }
        const bool trk = (k < ns) && L >= a.min_track_hits;
        const int len4 = trk ? (L + kWalkBatch - 1) & ~(kWalkBatch - 1) : 0;
        int n_trk, n_ent;
        const int r_trk = wave_excl_sum(trk ? 1 : 0, n_trk);
        const int r_ent = wave_excl_sum(len4, n_ent);
        int s0 = 0, c0 = 0;
        if (lane == 0 && n_trk) {
            s0 = atomicAdd(&a.cnt->n_tseeds, n_trk);
            c0 = atomicAdd(&a.cnt->chain_next, n_ent);
        }
        s0 = __shfl(s0, 0);
        c0 = __shfl(c0, 0);
        const int slot = s0 + r_trk;
        const int64_t off = (int64_t)c0 + r_ent;
        if (trk && slot < a.tseed_cap && off + len4 <= (int64_t)a.chain_cap) {
            a.tseed[slot] = p;
            a.tlen[slot] = L;
            a.tchoff[slot] = (int32_t)off;
            const Rec e0 = a.rec[p];
            const int si = e0.sr >> 8;
            atomicOr(&a.bits[a.si[si].word_base + (e0.id >> 5)], 1u << (e0.id & 31));
            Rec *dst = a.chain + off;
            // the first kWalkKeep clusters: independent gathers
#pragma unroll
            for (int j0 = 0; j0 < kWalkKeep; j0 += kWalkBatch) {
                if (j0 < L) {
                    Rec buf[kWalkBatch];
#pragma unroll
                    for (int b = 0; b < kWalkBatch; b++) {
                        const int j = j0 + b;
                        if (j < L) {
                            buf[b] = a.rec[pos[j]];
                            if (a.follow) buf[b].id = pos[j];   // the following reads sorted positions
                        } else {
                            buf[b] = Rec{0.f, 0.f, -1, e0.sr};
                        }
                    }
#pragma unroll
                    for (int b = 0; b < kWalkBatch; b++)
                        reinterpret_cast<int4 *>(dst + j0)[b] = *reinterpret_cast<const int4 *>(&buf[b]);
                }
            }
            // the rest: follow the links on from the last kept position
            int q = pos[kWalkKeep - 1];
            for (int j0 = kWalkKeep; j0 < L; j0 += kWalkBatch) {
                Rec buf[kWalkBatch];
#pragma unroll
                for (int b = 0; b < kWalkBatch; b++) {
                    const int j = j0 + b;
                    if (j < L) {
                        q = a.upc[q];
                        buf[b] = a.rec[q];
                        if (a.follow) buf[b].id = q;
                    } else {
                        buf[b] = Rec{0.f, 0.f, -1, e0.sr};
                    }
                }
#pragma unroll
                for (int b = 0; b < kWalkBatch; b++)
                    reinterpret_cast<int4 *>(dst + j0)[b] = *reinterpret_cast<const int4 *>(&buf[b]);
            }
        } else if (trk) {
            atomicAdd(&a.cnt->overflow, 1);
        }
    }
}

void launch_walk(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL(k_walk, dim3(l.grid), dim3(256), 0, s, a);
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
            a.choff[g] = a.tchoff[k];
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

// Canonical cluster lists and the assignment. The lists: the input indices
// of the chain copies, written in list order (the lists of a range of tracks
// are contiguous). The assignment is a permutation from track order to input
// order; instead of one scattered 4-byte store per cluster it goes through
// buckets of kAsgBucket input indices: each workgroup takes a range of tracks, counts its clusters per
// bucket in LDS, reserves one run per bucket and writes (input index, track
// number) pairs there; k_asg_fill then builds each bucket's slice of the
// assignment in LDS (-1 where no pair) and writes it out whole.
constexpr int kAsgBucket = 16384;          // input indices per bucket (64 KB of assignment)
constexpr int kAsgTracks = 512;            // tracks per workgroup range
constexpr int kAsgHist = 4096;             // buckets a range may span (else direct stores)

__global__ __launch_bounds__(256) void k_lists(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    __shared__ int32_t h[kAsgHist];
    // per-track values of the range, loaded in parallel once (a track's
    // sector and offsets are a chain of dependent loads)
    __shared__ int32_t m_len[kAsgTracks], m_cl[kAsgTracks], m_choff[kAsgTracks], m_ib[kAsgTracks],
        m_tn[kAsgTracks];
    __shared__ int32_t s_lo, s_span;
    const int nt = min(a.cnt->n_tracks, a.trk_cap);
    for (int g0 = blockIdx.x * kAsgTracks; g0 < nt; g0 += gridDim.x * kAsgTracks) {
        const int g1 = min(g0 + kAsgTracks, nt);
        for (int g = g0 + threadIdx.x; g < g1; g += blockDim.x) {
            const int si = a.chain[a.choff[g]].sr >> 8;
            const int k = g - g0;
            m_len[k] = a.trk_len[g];
            m_cl[k] = a.cl_off[g];
            m_choff[k] = a.choff[g];
            m_ib[k] = a.si[si].in_base;
            m_tn[k] = g - a.st[si].trk_base;
            if (g == g0) s_lo = a.si[si].in_base / kAsgBucket;
            if (g == g1 - 1) s_span = (a.si[si].in_base + a.si[si].n) / kAsgBucket;   // last bucket of the range
        }
        __syncthreads();
        const int blo = s_lo, span = s_span - s_lo + 1;
        const bool bucketed = span <= kAsgHist;
        if (bucketed) {
            for (int b = threadIdx.x; b < span; b += blockDim.x) h[b] = 0;
            __syncthreads();
        }
        // lists, and the bucket counts: each wave takes whole tracks of the
        // range, its lanes the track's clusters (coalesced record loads and
        // list stores, no search for a position's track)
        const int nk = g1 - g0;
        const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
        for (int k = threadIdx.x >> 6; k < nk; k += nw) {
            const int L = m_len[k], cl = m_cl[k], co = m_choff[k], ib = m_ib[k], tn = m_tn[k];
            for (int j = lane; j < L; j += 64) {
                const int id = a.chain[co + j].id;
                a.clusters[cl + j] = id;
                const int gi = ib + id;
                if (bucketed) {
                    atomicAdd(&h[gi / kAsgBucket - blo], 1);
                } else {
                    const int bk = gi / kAsgBucket;   // a range spanning many sectors: one grab per pair
                    a.asg_pairs[(int64_t)bk * kAsgBucket + atomicAdd(&a.asg_cnt[bk], 1)] = make_int2(gi, tn);
                }
            }
        }
        if (bucketed) {   // uniform
            __syncthreads();
            for (int b = threadIdx.x; b < span; b += blockDim.x) {
                const int v = h[b];
                // runs are reserved inside the bucket's fixed region (a bucket
                // holds at most kAsgBucket pairs: one per input index)
                h[b] = v ? (blo + b) * kAsgBucket + atomicAdd(&a.asg_cnt[blo + b], v) : 0;   // < n_in + kAsgBucket
            }
            __syncthreads();
            for (int k = threadIdx.x >> 6; k < nk; k += nw) {
                const int L = m_len[k], cl = m_cl[k], ib = m_ib[k], tn = m_tn[k];
                for (int j = lane; j < L; j += 64) {
                    const int gi = ib + a.clusters[cl + j];
                    a.asg_pairs[(int64_t)atomicAdd(&h[gi / kAsgBucket - blo], 1)] = make_int2(gi, tn);
                }
            }
        }
        __syncthreads();
    }
}

// One workgroup per bucket: the bucket's slice of the assignment (16-byte
// vectors for the fill and the write-out; 1024 threads, as two 64 KB images
// fit a CU).
constexpr int kAsgFillBlock = 1024;

__global__ __launch_bounds__(kAsgFillBlock) void k_asg_fill(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    __shared__ int4 img4[kAsgBucket / 4];
    int32_t *img = reinterpret_cast<int32_t *>(img4);
    const int nb = (a.n_in + kAsgBucket - 1) / kAsgBucket;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const int i0 = b * kAsgBucket, m = min(kAsgBucket, a.n_in - i0);
        for (int k = threadIdx.x; k < kAsgBucket / 4; k += blockDim.x) img4[k] = make_int4(-1, -1, -1, -1);
        __syncthreads();
        const int np = min(a.asg_cnt[b], kAsgBucket);
        const int2 *pr = a.asg_pairs + (int64_t)i0;
        for (int k = threadIdx.x; k < np; k += blockDim.x) {
            const int2 v = pr[k];
            const int o = v.x - i0;
            if ((unsigned)o < (unsigned)m) img[o] = v.y;
        }
        __syncthreads();
        // i0 is a multiple of kAsgBucket: the slice starts 16-byte aligned
        int4 *dst4 = reinterpret_cast<int4 *>(a.assign + i0);
        for (int k = threadIdx.x; k < m / 4; k += blockDim.x) dst4[k] = img4[k];
        for (int k = (m & ~3) + threadIdx.x; k < m; k += blockDim.x) a.assign[i0 + k] = img[k];
        __syncthreads();
    }
}

void launch_lists(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL(k_lists, dim3(l.grid), dim3(256), 0, s, a);
    const int nb = (a.n_in + kAsgBucket - 1) / kAsgBucket;
    if (nb > 0) hipLaunchKernelGGL(k_asg_fill, dim3(min(nb, 4096)), dim3(kAsgFillBlock), 0, s, a);
}

// Track slots ordered by decreasing chain length (counting sort), so that the
// lanes of a fit wave carry chains of nearly equal length.
__global__ __launch_bounds__(256) void k_len_hist(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    __shared__ int h[kLenBins];
    for (int b = threadIdx.x; b < kLenBins; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const int nt = min(a.cnt->n_tracks, a.trk_cap);
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nt; g += gridDim.x * blockDim.x)
        atomicAdd(&h[min(a.trk_len[g], kLenBins - 1)], 1);
    __syncthreads();
    for (int b = threadIdx.x; b < kLenBins; b += blockDim.x)
        if (h[b]) atomicAdd(&a.lhist[b], h[b]);
}

__global__ __launch_bounds__(kLenBins) void k_len_scan(KArgs a) {
    __shared__ int sh[kLenBins];
    // bucket b (length) goes before shorter buckets: scan in decreasing length
    const int b = kLenBins - 1 - (int)threadIdx.x;
    const int v = a.lhist[b];
    int tot;
    const int e = block_excl_scan(v, sh, tot);
    a.lhist[b] = e;
}

constexpr int kLenPer = 8;

__global__ __launch_bounds__(256) void k_len_scatter(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    __shared__ int h[kLenBins], base[kLenBins];
    const int nt = min(a.cnt->n_tracks, a.trk_cap);
    const int chunk = 256 * kLenPer;
    for (int g0 = blockIdx.x * chunk; g0 < nt; g0 += gridDim.x * chunk) {
        for (int b = threadIdx.x; b < kLenBins; b += blockDim.x) h[b] = 0;
        __syncthreads();
        int lb[kLenPer];
#pragma unroll
        for (int k = 0; k < kLenPer; k++) {
            const int g = g0 + k * 256 + threadIdx.x;
            lb[k] = (g < nt) ? min(a.trk_len[g], kLenBins - 1) : -1;
            if (lb[k] >= 0) atomicAdd(&h[lb[k]], 1);
        }
        __syncthreads();
        for (int b = threadIdx.x; b < kLenBins; b += blockDim.x) {
            base[b] = h[b] ? atomicAdd(&a.lhist[b], h[b]) : 0;
            h[b] = 0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kLenPer; k++)
            if (lb[k] >= 0) a.perm[base[lb[k]] + atomicAdd(&h[lb[k]], 1)] = g0 + k * 256 + threadIdx.x;
        __syncthreads();
    }
}

void launch_len_sort(const KArgs &a, Launch l, hipStream_t s) {
    launch_fill_i32(a.lhist, kLenBins, 0, s);
    hipLaunchKernelGGL(k_len_hist, dim3(l.grid), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_len_scan, dim3(1), dim3(kLenBins), 0, s, a);
    hipLaunchKernelGGL(k_len_scatter, dim3(l.grid), dim3(256), 0, s, a);
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

void launch_scan_i32(const int32_t *in, int32_t n, int32_t *out, int32_t *total_dst, int32_t *tmp, hipStream_t s) {
    scan_impl(I32In{in}, nullptr, n, n, out, total_dst, tmp, s);
}

void launch_scan_i32_dev(const int32_t *in, const int32_t *n_dev, int32_t n_cap, int32_t *out, int32_t *total_dst,
                         int32_t *tmp, hipStream_t s) {
    scan_impl(I32In{in}, n_dev, 0, n_cap, out, total_dst, tmp, s);
}

}  // namespace tpcca
