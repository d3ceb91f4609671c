// Search-grid construction: per sector, clusters are grouped by pad row and
// each row is ordered by fine drift-time bin (kFinePerCb per coarse bin), with
// coarse time bins giving O(1) range lookups. The grid is an acceleration
// structure only: neighbour candidate sets are decided by exact predicates
// later, so the layout cannot change any result.
//
// A row of a 10 ms frame holds tens of thousands of clusters, more than LDS
// holds, so the histogram and the scatter already split every row into
// buckets by time slab (floor(t / kSlabW), clamped; 4096 cm, a few thousand
// clusters of a 10 ms frame row); the row sort then orders one bucket at a
// time, its records in registers and its writes confined to the bucket's
// range. The coarse bins are aligned so that each lies in one slab: their
// width is a power of two (at most the slab width) and their origin a
// multiple of it, which also makes every bin and slab index exact.
//
// Kernels (persistent, grid-stride over device-side work counts):
//   k_si_init    reset per-sector state
//   k_hist       per-chunk LDS histogram of the (row, slab) buckets + time
//                range, validation
//   k_si_rows    per sector: bin geometry
//   k_si_prefix  sorted-space base of every sector
//   k_si_buckets per sector: bucket starts (row-major, slab-minor)
//   k_scatter    scatter of clusters into their buckets (staged in LDS)
//   k_rowsort    per bucket: counting sort by fine time bin; writes the
//                coarse-bin offsets (and fine-bin starts) of its bins
#include "tpcca_internal.h"

namespace tpcca {

__device__ inline bool valid_cluster(int r, float y, float t, int n_rows) {
    return r < n_rows && __builtin_isfinite(y) && __builtin_isfinite(t);
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t n4 = n >> 2;
    int4 v4 = make_int4(v, v, v, v);
    int4 *p4 = reinterpret_cast<int4 *>(p);
    for (int64_t k = i; k < n4; k += stride) p4[k] = v4;
    for (int64_t k = (n4 << 2) + i; k < n; k += stride) p[k] = v;
}

// Plain streaming copy (16-byte vectors), the reference for traffic counters.
__global__ __launch_bounds__(256) void k_copy(const int4 *__restrict__ src, int4 *__restrict__ dst, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

void launch_copy(const void *src, void *dst, int64_t n16, int grid, hipStream_t s) {
    if (n16 <= 0) return;
    hipLaunchKernelGGL(k_copy, dim3(max(grid, 1)), dim3(256), 0, s, (const int4 *)src, (int4 *)dst, n16);
}

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return;
    int64_t blocks = ((n >> 2) + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
}

__global__ void k_si_init(KArgs a) {
    for (int si = blockIdx.x * blockDim.x + threadIdx.x; si < a.n_si; si += gridDim.x * blockDim.x) {
        SiState z = {};
        z.tmin_key = 0xffffffffu;
        z.tmax_key = 0u;
        a.st[si] = z;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Counters c = {};
        *a.cnt = c;
    }
}

// Every workgroup takes a contiguous range of chunks (consecutive chunks
// mostly belong to one sector) and keeps its LDS counts and time range until
// the sector changes, so the flush to global memory happens about once per
// (workgroup, sector); each thread loads kHistPer inputs before it counts
// them.
constexpr int kHistPer = 4;

__global__ __launch_bounds__(256) void k_hist(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    __shared__ int32_t h[kMaxRows * kNSlabMax];
    __shared__ uint32_t smin, smax;
    __shared__ int32_t sinv;
    const int R = a.n_rows, nbk = R * kNSlabMax, bd = blockDim.x;
    const int per = (a.n_chunks + gridDim.x - 1) / gridDim.x;
    const int c0 = blockIdx.x * per, c1 = min(c0 + per, a.n_chunks);
    for (int k = threadIdx.x; k < nbk; k += bd) h[k] = 0;
    if (threadIdx.x == 0) {
        smin = 0xffffffffu;
        smax = 0u;
        sinv = 0;
    }
    __syncthreads();
    uint32_t lmin = 0xffffffffu, lmax = 0u;
    int linv = 0;
    for (int c = c0; c < c1; c++) {
        const int si = a.chunk[2 * c], start = a.chunk[2 * c + 1];
        const SiDesc d = a.si[si];
        const int end = min(start + kChunk, d.n);
        for (int i0 = start + threadIdx.x; i0 < end; i0 += bd * kHistPer) {
            int rr[kHistPer];
            float yy[kHistPer], tt[kHistPer];
#pragma unroll
            for (int u = 0; u < kHistPer; u++) {
                const int i = i0 + u * bd;
                rr[u] = -1;
                yy[u] = tt[u] = 0.f;
                if (i < end) {
                    rr[u] = d.row[i];
                    yy[u] = d.y[i];
                    tt[u] = d.t[i];
                }
            }
#pragma unroll
            for (int u = 0; u < kHistPer; u++) {
                if (rr[u] < 0) continue;
                if (valid_cluster(rr[u], yy[u], tt[u], R)) {
                    atomicAdd(&h[rr[u] * kNSlabMax + slab_of_t(tt[u])], 1);
                    const uint32_t k = fkey(tt[u]);
                    lmin = min(lmin, k);
                    lmax = max(lmax, k);
                } else {
                    linv++;
                }
            }
        }
        // flush when the next chunk of this workgroup is another sector's
        const bool flush = c + 1 == c1 || a.chunk[2 * (c + 1)] != si;   // uniform
        if (!flush) continue;
        for (int off = 32; off > 0; off >>= 1) {
            lmin = min(lmin, (uint32_t)__shfl_xor((int)lmin, off));
            lmax = max(lmax, (uint32_t)__shfl_xor((int)lmax, off));
            linv += __shfl_xor(linv, off);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicMin(&smin, lmin);
            atomicMax(&smax, lmax);
            if (linv) atomicAdd(&sinv, linv);
        }
        lmin = 0xffffffffu;
        lmax = 0u;
        linv = 0;
        __syncthreads();
        int32_t *g = a.bcnt + (int64_t)si * nbk;
        for (int k = threadIdx.x; k < nbk; k += bd) {
            if (h[k]) atomicAdd(&g[k], h[k]);
            h[k] = 0;
        }
        if (threadIdx.x == 0) {
            if (smax >= smin) {
                atomicMin(&a.st[si].tmin_key, smin);
                atomicMax(&a.st[si].tmax_key, smax);
            }
            if (sinv) atomicAdd(&a.cnt->n_invalid, sinv);
            smin = 0xffffffffu;
            smax = 0u;
            sinv = 0;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_si_rows(KArgs a) {
    __shared__ int32_t sc[256];
    const int R = a.n_rows;
    const int r = threadIdx.x;
    for (int si = blockIdx.x; si < a.n_si; si += gridDim.x) {
        int v = 0;
        if (r < R) {
            const int32_t *c = a.bcnt + ((int64_t)si * R + r) * kNSlabMax;
#pragma unroll
            for (int k = 0; k < kNSlabMax; k++) v += c[k];
        }
        sc[r] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int x = (r >= off) ? sc[r - off] : 0;
            __syncthreads();
            sc[r] += x;
            __syncthreads();
        }
        if (r == 0) {
            SiState s = a.st[si];
            const int nv = sc[255];
            float tmin = 0.f, tmax = 0.f;
            if (nv > 0) {
                tmin = fkey_inv(s.tmin_key);
                tmax = fkey_inv(s.tmax_key);
            }
            // coarse bins: a power-of-two width, at least cbw_min and wide
            // enough for kNcbMax - 4 bins to cover the range, from an origin
            // that is a multiple of the width (exact bin indices, each bin
            // inside one time slab)
            const float range = __fsub_rn(tmax, tmin);
            float cbw = 0.f, t0 = tmin;
            int ncb = 1;
            if (__builtin_isfinite(range)) {
                float raw = fmaxf(a.cbw_min, range / (float)(kNcbMax - 4));
                // bins wider than a slab: every row is one bucket, so a row
                // may have no more bins than a bucket's histogram holds
                if (raw > kSlabW) raw = fmaxf(raw, range / (float)(kSortBins / kFinePerCb - 4));
                int e;
                const float m = frexpf(raw, &e);   // raw = m * 2^e, m in [0.5, 1)
                cbw = m == 0.5f ? raw : ldexpf(1.0f, e);
                t0 = __fmul_rn(floorf(tmin / cbw), cbw);
                ncb = (int)floorf((tmax - t0) / cbw) + 1;
                ncb = min(max(ncb, 1), kNcbMax);
            }
            s.t0 = t0;
            s.inv_cbw = cbw > 0.f ? 1.0f / cbw : 0.f;
            s.ncb = ncb;
            s.n_valid = nv;
            s.cps = (cbw > 0.f && cbw <= kSlabW) ? (int)(kSlabW / cbw) : 0;
            a.st[si] = s;
        }
        __syncthreads();
    }
}

// exclusive block scan of two ints over blockDim (<= 1024) threads
__device__ inline void block_scan2(int &v0, int &v1, int &tot0, int &tot1, int *sh0, int *sh1) {
    const int tid = threadIdx.x, n = blockDim.x;
    sh0[tid] = v0;
    sh1[tid] = v1;
    __syncthreads();
    for (int off = 1; off < n; off <<= 1) {
        const int x0 = (tid >= off) ? sh0[tid - off] : 0;
        const int x1 = (tid >= off) ? sh1[tid - off] : 0;
        __syncthreads();
        sh0[tid] += x0;
        sh1[tid] += x1;
        __syncthreads();
    }
    tot0 = sh0[n - 1];
    tot1 = sh1[n - 1];
    v0 = sh0[tid] - v0;
    v1 = sh1[tid] - v1;
    __syncthreads();
}

__global__ __launch_bounds__(1024) void k_si_prefix(KArgs a) {
    __shared__ int sh0[1024], sh1[1024];
    int carry_s = 0;
    for (int base = 0; base < a.n_si; base += blockDim.x) {
        const int si = base + threadIdx.x;
        int nv = 0, nz = 0;
        if (si < a.n_si) nv = a.st[si].n_valid;
        int tv, tz;
        block_scan2(nv, nz, tv, tz, sh0, sh1);
        if (si < a.n_si) a.st[si].sbase = carry_s + nv;
        carry_s += tv;
    }
    if (threadIdx.x == 0) a.cnt->n_valid_total = carry_s;
}

void launch_grid_hist(const KArgs &a, Launch l, hipStream_t s) {
    int g = a.n_si < 1 ? 1 : a.n_si;
    hipLaunchKernelGGL(k_si_init, dim3((g + 255) / 256), dim3(256), 0, s, a);
    if (a.n_chunks > 0)
        hipLaunchKernelGGL(k_hist, dim3(min(l.grid, a.n_chunks)), dim3(256), 0, s, a);
}

// Bucket starts of every sector: exclusive prefix over (row, slab) in row
// order, slab order within a row (so a row's buckets are contiguous and in
// time order). 1024 threads, two buckets each.
__global__ __launch_bounds__(1024) void k_si_buckets(KArgs a) {
    __shared__ int32_t wsum[16];
    const int nb = a.n_rows * kNSlabMax;   // <= 2040
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int si = blockIdx.x; si < a.n_si; si += gridDim.x) {
        const int32_t *cnt = a.bcnt + (int64_t)si * nb;
        const int k0 = 2 * tid;
        const int v0 = k0 < nb ? cnt[k0] : 0, v1 = k0 + 1 < nb ? cnt[k0 + 1] : 0;
        const int v = v0 + v1;
        int x = v;
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        if (tid < 64) {
            const int u = tid < 16 ? wsum[tid] : 0;
            int z = u;
            for (int off = 1; off < 16; off <<= 1) {
                const int y = __shfl_up(z, off);
                if (tid >= off) z += y;
            }
            if (tid < 16) wsum[tid] = z - u;
        }
        __syncthreads();
        const int e = wsum[w] + x - v;
        int32_t *bs = a.bstart + (int64_t)si * nb, *bc = a.bcur + (int64_t)si * nb;
        if (k0 < nb) {
            bs[k0] = e;
            bc[k0] = e;
        }
        if (k0 + 1 < nb) {
            bs[k0 + 1] = e + v0;
            bc[k0 + 1] = e + v0;
        }
        __syncthreads();
    }
}

void launch_grid_setup(const KArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_si_rows, dim3(min(a.n_si, 4096)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_si_prefix, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_si_buckets, dim3(min(a.n_si, 4096)), dim3(1024), 0, s, a);
}

// Scatter into the (row, slab) buckets, one chunk of kChunk clusters at a
// time: the chunk's clusters are ranked per bucket in LDS, the workgroup
// takes one range of every bucket's cursor, stages the records grouped by
// bucket in LDS and writes them out in that order, so consecutive lanes write
// consecutive addresses of one bucket's range. Each input is read once.
constexpr int kScatterBlock = 1024;
constexpr int kScatterPer = kChunk / kScatterBlock;
constexpr int kScatterBk = kMaxRows * kNSlabMax;
static_assert(kScatterPer * kScatterBlock == kChunk, "a chunk must split evenly over the workgroup");
static_assert(kScatterBk <= 2 * kScatterBlock, "the bucket scan takes two buckets per thread");

__global__ __launch_bounds__(kScatterBlock) void k_scatter(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    __shared__ Rec stage[kChunk];
    __shared__ int32_t h[kScatterBk + 1], ls[kScatterBk + 1], gb[kScatterBk + 1];
    __shared__ int32_t wsum[kScatterBlock / 64];
    __shared__ int32_t s_nv;
    const int R = a.n_rows, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nbk = R * kNSlabMax;   // <= 2 * kScatterBlock
    // the inputs of the workgroup's next chunk are loaded while the current
    // one is written out
    int rr[kScatterPer];
    float yy[kScatterPer], tt[kScatterPer];
    auto fetch = [&](int c) {
        const int si = a.chunk[2 * c], i0 = a.chunk[2 * c + 1];
        const SiDesc d = a.si[si];
        const int i1 = min(i0 + kChunk, d.n);
#pragma unroll
        for (int k = 0; k < kScatterPer; k++) {
            const int i = i0 + k * kScatterBlock + tid;
            rr[k] = -1;
            yy[k] = tt[k] = 0.f;
            if (i < i1) {
                rr[k] = d.row[i];
                yy[k] = d.y[i];
                tt[k] = d.t[i];
            }
        }
    };
    if (blockIdx.x < a.n_chunks) fetch(blockIdx.x);
    for (int c = blockIdx.x; c < a.n_chunks; c += gridDim.x) {
        const int si = a.chunk[2 * c], i0 = a.chunk[2 * c + 1];
        const SiState S = a.st[si];
        for (int k = tid; k < nbk; k += kScatterBlock) h[k] = 0;
        __syncthreads();
        int bk[kScatterPer], rk[kScatterPer];
#pragma unroll
        for (int k = 0; k < kScatterPer; k++) {
            bk[k] = rr[k] >= 0 && valid_cluster(rr[k], yy[k], tt[k], R) ? rr[k] * kNSlabMax + slab_of_t(tt[k]) : -1;
            rk[k] = bk[k] >= 0 ? atomicAdd(&h[bk[k]], 1) : 0;
        }
        __syncthreads();
        // one global range of every bucket (all reservations in flight at
        // once) and the bucket starts inside the stage (workgroup scan, two
        // buckets per thread)
        {
            int32_t *cur = a.bcur + (int64_t)si * nbk;
            for (int k = tid; k < nbk; k += kScatterBlock) {
                const int v = h[k];
                gb[k] = v ? S.sbase + atomicAdd(&cur[k], v) : 0;
            }
            const int k0 = 2 * tid;
            const int v0 = k0 < nbk ? h[k0] : 0, v1 = k0 + 1 < nbk ? h[k0 + 1] : 0;
            const int v = v0 + v1;
            int x = v;
            for (int off = 1; off < 64; off <<= 1) {
                const int u = __shfl_up(x, off);
                if (lane >= off) x += u;
            }
            if (lane == 63) wsum[w] = x;
            __syncthreads();
            if (tid < 64) {
                const int u = tid < kScatterBlock / 64 ? wsum[tid] : 0;
                int z = u;
                for (int off = 1; off < 64; off <<= 1) {
                    const int q = __shfl_up(z, off);
                    if (tid >= off) z += q;
                }
                if (tid < kScatterBlock / 64) wsum[tid] = z - u;
                if (tid == kScatterBlock / 64 - 1) s_nv = z;
            }
            __syncthreads();
            const int e = wsum[w] + x - v;
            if (k0 < nbk) ls[k0] = e;
            if (k0 + 1 < nbk) ls[k0 + 1] = e + v0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kScatterPer; k++) {
            if (bk[k] >= 0) {
                Rec e;
                e.y = yy[k];
                e.t = tt[k];
                e.id = i0 + k * kScatterBlock + tid;
                e.sr = (si << 8) | (bk[k] / kNSlabMax);
                stage[ls[bk[k]] + rk[k]] = e;
            }
        }
        __syncthreads();
        if (c + gridDim.x < a.n_chunks) fetch(c + gridDim.x);
        const int nv = s_nv;
        for (int j = tid; j < nv; j += kScatterBlock) {
            const Rec e = stage[j];
            const int b = (e.sr & 255) * kNSlabMax + slab_of_t(e.t);
            a.tmp[gb[b] + (j - ls[b])] = e;
        }
        __syncthreads();
    }
}

void launch_grid_scatter(const KArgs &a, Launch l, hipStream_t s) {
    if (a.n_chunks > 0) hipLaunchKernelGGL(k_scatter, dim3(min(l.grid, a.n_chunks)), dim3(kScatterBlock), 0, s, a);
}

constexpr int kSortBlock = 1024;
constexpr int kSortPer = kSortCap / kSortBlock;
static_assert(kSortPer * kSortBlock == kSortCap, "the register sort holds kSortPer records per thread");
static_assert(kSortCap <= 8192 && kNcbMax * kFinePerCb <= (1 << 18), "bin and rank share one int (18 + 13 bits)");

// Exclusive scan of fh[0, nb) in place: each thread sums a contiguous run of
// bins, then wave and workgroup prefixes of the runs.
__device__ inline void lds_scan_excl(int32_t *fh, int nb, int32_t *wsum) {
    const int tid = threadIdx.x, bd = blockDim.x, lane = tid & 63, w = tid >> 6, nw = bd >> 6;
    const int per = (nb + bd - 1) / bd;
    const int lo = min(tid * per, nb), hi = min(lo + per, nb);
    int sum = 0;
    for (int b = lo; b < hi; b++) sum += fh[b];
    int x = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (tid < 64) {
        const int u = tid < nw ? wsum[tid] : 0;
        int z = u;
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(z, off);
            if (tid >= off) z += y;
        }
        if (tid < nw) wsum[tid] = z - u;
    }
    __syncthreads();
    int run = wsum[w] + x - sum;
    for (int b = lo; b < hi; b++) {
        const int v = fh[b];
        fh[b] = run;
        run += v;
    }
    __syncthreads();
}

// One (row, slab) bucket at a time. A bucket of at most sort_cap clusters
// is read once into registers; one LDS atomic per cluster gives both the
// fine-bin histogram and the cluster's rank inside its bin, and after the
// scan every record is written straight to its place (the writes stay in the
// bucket's range, so partial lines merge in the cache). A larger bucket
// takes two passes over global memory. Order inside a fine bin is arbitrary:
// the neighbour tiles order each bin by y cell in LDS. The coarse bins of the
// bucket get their offsets (and, when asked, the starts of their fine bins
// 1..kFinePerCb-1, one byte each, 255: beyond a byte); the row's last bucket
// also writes the row's end.
__global__ __launch_bounds__(kSortBlock) void k_rowsort(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    __shared__ int32_t fh[kSortBins];
    __shared__ int32_t wsum[kSortBlock / 64];
    const int R = a.n_rows;
    const int nbk = a.n_si * R * kNSlabMax;
    const int tid = threadIdx.x, bd = blockDim.x;
    for (int bk = blockIdx.x; bk < nbk; bk += gridDim.x) {
        const int seg = bk / kNSlabMax, slab = bk - seg * kNSlabMax;
        const int si = seg / R;
        const SiState S = a.st[si];
        const int ncb = S.ncb, cps = S.cps;
        int cb0 = 0, cb1 = ncb, n = 0;
        if (cps > 0) {
            // slab s holds the coarse bins of [s, s + 1) * kSlabW (the first
            // and the last slab also what the clamp puts there)
            const int k0 = (int)__fmul_rn(S.t0, S.inv_cbw);   // the origin in bins (exact)
            if (slab > 0) cb0 = min(max(slab * cps - k0, 0), ncb);
            if (slab < kNSlabMax - 1) cb1 = min(max((slab + 1) * cps - k0, 0), ncb);
            n = a.bcnt[bk];
        } else {
            // coarse bins wider than a slab: slab 0 sorts the whole row (its
            // buckets are contiguous)
            if (slab != 0) continue;
            for (int k = 0; k < kNSlabMax; k++) n += a.bcnt[bk + k];
        }
        const bool last = cps == 0 || slab == kNSlabMax - 1;   // writes the row's end
        const int f0 = cb0 * kFinePerCb, nb = (cb1 - cb0) * kFinePerCb, nf = ncb * kFinePerCb;
        const int start = S.sbase + a.bstart[bk];
        int32_t *co = a.coff + (int64_t)seg * (kNcbMax + 1);
        uint32_t *fo = a.foff ? a.foff + (int64_t)seg * kNcbMax : nullptr;
        if (n == 0) {
            for (int cb = cb0 + tid; cb < cb1; cb += bd) {
                co[cb] = start;
                if (fo) fo[cb] = 0u;
            }
            if (last && tid == 0) co[ncb] = start;
            continue;
        }
        for (int b = tid; b < nb; b += bd) fh[b] = 0;
        __syncthreads();
        const bool fast = n <= a.sort_cap;   // uniform
        Rec e[kSortPer];
        int lr[kSortPer];   // local fine bin << 13 | rank inside the bin (-1: none)
        if (fast) {
#pragma unroll
            for (int j = 0; j < kSortPer; j++) {
                const int k = tid + j * bd;
                if (k < n) e[j] = a.tmp[start + k];
            }
#pragma unroll
            for (int j = 0; j < kSortPer; j++) {
                lr[j] = -1;
                if (tid + j * bd < n) {
                    const int l = min(max(fine_bin(e[j].t, S.t0, S.inv_cbw, nf) - f0, 0), nb - 1);
                    lr[j] = (l << 13) | atomicAdd(&fh[l], 1);
                }
            }
        } else {
            for (int k = tid; k < n; k += bd)
                atomicAdd(&fh[min(max(fine_bin(a.tmp[start + k].t, S.t0, S.inv_cbw, nf) - f0, 0), nb - 1)], 1);
        }
        __syncthreads();
        lds_scan_excl(fh, nb, wsum);
        for (int cb = cb0 + tid; cb < cb1; cb += bd) {
            const int b0 = fh[(cb - cb0) * kFinePerCb];
            co[cb] = start + b0;
            if (fo) {
                uint32_t packed = 0u;
#pragma unroll
                for (int k = 1; k < kFinePerCb; k++)
                    packed |= (uint32_t)min(fh[(cb - cb0) * kFinePerCb + k] - b0, 255) << (8 * (k - 1));
                fo[cb] = packed;
            }
        }
        if (last && tid == 0) co[ncb] = start + n;
        if (fast) {
#pragma unroll
            for (int j = 0; j < kSortPer; j++)
                if (lr[j] >= 0) a.rec[start + fh[lr[j] >> 13] + (lr[j] & 8191)] = e[j];
        } else {
            __syncthreads();   // the offsets above have read fh; it now becomes the cursors
            for (int k = tid; k < n; k += bd) {
                const Rec r = a.tmp[start + k];
                const int l = min(max(fine_bin(r.t, S.t0, S.inv_cbw, nf) - f0, 0), nb - 1);
                a.rec[start + atomicAdd(&fh[l], 1)] = r;
            }
        }
        __syncthreads();
    }
}

void launch_grid_rowsort(const KArgs &a, Launch l, hipStream_t s) {
    const int nbk = a.n_si * a.n_rows * kNSlabMax;
    if (nbk > 0)
        hipLaunchKernelGGL(k_rowsort, dim3(min(l.grid, nbk)), dim3(kSortBlock), 0, s, a);
}

}  // namespace tpcca
