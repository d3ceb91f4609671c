// Search-grid construction: per sector, clusters are grouped by pad row and
// each row is ordered by fine drift-time bin (2 per coarse bin), with coarse
// time bins giving O(1) range lookups. The grid is an acceleration structure
// only: neighbour candidate sets are decided by exact predicates later, so
// the layout cannot change any result.
//
// Kernels (persistent, grid-stride over device-side work counts):
//   k_si_init   reset per-sector state
//   k_hist      per-chunk LDS row histogram + time range, validation
//   k_si_rows   per sector: row prefix, bin geometry
//   k_si_prefix sorted-space base of every sector
//   k_scatter   scatter of clusters into row segments (staged by row in LDS)
//   k_rowsort   per (sector,row): counting sort by fine time bin (LDS
//               histogram, scatter); writes the coarse bin offsets used by
//               the neighbour tiles
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

__global__ __launch_bounds__(256) void k_hist(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    __shared__ int32_t h[kMaxRows];
    __shared__ uint32_t smin, smax;
    __shared__ int32_t sinv;
    const int R = a.n_rows;
    for (int c = blockIdx.x; c < a.n_chunks; c += gridDim.x) {
        const int si = a.chunk[2 * c], start = a.chunk[2 * c + 1];
        const SiDesc d = a.si[si];
        const int end = min(start + kChunk, d.n);
        for (int r = threadIdx.x; r < R; r += blockDim.x) h[r] = 0;
        if (threadIdx.x == 0) {
            smin = 0xffffffffu;
            smax = 0u;
            sinv = 0;
        }
        __syncthreads();
        uint32_t lmin = 0xffffffffu, lmax = 0u;
        int linv = 0;
        for (int i = start + threadIdx.x; i < end; i += blockDim.x) {
            const int r = d.row[i];
            const float y = d.y[i], t = d.t[i];
            if (valid_cluster(r, y, t, R)) {
                atomicAdd(&h[r], 1);
                const uint32_t k = fkey(t);
                lmin = min(lmin, k);
                lmax = max(lmax, k);
            } else {
                linv++;
            }
        }
        // wave reductions, then one LDS atomic per wave
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
        __syncthreads();
        for (int r = threadIdx.x; r < R; r += blockDim.x)
            if (h[r]) atomicAdd(&a.rcnt[si * R + r], h[r]);
        if (threadIdx.x == 0) {
            if (smax >= smin) {
                atomicMin(&a.st[si].tmin_key, smin);
                atomicMax(&a.st[si].tmax_key, smax);
            }
            if (sinv) atomicAdd(&a.cnt->n_invalid, sinv);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_si_rows(KArgs a) {
    __shared__ int32_t sc[256];
    const int R = a.n_rows;
    const int r = threadIdx.x;
    for (int si = blockIdx.x; si < a.n_si; si += gridDim.x) {
        const int v = (r < R) ? a.rcnt[si * R + r] : 0;
        sc[r] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int x = (r >= off) ? sc[r - off] : 0;
            __syncthreads();
            sc[r] += x;
            __syncthreads();
        }
        if (r < R) {
            a.rstart[si * R + r] = sc[r] - v;
            a.rcur[si * R + r] = sc[r] - v;
        }
        if (r == 0) {
            SiState s = a.st[si];
            const int nv = sc[255];
            float tmin = 0.f, tmax = 0.f;
            if (nv > 0) {
                tmin = fkey_inv(s.tmin_key);
                tmax = fkey_inv(s.tmax_key);
            }
            const float range = __fsub_rn(tmax, tmin);
            float inv;
            int ncb;
            if (__builtin_isfinite(range)) {
                const float cbw = fmaxf(a.cbw_min, range / (float)(kNcbMax - 4));
                inv = 1.0f / cbw;
                ncb = (int)__fmul_rn(range, inv) + 1;
                ncb = min(max(ncb, 1), kNcbMax);
            } else {
                inv = 0.f;
                ncb = 1;
            }
            s.t0 = tmin;
            s.inv_cbw = inv;
            s.ncb = ncb;
            s.n_valid = nv;
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

void launch_grid_setup(const KArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_si_rows, dim3(min(a.n_si, 4096)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_si_prefix, dim3(1), dim3(1024), 0, s, a);
}

// Scatter into row segments, one chunk of kChunk clusters at a time: the
// chunk's clusters are ranked per row in LDS, the workgroup takes one range
// of every row's segment cursor, stages the records grouped by row in LDS and
// writes them out in that order, so consecutive lanes write consecutive
// addresses of one row's range. Each input is read once.
constexpr int kScatterBlock = 1024;
constexpr int kScatterPer = kChunk / kScatterBlock;
static_assert(kScatterPer * kScatterBlock == kChunk, "a chunk must split evenly over the workgroup");

__global__ __launch_bounds__(kScatterBlock) void k_scatter(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    __shared__ Rec stage[kChunk];
    __shared__ int32_t h[kMaxRows + 1], ls[kMaxRows + 1], gb[kMaxRows + 1];
    __shared__ int32_t s_nv;
    const int R = a.n_rows, tid = threadIdx.x;
    for (int c = blockIdx.x; c < a.n_chunks; c += gridDim.x) {
        const int si = a.chunk[2 * c], i0 = a.chunk[2 * c + 1];
        const SiDesc d = a.si[si];
        const int sbase = a.st[si].sbase;
        const int i1 = min(i0 + kChunk, d.n);
        for (int r = tid; r < R; r += kScatterBlock) h[r] = 0;
        __syncthreads();
        int rr[kScatterPer], rk[kScatterPer];
        float yy[kScatterPer], tt[kScatterPer];
#pragma unroll
        for (int k = 0; k < kScatterPer; k++) {
            const int i = i0 + k * kScatterBlock + tid;
            rr[k] = -1;
            yy[k] = 0.f;
            tt[k] = 0.f;
            if (i < i1) {
                const int r = d.row[i];
                yy[k] = d.y[i];
                tt[k] = d.t[i];
                if (valid_cluster(r, yy[k], tt[k], R)) rr[k] = r;
            }
        }
#pragma unroll
        for (int k = 0; k < kScatterPer; k++) rk[k] = rr[k] >= 0 ? atomicAdd(&h[rr[k]], 1) : 0;
        __syncthreads();
        // row starts inside the stage (one wave scans the rows) and one
        // global range of every row's segment
        if (tid < 64) {
            int carry = 0;
            for (int r0 = 0; r0 < R; r0 += 64) {
                const int r = r0 + tid;
                const int v = r < R ? h[r] : 0;
                int x = v;
                for (int off = 1; off < 64; off <<= 1) {
                    const int u = __shfl_up(x, off);
                    if (tid >= off) x += u;
                }
                if (r < R) {
                    ls[r] = carry + x - v;
                    gb[r] = v ? sbase + atomicAdd(&a.rcur[si * R + r], v) : 0;
                }
                carry += __shfl(x, 63);
            }
            if (tid == 0) s_nv = carry;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kScatterPer; k++) {
            if (rr[k] >= 0) {
                Rec e;
                e.y = yy[k];
                e.t = tt[k];
                e.id = i0 + k * kScatterBlock + tid;
                e.sr = (si << 8) | rr[k];
                stage[ls[rr[k]] + rk[k]] = e;
            }
        }
        __syncthreads();
        const int nv = s_nv;
        for (int j = tid; j < nv; j += kScatterBlock) {
            const Rec e = stage[j];
            const int r = e.sr & 255;
            a.tmp[gb[r] + (j - ls[r])] = e;
        }
        __syncthreads();
    }
}

void launch_grid_scatter(const KArgs &a, Launch l, hipStream_t s) {
    if (a.n_chunks > 0) hipLaunchKernelGGL(k_scatter, dim3(min(l.grid, a.n_chunks)), dim3(kScatterBlock), 0, s, a);
}

constexpr int kFineMax = kNcbMax * kFinePerCb;
constexpr int kSortBlock = 1024;

__global__ __launch_bounds__(kSortBlock) void k_rowsort(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    __shared__ int32_t fh[kFineMax];
    __shared__ int32_t part[kSortBlock];
    const int R = a.n_rows;
    const int nseg = a.n_si * R;
    const int tid = threadIdx.x, bd = blockDim.x;
    for (int seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
        const int si = seg / R;
        const SiState s = a.st[si];
        const int n = a.rcnt[seg];
        const int start = s.sbase + a.rstart[seg];
        const int ncb = s.ncb, nf = ncb * kFinePerCb;
        const float t0 = s.t0, inv = s.inv_cbw;
        int32_t *co = a.coff + (int64_t)seg * (kNcbMax + 1);
        uint32_t *fo = a.foff ? a.foff + (int64_t)seg * kNcbMax : nullptr;
        if (n == 0) {
            for (int cb = tid; cb <= ncb; cb += bd) co[cb] = start;
            if (fo)
                for (int cb = tid; cb < ncb; cb += bd) fo[cb] = 0u;
            continue;
        }
        for (int b = tid; b < nf; b += bd) fh[b] = 0;
        __syncthreads();
        for (int k = tid; k < n; k += bd) atomicAdd(&fh[fine_bin(a.tmp[start + k].t, t0, inv, nf)], 1);
        __syncthreads();
        // exclusive scan of fh[0, nf)
        const int per = (nf + bd - 1) / bd;
        const int lo = min(tid * per, nf), hi = min(lo + per, nf);
        int sum = 0;
        for (int b = lo; b < hi; b++) sum += fh[b];
        part[tid] = sum;
        __syncthreads();
        for (int off = 1; off < bd; off <<= 1) {
            const int x = (tid >= off) ? part[tid - off] : 0;
            __syncthreads();
            part[tid] += x;
            __syncthreads();
        }
        int run = part[tid] - sum;
        for (int b = lo; b < hi; b++) {
            const int v = fh[b];
            fh[b] = run;
            run += v;
        }
        __syncthreads();
        for (int cb = tid; cb <= ncb; cb += bd) co[cb] = start + (cb < ncb ? fh[cb * kFinePerCb] : n);
        if (fo) {
            // the fine-bin starts of each coarse bin (for searches that read
            // the sorted space directly)
            for (int cb = tid; cb < ncb; cb += bd) {
                const int b0 = fh[cb * kFinePerCb];
                uint32_t packed = 0u;
#pragma unroll
                for (int k = 1; k < kFinePerCb; k++)
                    packed |= (uint32_t)min(fh[cb * kFinePerCb + k] - b0, 255) << (8 * (k - 1));
                fo[cb] = packed;
            }
        }
        __syncthreads();
        // counting-sort scatter by fine bin (order inside a bin is arbitrary:
        // the neighbour tiles order each bin by y cell in LDS)
        for (int k = tid; k < n; k += bd) {
            const Rec e = a.tmp[start + k];
            a.rec[start + atomicAdd(&fh[fine_bin(e.t, t0, inv, nf)], 1)] = e;
        }
        __syncthreads();
    }
}

void launch_grid_rowsort(const KArgs &a, Launch l, hipStream_t s) {
    const int nseg = a.n_si * a.n_rows;
    if (nseg > 0)
        hipLaunchKernelGGL(k_rowsort, dim3(min(l.grid, nseg)), dim3(kSortBlock), 0, s, a);
}

}  // namespace tpcca
