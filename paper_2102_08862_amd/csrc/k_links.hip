// Neighbour finding: one lane per cluster, one workgroup per tile (a sector,
// a pad row r and a slab of kTileCb coarse time bins). The rows r-2..r+2 of
// the slab plus one coarse bin of halo on each side are staged in LDS; a
// lane finds, for gap g = 1 then 2, the exact time windows on rows r-g and
// r+g by binary search in the time-ordered rows, and scores every (down, up)
// pair that passes the box cut:
//
//   ry = (y_i - y_d) - w*(y_u - y_d),  rt = (t_i - t_d) - w*(t_u - t_d),
//   c  = ry*ry + rt*rt,                accepted if c <= pair_c2,
//
// with w = (x_r - x_{r-g}) / (x_{r+g} - x_{r-g}) precomputed in FP32 on the
// host. Every operation is a separately rounded FP32 op (no contraction),
// so the decisions are bit-identical to any IEEE implementation of the same
// sequence. The winner is the lexicographic minimum of (c, up input index,
// down input index). Time is the seeding coordinate: no z or vertex is used.
//
// Tiles are visited persistently in an XCD-aware order: the logical tile
// order is (sector, slab, row), and each XCD takes a contiguous range of it,
// so the five rows that share staged data are processed on the same XCD at
// about the same time and the re-reads hit that XCD's L2.
#include "tpcca_internal.h"

namespace tpcca {

struct LdsRows {
    const float *y, *t;
    const int32_t *id;
    int32_t pos0, n;
    __device__ float Y(int k) const { return y[k]; }
    __device__ float T(int k) const { return t[k]; }
    __device__ int32_t I(int k) const { return id[k]; }
};

struct GlbRows {
    const Rec *r;
    int32_t pos0, n;
    __device__ float Y(int k) const { return r[pos0 + k].y; }
    __device__ float T(int k) const { return r[pos0 + k].t; }
    __device__ int32_t I(int k) const { return r[pos0 + k].id; }
};

// first k with !(ti - t_k > wt)
template <class V>
__device__ inline int win_lo(const V &v, float ti, float wt) {
    int lo = 0, hi = v.n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (__fsub_rn(ti, v.T(mid)) > wt) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// first k with t_k - ti > wt
template <class V>
__device__ inline int win_hi(const V &v, float ti, float wt) {
    int lo = 0, hi = v.n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (__fsub_rn(v.T(mid), ti) > wt) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

template <class V>
__device__ inline bool best_pair(const V &D, const V &U, float yi, float ti, float w, float wy, float wt, float c2,
                                 int &bu, int &bd) {
    const int dlo = win_lo(D, ti, wt), dhi = win_hi(D, ti, wt);
    const int ulo = win_lo(U, ti, wt), uhi = win_hi(U, ti, wt);
    bool found = false;
    float bc = 0.f;
    int biu = 0, bid = 0;
    for (int kd = dlo; kd < dhi; kd++) {
        const float yd = D.Y(kd), td = D.T(kd);
        if (!(fabsf(__fsub_rn(yi, yd)) <= wy && fabsf(__fsub_rn(ti, td)) <= wt)) continue;
        const int idd = D.I(kd);
        const float ady = __fsub_rn(yi, yd);
        const float adt = __fsub_rn(ti, td);
        for (int ku = ulo; ku < uhi; ku++) {
            const float yu = U.Y(ku), tu = U.T(ku);
            if (!(fabsf(__fsub_rn(yu, yi)) <= wy && fabsf(__fsub_rn(tu, ti)) <= wt)) continue;
            const float by = __fsub_rn(yu, yd);
            const float bt = __fsub_rn(tu, td);
            const float ry = __fsub_rn(ady, __fmul_rn(w, by));
            const float rt = __fsub_rn(adt, __fmul_rn(w, bt));
            const float c = __fadd_rn(__fmul_rn(ry, ry), __fmul_rn(rt, rt));
            if (!(c <= c2)) continue;
            const int idu = U.I(ku);
            if (!found || c < bc || (c == bc && (idu < biu || (idu == biu && idd < bid)))) {
                found = true;
                bc = c;
                biu = idu;
                bid = idd;
                bu = U.pos0 + ku;
                bd = D.pos0 + kd;
            }
        }
    }
    return found;
}

constexpr int kLinkBlock = 256;

__global__ __launch_bounds__(kLinkBlock) void k_links(KArgs a) {
    __shared__ float sy[2 * kMaxGap][kStageCap];
    __shared__ float st[2 * kMaxGap][kStageCap];
    __shared__ int32_t sid[2 * kMaxGap][kStageCap];
    __shared__ int32_t s_lo[2 * kMaxGap], s_n[2 * kMaxGap];
    __shared__ int32_t s_glb, s_links, s_abort;
    const int R = a.n_rows;
    const int G = a.max_gap;
    const int ntiles = min(a.cnt->n_tiles, 0x7ffffff0);
    const int per = (ntiles + 7) / 8;
    const int nlog = per * 8;
    int iter = 0;
    for (int wv = blockIdx.x; wv < nlog; wv += gridDim.x, iter++) {
        const int L = (wv & 7) * per + (wv >> 3);
        if ((iter & 15) == 0) {
            if (threadIdx.x == 0) s_abort = __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __syncthreads();
            if (s_abort) break;
        }
        if (L >= ntiles) continue;
        // tile -> (sector instance, slab, row)
        int lo = 0, hi = a.n_si - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.st[mid].tile_base <= L) lo = mid;
            else hi = mid - 1;
        }
        const int si = lo;
        const int local = L - a.st[si].tile_base;
        const int slab = local / R;
        const int r = local - slab * R;
        const int ncb = a.st[si].ncb;
        const int cb0 = slab * kTileCb;
        const int cb1 = min(cb0 + kTileCb, ncb);
        const int32_t *co_r = a.coff + (int64_t)(si * R + r) * (kNcbMax + 1);
        const int own_lo = co_r[cb0], own_hi = co_r[cb1];
        if (own_lo >= own_hi) continue;
        if (threadIdx.x == 0) {
            s_glb = 0;
            s_links = 0;
        }
        if (threadIdx.x < 2 * kMaxGap) {
            const int j = threadIdx.x;
            const int g = (j < kMaxGap) ? (kMaxGap - j) : (j - kMaxGap + 1);  // j: r-2, r-1, r+1, r+2
            const int rr = (j < kMaxGap) ? r - g : r + g;
            int plo = 0, pn = 0;
            if (g <= G && rr >= 0 && rr < R) {
                const int32_t *co = a.coff + (int64_t)(si * R + rr) * (kNcbMax + 1);
                plo = co[max(cb0 - 1, 0)];
                pn = co[min(cb1 + 1, ncb)] - plo;
            }
            s_lo[j] = plo;
            s_n[j] = pn;
        }
        __syncthreads();
        for (int j = 0; j < 2 * kMaxGap; j++)
            if (s_n[j] > kStageCap) s_glb = 1;
        __syncthreads();
        const bool glb = s_glb != 0;
        if (!glb) {
            for (int j = 0; j < 2 * kMaxGap; j++) {
                const int n = s_n[j], plo = s_lo[j];
                for (int k = threadIdx.x; k < n; k += blockDim.x) {
                    const Rec e = a.rec[plo + k];
                    sy[j][k] = e.y;
                    st[j][k] = e.t;
                    sid[j][k] = e.id;
                }
            }
        }
        __syncthreads();
        int nl = 0;
        for (int p = own_lo + threadIdx.x; p < own_hi; p += blockDim.x) {
            const Rec me = a.rec[p];
            int bu = -1, bd = -1;
            for (int g = 1; g <= G; g++) {
                if (r - g < 0 || r + g > R - 1) continue;
                const int jd = kMaxGap - g, ju = kMaxGap + g - 1;
                const float w = a.w_tab[r * kMaxGap + g - 1];
                const float wy = a.win_y[g - 1], wt = a.win_t[g - 1];
                bool f;
                if (!glb) {
                    LdsRows D{sy[jd], st[jd], sid[jd], s_lo[jd], s_n[jd]};
                    LdsRows U{sy[ju], st[ju], sid[ju], s_lo[ju], s_n[ju]};
                    f = best_pair(D, U, me.y, me.t, w, wy, wt, a.pair_c2, bu, bd);
                } else {
                    GlbRows D{a.rec, s_lo[jd], s_n[jd]};
                    GlbRows U{a.rec, s_lo[ju], s_n[ju]};
                    f = best_pair(D, U, me.y, me.t, w, wy, wt, a.pair_c2, bu, bd);
                }
                if (f) break;
                bu = -1;
                bd = -1;
            }
            a.link[p] = make_int2(bu, bd);
            nl += (bu >= 0);
        }
        for (int off = 32; off > 0; off >>= 1) nl += __shfl_xor(nl, off);
        if ((threadIdx.x & 63) == 0 && nl) atomicAdd(&s_links, nl);
        __syncthreads();
        if (threadIdx.x == 0 && s_links) atomicAdd(&a.cnt->n_links, s_links);
    }
}

void launch_links(const KArgs &a, Launch l, hipStream_t s) {
    int grid = (l.grid / 8) * 8;
    if (grid < 8) grid = 8;
    hipLaunchKernelGGL(k_links, dim3(grid), dim3(kLinkBlock), 0, s, a);
}

}  // namespace tpcca
