// Neighbour finding: one lane per cluster, one workgroup per strip (a sector
// and a slab of coarse time bins), sweeping the pad rows of the strip in
// order. The rows r-2..r+2 (plus one coarse bin of time halo on each side)
// live in a five-slot LDS ring: each step stages the one new row r+2, builds
// a small time index over it, and then every lane scores the candidates of
// one cluster of row r:
//
//   ry = (y_i - y_d) - w*(y_u - y_d),  rt = (t_i - t_d) - w*(t_u - t_d),
//   c  = ry*ry + rt*rt,                accepted if c <= pair_c2,
//
// over down clusters d on row r-g and up clusters u on row r+g inside the
// box |y - y_i| <= g*win_y, |t - t_i| <= g*win_t, for g = 1, then g = 2 only
// if g = 1 found nothing. w = (x_r - x_{r-g}) / (x_{r+g} - x_{r-g}) comes
// precomputed in FP32 from the host. Every operation is one separately
// rounded FP32 op (no contraction), so the decisions are bit-identical to
// any IEEE implementation of the same sequence. The winner is the
// lexicographic minimum of (c, up input index, down input index). Time is the
// seeding coordinate; no z or vertex is involved.
//
// Strips come from a device-side work queue, so uneven sectors and frames
// balance across the persistent workgroups. A row whose staged range does not
// fit its LDS slot is read from global memory (L2) instead, with the same
// predicates.
#include "tpcca_internal.h"

namespace tpcca {

constexpr int kSweepBlock = 256;
constexpr int kSlots = 2 * kMaxGap + 1;
constexpr int kSlotCap = 768;
constexpr int kIdxPerCb = 8;                                  // index bins per coarse bin
constexpr int kIdxMax = (kMaxStripCb + 2) * kIdxPerCb + 1;

struct LdsSlot {
    const float *y, *t;
    const int32_t *id;
    const int32_t *first;  // index bin -> first position with bin >= it
    int32_t pos0, n, nb;
    float T0, sidx;        // index bin = floor((t - T0) * sidx)
    __device__ float Y(int k) const { return y[k]; }
    __device__ float T(int k) const { return t[k]; }
    __device__ int32_t I(int k) const { return id[k]; }
    // a position at or before the first element with time >= tl
    __device__ int start(float tl) const {
        int b = (int)floorf(__fmul_rn(__fsub_rn(tl, T0), sidx)) - 1;
        b = min(max(b, 0), nb);
        return first[b];
    }
};

struct GlbSlot {
    const Rec *r;
    const int32_t *co;     // coarse offsets of the row
    int32_t pos0, n, cb_lo;
    float t0, inv_cbw;
    __device__ float Y(int k) const { return r[pos0 + k].y; }
    __device__ float T(int k) const { return r[pos0 + k].t; }
    __device__ int32_t I(int k) const { return r[pos0 + k].id; }
    __device__ int start(float tl) const {
        // every time >= tl - 1 coarse bin lies at or after this coarse bin
        int cb = (int)floorf(__fmul_rn(__fsub_rn(tl, t0), inv_cbw)) - 1;
        cb = max(cb, cb_lo);
        const int p = co[cb] - pos0;
        return min(max(p, 0), n);
    }
};

template <class VD, class VU>
__device__ inline bool best_pair(const VD &D, const VU &U, float yi, float ti, float w, float wy, float wt,
                                 float c2, int &bu, int &bd) {
    const float tl = __fsub_rn(ti, wt);
    const int sd = D.start(tl), su = U.start(tl);
    bool found = false;
    float bc = 0.f;
    int biu = 0, bid = 0;
    for (int kd = sd; kd < D.n; kd++) {
        const float td = D.T(kd);
        if (__fsub_rn(td, ti) > wt) break;
        const float yd = D.Y(kd);
        if (!(fabsf(__fsub_rn(yi, yd)) <= wy && fabsf(__fsub_rn(ti, td)) <= wt)) continue;
        const float ady = __fsub_rn(yi, yd);
        const float adt = __fsub_rn(ti, td);
        int idd = -1;
        for (int ku = su; ku < U.n; ku++) {
            const float tu = U.T(ku);
            if (__fsub_rn(tu, ti) > wt) break;
            const float yu = U.Y(ku);
            if (!(fabsf(__fsub_rn(yu, yi)) <= wy && fabsf(__fsub_rn(tu, ti)) <= wt)) continue;
            const float by = __fsub_rn(yu, yd);
            const float bt = __fsub_rn(tu, td);
            const float ry = __fsub_rn(ady, __fmul_rn(w, by));
            const float rt = __fsub_rn(adt, __fmul_rn(w, bt));
            const float c = __fadd_rn(__fmul_rn(ry, ry), __fmul_rn(rt, rt));
            if (!(c <= c2)) continue;
            if (idd < 0) idd = D.I(kd);
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

// Number of clusters inside the box on each of the two rows.
template <class VD, class VU>
__device__ inline int box_count(const VD &D, const VU &U, float yi, float ti, float wy, float wt) {
    const float tl = __fsub_rn(ti, wt);
    int n = 0;
    for (int k = D.start(tl); k < D.n; k++) {
        const float td = D.T(k);
        if (__fsub_rn(td, ti) > wt) break;
        n += (fabsf(__fsub_rn(yi, D.Y(k))) <= wy && fabsf(__fsub_rn(ti, td)) <= wt);
    }
    for (int k = U.start(tl); k < U.n; k++) {
        const float tu = U.T(k);
        if (__fsub_rn(tu, ti) > wt) break;
        n += (fabsf(__fsub_rn(U.Y(k), yi)) <= wy && fabsf(__fsub_rn(tu, ti)) <= wt);
    }
    return n;
}

__device__ inline uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// The 12 triplet features, every FP32 operation separately rounded in a
// fixed order (division and square root correctly rounded), then BF16.
__device__ inline void triplet_features(float yd, float td, float xd, float yi, float ti, float xi, float yu, float tu,
                                        float xu, int g, float wy, float wt, float w, float c2s, int ncand,
                                        uint16_t *f) {
    const float dyu = __fsub_rn(yu, yi), dtu = __fsub_rn(tu, ti);
    const float dyd = __fsub_rn(yi, yd), dtd = __fsub_rn(ti, td);
    const float by = __fsub_rn(yu, yd), bt = __fsub_rn(tu, td);
    const float ry = __fsub_rn(dyd, __fmul_rn(w, by));
    const float rt = __fsub_rn(dtd, __fmul_rn(w, bt));
    const float ax = __fsub_rn(xi, xd), cx = __fsub_rn(xu, xd), ux = __fsub_rn(xu, xi);
    const float cr = __fsub_rn(__fmul_rn(ax, by), __fmul_rn(dyd, cx));
    const float dab = __fsqrt_rn(__fadd_rn(__fmul_rn(ax, ax), __fmul_rn(dyd, dyd)));
    const float dac = __fsqrt_rn(__fadd_rn(__fmul_rn(cx, cx), __fmul_rn(by, by)));
    const float dbc = __fsqrt_rn(__fadd_rn(__fmul_rn(ux, ux), __fmul_rn(dyu, dyu)));
    const float den = __fmul_rn(__fmul_rn(dab, dac), dbc);
    const float kap = __fdiv_rn(__fmul_rn(2.0f, cr), den);
    f[0] = bf16_rne(__fdiv_rn(dyu, wy));
    f[1] = bf16_rne(__fdiv_rn(dtu, wt));
    f[2] = bf16_rne(__fdiv_rn(dyd, wy));
    f[3] = bf16_rne(__fdiv_rn(dtd, wt));
    f[4] = bf16_rne((float)g);
    f[5] = bf16_rne(__fdiv_rn(xi, 245.0f));
    f[6] = bf16_rne(__fdiv_rn(ry, c2s));
    f[7] = bf16_rne(__fdiv_rn(rt, c2s));
    f[8] = bf16_rne(__fdiv_rn(kap, 0.015f));
    f[9] = bf16_rne(__fdiv_rn(by, cx));
    f[10] = bf16_rne(__fdiv_rn(bt, cx));
    f[11] = bf16_rne(__fdiv_rn((float)ncand, 8.0f));
    f[12] = f[13] = f[14] = f[15] = 0;
}

// Visit every accepted pair (c <= c2) of the cluster in the fixed order
// (down clusters in time order, then up clusters in time order); with
// write = false it only counts them.
template <bool write, class VD, class VU>
__device__ inline int visit_pairs(const VD &D, const VU &U, float yi, float ti, float xd, float xi, float xu, int g,
                                  float w, float wy, float wt, float c2, float c2s, int ncand, const KArgs &a,
                                  int slot) {
    const float tl = __fsub_rn(ti, wt);
    const int sd = D.start(tl), su = U.start(tl);
    int n = 0;
    for (int kd = sd; kd < D.n; kd++) {
        const float td = D.T(kd);
        if (__fsub_rn(td, ti) > wt) break;
        const float yd = D.Y(kd);
        if (!(fabsf(__fsub_rn(yi, yd)) <= wy && fabsf(__fsub_rn(ti, td)) <= wt)) continue;
        const float ady = __fsub_rn(yi, yd);
        const float adt = __fsub_rn(ti, td);
        for (int ku = su; ku < U.n; ku++) {
            const float tu = U.T(ku);
            if (__fsub_rn(tu, ti) > wt) break;
            const float yu = U.Y(ku);
            if (!(fabsf(__fsub_rn(yu, yi)) <= wy && fabsf(__fsub_rn(tu, ti)) <= wt)) continue;
            const float by = __fsub_rn(yu, yd);
            const float bt = __fsub_rn(tu, td);
            const float ry = __fsub_rn(ady, __fmul_rn(w, by));
            const float rt = __fsub_rn(adt, __fmul_rn(w, bt));
            const float c = __fadd_rn(__fmul_rn(ry, ry), __fmul_rn(rt, rt));
            if (!(c <= c2)) continue;
            if (write) {
                const int k = slot + n;
                uint16_t f[kMlpInP];
                triplet_features(yd, td, xd, yi, ti, xi, yu, tu, xu, g, wy, wt, w, c2s, ncand, f);
                uint4 *dst = reinterpret_cast<uint4 *>(a.pfeat + (int64_t)k * kMlpInP);
                dst[0] = make_uint4(f[0] | ((uint32_t)f[1] << 16), f[2] | ((uint32_t)f[3] << 16),
                                    f[4] | ((uint32_t)f[5] << 16), f[6] | ((uint32_t)f[7] << 16));
                dst[1] = make_uint4(f[8] | ((uint32_t)f[9] << 16), f[10] | ((uint32_t)f[11] << 16), 0u, 0u);
                a.pd[k] = D.pos0 + kd;
                a.pu[k] = U.pos0 + ku;
                a.pc[k] = c;
            }
            n++;
        }
    }
    return n;
}

template <bool Enum>
__global__ __launch_bounds__(kSweepBlock) void k_links(KArgs a) {
    __shared__ float sy[kSlots][kSlotCap];
    __shared__ float st[kSlots][kSlotCap];
    __shared__ int32_t sid[kSlots][kSlotCap];
    __shared__ int32_t sfirst[kSlots][kIdxMax];
    __shared__ int32_t s_lo[kSlots], s_n[kSlots], s_glb[kSlots];
    __shared__ int32_t s_strip, s_links, s_glbrows;
    __shared__ int32_t s_scan[kSweepBlock];
    __shared__ int32_t s_cpos, s_cend, s_base;
    const int R = a.n_rows;
    const int G = a.max_gap;
    const int tid = threadIdx.x;
    const int n_strips = a.cnt->n_strips;
    int iter = 0;
    for (;; iter++) {
        if (tid == 0) {
            int v = atomicAdd(&a.cnt->strip_next, 1);
            if ((iter & 7) == 0 && abort_requested(a)) v = n_strips;
            s_strip = v;
            s_links = 0;
            s_glbrows = 0;
            if (iter == 0) {
                s_cpos = 0;
                s_cend = 0;
            }
        }
        __syncthreads();
        const int strip = s_strip;
        if (strip >= n_strips) break;
        // strip -> sector instance
        int lo = 0, hi = a.n_si - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.st[mid].strip_base <= strip) lo = mid;
            else hi = mid - 1;
        }
        const int si = lo;
        const SiState S = a.st[si];
        const int slab = strip - S.strip_base;
        const int cb0 = slab * S.tcb;
        const int cb1 = min(cb0 + S.tcb, S.ncb);
        const int cb_lo = max(cb0 - 1, 0);
        const int cb_hi = min(cb1 + 1, S.ncb);
        const float cbw = 1.0f / S.inv_cbw;
        const float T0 = __fadd_rn(S.t0, __fmul_rn((float)cb_lo, cbw));
        const float sidx = __fmul_rn(S.inv_cbw, (float)kIdxPerCb);
        const int nb = (cb_hi - cb_lo) * kIdxPerCb;
        const int32_t *co_si = a.coff + (int64_t)si * R * (kNcbMax + 1);
        int nl = 0;

        // stage row rr into its ring slot and build the slot's time index
        auto stage = [&](int rr) {
            const int j = rr % kSlots;
            const int32_t *co = co_si + (int64_t)rr * (kNcbMax + 1);
            const int plo = co[cb_lo];
            const int n = co[cb_hi] - plo;
            const bool glb = n > kSlotCap;
            if (!glb) {
                for (int k = tid; k < n; k += kSweepBlock) {
                    const Rec e = a.rec[plo + k];
                    sy[j][k] = e.y;
                    st[j][k] = e.t;
                    sid[j][k] = e.id;
                }
            }
            if (tid == 0) {
                s_lo[j] = plo;
                s_n[j] = n;
                s_glb[j] = glb ? 1 : 0;
                if (glb) s_glbrows++;
            }
            __syncthreads();
            if (!glb) {
                for (int k = tid; k <= n; k += kSweepBlock) {
                    int bk = nb + 1, bp = -1;
                    if (k < n) bk = min(max((int)floorf(__fmul_rn(__fsub_rn(st[j][k], T0), sidx)), 0), nb);
                    if (k > 0) bp = min(max((int)floorf(__fmul_rn(__fsub_rn(st[j][k - 1], T0), sidx)), 0), nb);
                    for (int b = bp + 1; b <= min(bk, nb); b++) sfirst[j][b] = k;
                }
            }
        };

        for (int r = 0; r < min(kMaxGap, R); r++) stage(r);
        for (int r = 0; r < R; r++) {
            if (r + kMaxGap < R) stage(r + kMaxGap);
            __syncthreads();
            // own clusters of row r: coarse bins [cb0, cb1)
            const int32_t *co_r = co_si + (int64_t)r * (kNcbMax + 1);
            const int jr = r % kSlots;
            const int own_lo = co_r[cb0], own_hi = co_r[cb1];
            for (int base = own_lo; base < own_hi; base += kSweepBlock) {
                const int p = base + tid;
                const bool act = p < own_hi;
                float yi = 0.f, ti = 0.f;
                if (act) {
                    const int k = p - s_lo[jr];
                    if (!s_glb[jr]) {
                        yi = sy[jr][k];
                        ti = st[jr][k];
                    } else {
                        const Rec e = a.rec[p];
                        yi = e.y;
                        ti = e.t;
                    }
                }
                int bu = -1, bd = -1;
                int ng[kMaxGap] = {};
                int nc[kMaxGap] = {};
                for (int g = 1; g <= G && act; g++) {
                    if (r - g < 0 || r + g > R - 1) continue;
                    const int jd = (r - g) % kSlots, ju = (r + g) % kSlots;
                    const float w = a.w_tab[r * kMaxGap + g - 1];
                    const float wy = a.win_y[g - 1], wt = a.win_t[g - 1];
                    const bool gd = s_glb[jd] != 0, gu = s_glb[ju] != 0;
                    LdsSlot LD{sy[jd], st[jd], sid[jd], sfirst[jd], s_lo[jd], s_n[jd], nb, T0, sidx};
                    LdsSlot LU{sy[ju], st[ju], sid[ju], sfirst[ju], s_lo[ju], s_n[ju], nb, T0, sidx};
                    GlbSlot GD{a.rec, co_si + (int64_t)(r - g) * (kNcbMax + 1), s_lo[jd], s_n[jd], cb_lo, S.t0,
                               S.inv_cbw};
                    GlbSlot GU{a.rec, co_si + (int64_t)(r + g) * (kNcbMax + 1), s_lo[ju], s_n[ju], cb_lo, S.t0,
                               S.inv_cbw};
                    if (!Enum) {
                        bool f;
                        if (!gd && !gu) f = best_pair(LD, LU, yi, ti, w, wy, wt, a.pair_c2, bu, bd);
                        else if (!gd) f = best_pair(LD, GU, yi, ti, w, wy, wt, a.pair_c2, bu, bd);
                        else if (!gu) f = best_pair(GD, LU, yi, ti, w, wy, wt, a.pair_c2, bu, bd);
                        else f = best_pair(GD, GU, yi, ti, w, wy, wt, a.pair_c2, bu, bd);
                        if (f) break;
                        bu = -1;
                        bd = -1;
                    } else {
                        const float xd = a.row_x[r - g], xi = a.row_x[r], xu = a.row_x[r + g];
                        int ncd, npr;
                        if (!gd && !gu) {
                            ncd = box_count(LD, LU, yi, ti, wy, wt);
                            npr = visit_pairs<false>(LD, LU, yi, ti, xd, xi, xu, g, w, wy, wt, a.pair_c2, a.c2s, ncd, a, 0);
                        } else if (!gd) {
                            ncd = box_count(LD, GU, yi, ti, wy, wt);
                            npr = visit_pairs<false>(LD, GU, yi, ti, xd, xi, xu, g, w, wy, wt, a.pair_c2, a.c2s, ncd, a, 0);
                        } else if (!gu) {
                            ncd = box_count(GD, LU, yi, ti, wy, wt);
                            npr = visit_pairs<false>(GD, LU, yi, ti, xd, xi, xu, g, w, wy, wt, a.pair_c2, a.c2s, ncd, a, 0);
                        } else {
                            ncd = box_count(GD, GU, yi, ti, wy, wt);
                            npr = visit_pairs<false>(GD, GU, yi, ti, xd, xi, xu, g, w, wy, wt, a.pair_c2, a.c2s, ncd, a, 0);
                        }
                        ng[g - 1] = npr;
                        nc[g - 1] = ncd;
                    }
                }
                if (!Enum) {
                    if (act) {
                        a.link[p] = make_int2(bu, bd);
                        nl += (bu >= 0);
                    }
                } else {
                    // reserve this lane's pool slots: block scan, chunked grabs
                    int tot = 0;
#pragma unroll
                    for (int g = 0; g < kMaxGap; g++) tot += ng[g];
                    s_scan[tid] = tot;
                    __syncthreads();
                    for (int off = 1; off < kSweepBlock; off <<= 1) {
                        const int xv = (tid >= off) ? s_scan[tid - off] : 0;
                        __syncthreads();
                        s_scan[tid] += xv;
                        __syncthreads();
                    }
                    const int excl = s_scan[tid] - tot;
                    if (tid == kSweepBlock - 1) {
                        const int total = s_scan[tid];
                        if (s_cpos + total > s_cend) {
                            const int grab = max(total, kPoolChunk);
                            s_cpos = atomicAdd(&a.cnt->pool_next, grab);
                            s_cend = s_cpos + grab;
                        }
                        s_base = s_cpos;
                        s_cpos += total;
                        if (total) atomicAdd(&a.cnt->pool_used, total);
                    }
                    __syncthreads();
                    const int slot0 = s_base + excl;
                    if (act) {
                        const bool fits = slot0 + tot <= a.pool_cap;
                        if (fits) {
                            int sl = slot0;
                            for (int g = 1; g <= G; g++) {
                                if (ng[g - 1] == 0) continue;
                                const int jd = (r - g) % kSlots, ju = (r + g) % kSlots;
                                const float w = a.w_tab[r * kMaxGap + g - 1];
                                const float wy = a.win_y[g - 1], wt = a.win_t[g - 1];
                                const float xd = a.row_x[r - g], xi = a.row_x[r], xu = a.row_x[r + g];
                                const bool gd = s_glb[jd] != 0, gu = s_glb[ju] != 0;
                                LdsSlot LD{sy[jd], st[jd], sid[jd], sfirst[jd], s_lo[jd], s_n[jd], nb, T0, sidx};
                                LdsSlot LU{sy[ju], st[ju], sid[ju], sfirst[ju], s_lo[ju], s_n[ju], nb, T0, sidx};
                                GlbSlot GD{a.rec, co_si + (int64_t)(r - g) * (kNcbMax + 1), s_lo[jd], s_n[jd], cb_lo,
                                           S.t0, S.inv_cbw};
                                GlbSlot GU{a.rec, co_si + (int64_t)(r + g) * (kNcbMax + 1), s_lo[ju], s_n[ju], cb_lo,
                                           S.t0, S.inv_cbw};
                                const int ncd = nc[g - 1];
                                if (!gd && !gu) visit_pairs<true>(LD, LU, yi, ti, xd, xi, xu, g, w, wy, wt, a.pair_c2, a.c2s, ncd, a, sl);
                                else if (!gd) visit_pairs<true>(LD, GU, yi, ti, xd, xi, xu, g, w, wy, wt, a.pair_c2, a.c2s, ncd, a, sl);
                                else if (!gu) visit_pairs<true>(GD, LU, yi, ti, xd, xi, xu, g, w, wy, wt, a.pair_c2, a.c2s, ncd, a, sl);
                                else visit_pairs<true>(GD, GU, yi, ti, xd, xi, xu, g, w, wy, wt, a.pair_c2, a.c2s, ncd, a, sl);
                                sl += ng[g - 1];
                            }
                            a.hoff[p] = slot0;
                        } else {
                            a.hoff[p] = -1;
                            atomicAdd(&a.cnt->pool_overflow, tot);
                        }
                        a.hn1[p] = ng[0];
                        a.hn2[p] = kMaxGap > 1 ? ng[1] : 0;
                    }
                }
            }
            __syncthreads();
        }
        for (int off = 32; off > 0; off >>= 1) nl += __shfl_xor(nl, off);
        if ((tid & 63) == 0 && nl) atomicAdd(&s_links, nl);
        __syncthreads();
        if (tid == 0) {
            if (s_links) atomicAdd(&a.cnt->n_links, s_links);
            if (s_glbrows) atomicAdd(&a.cnt->n_glb_rows, s_glbrows);
        }
    }
}

void launch_links(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL(k_links<false>, dim3(max(l.grid, 1)), dim3(kSweepBlock), 0, s, a);
}

void launch_links_enum(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL(k_links<true>, dim3(max(l.grid, 1)), dim3(kSweepBlock), 0, s, a);
}

// Pruned links: per cluster, the best pair among its triplets whose logit
// is >= theta, gap 1 first, gap 2 only if no gap-1 triplet survives; the
// same (c, up id, down id) order as the plain finder.
__global__ __launch_bounds__(256) void k_select(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    const int n = min(a.cnt->n_valid_total, a.n_in);
    const float th = a.theta;
    int pruned = 0, nl = 0;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const int off = a.hoff[p];
        int bu = -1, bd = -1;
        if (off >= 0) {
            const int n1 = a.hn1[p], n2 = a.hn2[p];
            for (int g = 0; g < 2 && bu < 0; g++) {
                const int k0 = off + (g ? n1 : 0), k1 = k0 + (g ? n2 : n1);
                bool found = false;
                float bc = 0.f;
                int biu = 0, bid = 0;
                for (int k = k0; k < k1; k++) {
                    if (!(a.pz[k] >= th)) {
                        pruned++;
                        continue;
                    }
                    const float c = a.pc[k];
                    const int pu = a.pu[k], pd = a.pd[k];
                    const int idu = a.rec[pu].id, idd = a.rec[pd].id;
                    if (!found || c < bc || (c == bc && (idu < biu || (idu == biu && idd < bid)))) {
                        found = true;
                        bc = c;
                        biu = idu;
                        bid = idd;
                        bu = pu;
                        bd = pd;
                    }
                }
            }
        }
        a.link[p] = make_int2(bu, bd);
        nl += (bu >= 0);
    }
    for (int off = 32; off > 0; off >>= 1) {
        pruned += __shfl_xor(pruned, off);
        nl += __shfl_xor(nl, off);
    }
    if ((threadIdx.x & 63) == 0) {
        if (pruned) atomicAdd(&a.cnt->n_pruned, pruned);
        if (nl) atomicAdd(&a.cnt->n_links, nl);
    }
}

void launch_select(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL(k_select, dim3(max(l.grid, 1)), dim3(256), 0, s, a);
}

}  // namespace tpcca
