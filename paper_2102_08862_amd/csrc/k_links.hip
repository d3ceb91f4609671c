// Neighbour finding (the pair search of the cellular-automaton seeding, with
// drift time as the seeding coordinate). For every cluster i on pad row r and
// gap g = 1, then g = 2 only if g = 1 found nothing, the candidates are the
// clusters d on row r-g and u on row r+g inside the box |y - y_i| <= g*win_y,
// |t - t_i| <= g*win_t, and a pair is scored
//
//   ry = (y_i - y_d) - w*(y_u - y_d),  rt = (t_i - t_d) - w*(t_u - t_d),
//   c  = ry*ry + rt*rt,                accepted if c <= pair_c2,
//
// with w = (x_r - x_{r-g}) / (x_{r+g} - x_{r-g}) precomputed in FP32 on the
// host. Every operation is one separately rounded FP32 op (no contraction),
// so decisions are bit-identical to any IEEE implementation of the same
// sequence. The link is the lexicographic minimum of (c, up input index,
// down input index) over the accepted pairs, so the order in which pairs are
// visited cannot change it.
//
// Work decomposition: a tile is (sector instance, block of kTileRows pad
// rows, slab of coarse time bins). k_tiles cuts every (sector instance, row
// block) into slabs whose staged clusters (own rows plus kMaxGap rows on each
// side, plus one coarse bin of time on each side) fit the LDS budget; tiles
// come from a device work queue, so uneven sectors and frames balance over
// the persistent workgroups. Within a staged row the clusters are ordered by
// fine time bin (the row sort leaves them so) and, once staged in LDS, each
// fine bin by y cell: a box lookup visits the 1-3 fine bins the box overlaps
// and, in each, binary-searches its first y cell. A tile too dense for LDS (a single coarse bin over budget)
// runs the same search on global memory. Clusters without a g = 1 link go to
// an LDS queue and are searched at g = 2 by the whole workgroup.
#include <type_traits>

#include "mlp_tile.h"

namespace tpcca {

constexpr int kLinkBlock = 256;
constexpr int kSlots = kTileRows + 2 * kMaxGap;          // staged rows of a tile
constexpr int kTileFb = (kMaxTileCb + 2) * kFinePerCb;   // fine bins of a staged row
constexpr int kBatch = 8;                                // down candidates held in registers
constexpr int kQueueCap = 1024;                          // gap-2 queue of a tile (overflow: searched at once)
constexpr int kPrK = 4;                                  // pruned search: pairs per cluster and round

// The three searches: best pair (plain), every triplet to the pool (the
// pool is kept for inspection and training), triplets scored by the
// network inside the search (pruned).
enum LinkMode { kPlain = 0, kEnum = 1, kPrune = 2 };

// ---------------------------------------------------------------- tiles
// One workgroup per (sector instance, row block): cumulative staged counts
// per coarse bin in LDS, then wave 0 cuts greedy slabs, 64 candidate ends at
// a time (the staged count is non-decreasing in the slab end).
__global__ __launch_bounds__(256) void k_tiles(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    __shared__ int32_t cum[kNcbMax + 1];
    const int R = a.n_rows, nrb = a.n_rb;
    const int tid = threadIdx.x, lane = tid & 63;
    for (int w = blockIdx.x; w < a.n_si * nrb; w += gridDim.x) {
        const int si = w / nrb, rb = w - si * nrb;
        const SiState S = a.st[si];
        const int ncb = S.ncb;
        if (S.n_valid == 0) {
            if (tid == 0) a.ntile[w] = 0;
            continue;
        }
        const int r0 = rb * kTileRows, r1 = min(r0 + kTileRows, R);
        const int s0 = max(r0 - kMaxGap, 0), s1 = min(r1 + kMaxGap, R);
        const int32_t *co0 = a.coff + ((int64_t)si * R + s0) * (kNcbMax + 1);
        for (int cb = tid; cb <= ncb; cb += blockDim.x) {
            int sum = 0;
            for (int r = 0; r < s1 - s0; r++) {
                const int32_t *co = co0 + (int64_t)r * (kNcbMax + 1);
                sum += co[cb] - co[0];
            }
            cum[cb] = sum;
        }
        __syncthreads();
        if (tid < 64) {
            int16_t *ts = a.tstart + (int64_t)w * kNcbMax;
            const int budget = a.tile_budget;
            int c0 = 0, n = 0;
            while (c0 < ncb) {
                const int c1 = c0 + 1 + lane;     // candidate slab end (exclusive)
                bool ok = false;
                if (lane < kMaxTileCb && c1 <= ncb)
                    ok = cum[min(c1 + 1, ncb)] - cum[max(c0 - 1, 0)] <= budget;
                const int take = max(1, (int)__popcll(__ballot(ok)));
                if (lane == 0) ts[n] = (int16_t)c0;
                n++;
                c0 += take;
            }
            if (lane == 0) a.ntile[w] = n;
        }
        __syncthreads();
    }
}

// Tile list: tiles[tile_base[w] + k] = (w, cb0 | cb1 << 16).
__global__ __launch_bounds__(256) void k_tile_list(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    const int nrb = a.n_rb;
    for (int w = blockIdx.x; w < a.n_si * nrb; w += gridDim.x) {
        const int n = a.ntile[w], base = a.tile_base[w];
        const int ncb = a.st[w / nrb].ncb;
        const int16_t *ts = a.tstart + (int64_t)w * kNcbMax;
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            if (base + k >= a.tile_cap) break;
            const int c0 = ts[k], c1 = (k + 1 < n) ? ts[k + 1] : ncb;
            a.tiles[base + k] = make_int2(w, c0 | (c1 << 16));
        }
    }
}

void launch_tiles(const KArgs &a, hipStream_t s) {
    const int nw = a.n_si * a.n_rb;
    if (nw <= 0) return;
    hipLaunchKernelGGL(k_tiles, dim3(min(nw, 8192)), dim3(256), 0, s, a);
    launch_scan_i32(a.ntile, nw, a.tile_base, &a.cnt->n_tiles, a.scan_tmp, s);
    hipLaunchKernelGGL(k_tile_list, dim3(min(nw, 8192)), dim3(256), 0, s, a);
}

// ---------------------------------------------------------------- staged rows
// Staged row j of a tile: clusters [plo, plo + n) of the sorted space, its
// fine bins relative to the tile's first staged coarse bin.
struct TileGeo {
    float t0, inv_cbw;
    int nf;        // fine bins of the sector row
    int fb0;       // first staged fine bin
    int nfb;       // staged fine bins
};

// Rows held in LDS.
// Inside each fine bin the staged clusters are ordered by y cell.
struct LdsRows {
    static constexpr bool kYSorted = true;
    const float2 *yt;              // staged (y, t)
    const uint8_t *cell;           // staged y cells
    const int16_t *oq;             // staged cluster -> index in its row segment
    const int32_t *base;           // [kSlots] LDS index of row j's first cluster
    const int32_t *plo;            // [kSlots] first staged sorted position of row j
    const int16_t (*fs)[kTileFb + 1];
    __device__ float2 at(int j, int q) const { return yt[base[j] + q]; }
    __device__ int ycell(int j, int q, const YCell &) const { return cell[base[j] + q]; }
    __device__ int fstart(int j, int f) const { return fs[j][f]; }
    __device__ int pos(int j, int q) const { return plo[j] + oq[base[j] + q]; }
};

// Rows read from global memory (tiles over the LDS budget); the fine-bin
// starts come from a binary search inside the coarse bin.
struct GlbRows {
    static constexpr bool kYSorted = false;   // row order: fine bin only
    const Rec *rec;
    const int32_t *plo;            // [kSlots] (LDS) first staged position of row j
    const int32_t *n;              // [kSlots] (LDS) staged clusters of row j
    const int32_t *co_s0;          // coarse offsets of the first staged row
    TileGeo g;
    __device__ float2 at(int j, int q) const {
        const Rec e = rec[plo[j] + q];
        return make_float2(e.y, e.t);
    }
    __device__ int ycell(int j, int q, const YCell &yc) const { return ycell_of(yc, rec[plo[j] + q].y); }
    __device__ int pos(int j, int q) const { return plo[j] + q; }
    __device__ int fstart(int j, int f) const {
        if (f >= g.nfb) return n[j];
        const int fa = g.fb0 + f;
        const int32_t *co = co_s0 + (int64_t)j * (kNcbMax + 1);
        const int cb = fa / kFinePerCb;
        int lo = co[cb], hi = co[cb + 1];
        while (lo < hi) {
            const int m = (lo + hi) >> 1;
            if (fine_bin(rec[m].t, g.t0, g.inv_cbw, g.nf) < fa) lo = m + 1;
            else hi = m;
        }
        return lo - plo[j];
    }
};

// A bound that every time (or y) passing the box test lies beyond: the exact
// FP32 predicate |fl(a - b)| <= w admits |a - b| slightly above w.
__device__ inline float slack(float v, float w) { return __fadd_rn(__fmul_rn(fabsf(v), 1.0e-6f), __fmul_rn(w, 1.0e-3f)); }

// Visit the clusters of staged row j inside the box around (yi, ti), in row
// order, calling fn(q, y, t) with q the row-local index. The box test is the
// exact predicate: for the down row |yi - y| <= wy && |ti - t| <= wt, for
// the up row |y - yi| <= wy && |t - ti| <= wt.
template <bool Down, class Rows, class Fn>
__device__ inline void box_visit(const Rows &A, const TileGeo &G, const YCell &yc, int j, float yi, float ti, float wy,
                                 float wt, Fn &&fn) {
    const float sy = slack(yi, wy), st = slack(ti, wt);
    const int f0 = fine_bin(__fsub_rn(__fsub_rn(ti, wt), st), G.t0, G.inv_cbw, G.nf) - G.fb0;
    const int f1 = fine_bin(__fadd_rn(__fadd_rn(ti, wt), st), G.t0, G.inv_cbw, G.nf) - G.fb0;
    const int c0 = ycell_of(yc, __fsub_rn(__fsub_rn(yi, wy), sy));
    const int c1 = ycell_of(yc, __fadd_rn(__fadd_rn(yi, wy), sy));
    for (int f = max(f0, 0); f <= min(f1, G.nfb - 1); f++) {
        int lo = A.fstart(j, f);
        const int hi = A.fstart(j, f + 1);
        if (Rows::kYSorted) {
            int h = hi;
            while (lo < h) {
                const int m = (lo + h) >> 1;
                if (A.ycell(j, m, yc) < c0) lo = m + 1;
                else h = m;
            }
        }
        for (int q = lo; q < hi; q++) {
            if (Rows::kYSorted && A.ycell(j, q, yc) > c1) break;
            const float2 e = A.at(j, q);
            const bool in = Down ? (fabsf(__fsub_rn(yi, e.x)) <= wy && fabsf(__fsub_rn(ti, e.y)) <= wt)
                                 : (fabsf(__fsub_rn(e.x, yi)) <= wy && fabsf(__fsub_rn(e.y, ti)) <= wt);
            if (in) fn(q, e.x, e.y);
        }
    }
}

// The pair score c of the middle cluster (yi, ti) between (yd, td) and (yu, tu).
__device__ inline float pair_score(float yi, float ti, float yd, float td, float yu, float tu, float w) {
    const float ady = __fsub_rn(yi, yd);
    const float adt = __fsub_rn(ti, td);
    const float by = __fsub_rn(yu, yd);
    const float bt = __fsub_rn(tu, td);
    const float ry = __fsub_rn(ady, __fmul_rn(w, by));
    const float rt = __fsub_rn(adt, __fmul_rn(w, bt));
    return __fadd_rn(__fmul_rn(ry, ry), __fmul_rn(rt, rt));
}

// Every accepted pair (c <= c2) of cluster (yi, ti) between staged rows jd
// (down) and ju (up): on_pair(qd, yd, td, qu, yu, tu, c). Down candidates are
// taken kBatch at a time into registers, then the up row is visited once per
// batch.
template <class Rows, class Fn>
__device__ inline void visit_pairs(const Rows &A, const TileGeo &G, const YCell &ycd, const YCell &ycu, int jd,
                                   int ju, float yi, float ti, float w, float wy, float wt, float c2, Fn &&on_pair,
                                   int *n_box = nullptr) {
    // n_box (optional): clusters in the box on the down and the up row
    for (int skip = 0;; skip += kBatch) {
        float dy[kBatch], dt[kBatch];
        int dq[kBatch];
        int nd = 0, seen = 0;
        box_visit<true>(A, G, ycd, jd, yi, ti, wy, wt, [&](int q, float y, float t) {
            if (seen >= skip && nd < kBatch) {
#pragma unroll
                for (int k = 0; k < kBatch; k++)
                    if (k == nd) {
                        dy[k] = y;
                        dt[k] = t;
                        dq[k] = q;
                    }
                nd++;
            }
            seen++;
        });
        if (nd == 0) {
            if (n_box) {
                int nu = 0;
                box_visit<false>(A, G, ycu, ju, yi, ti, wy, wt, [&](int, float, float) { nu++; });
                *n_box = seen + nu;
            }
            return;
        }
        int nu = 0;
        box_visit<false>(A, G, ycu, ju, yi, ti, wy, wt, [&](int qu, float yu, float tu) {
            nu++;
#pragma unroll
            for (int k = 0; k < kBatch; k++) {
                if (k >= nd) break;
                const float c = pair_score(yi, ti, dy[k], dt[k], yu, tu, w);
                if (c <= c2) on_pair(dq[k], dy[k], dt[k], qu, yu, tu, c);
            }
        });
        if (n_box && skip == 0) *n_box = seen + nu;
        if (seen <= skip + kBatch) return;
    }
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
    f[0] = f2bf(__fdiv_rn(dyu, wy));
    f[1] = f2bf(__fdiv_rn(dtu, wt));
    f[2] = f2bf(__fdiv_rn(dyd, wy));
    f[3] = f2bf(__fdiv_rn(dtd, wt));
    f[4] = f2bf((float)g);
    f[5] = f2bf(__fdiv_rn(xi, 245.0f));
    f[6] = f2bf(__fdiv_rn(ry, c2s));
    f[7] = f2bf(__fdiv_rn(rt, c2s));
    f[8] = f2bf(__fdiv_rn(kap, 0.015f));
    f[9] = f2bf(__fdiv_rn(by, cx));
    f[10] = f2bf(__fdiv_rn(bt, cx));
    f[11] = f2bf(__fdiv_rn((float)ncand, 8.0f));
    f[12] = f[13] = f[14] = f[15] = 0;
}

// Shared state of one tile (Cap: clusters it can stage).
template <int Cap, int QCap = kQueueCap>
struct TileSharedT {
    static constexpr int kCap = Cap;
    float2 yt[Cap];
    uint8_t cell[Cap];
    int16_t oq[Cap];
    int16_t fs[kSlots][kTileFb + 1];
    int16_t queue[QCap];
    YCell yc[kSlots];
    int32_t base[kSlots + 1];      // LDS index of each staged row (prefix of n)
    int32_t plo[kSlots];           // first staged sorted position of each row
    int32_t n[kSlots];             // staged clusters of each row
    int32_t olo[kSlots];           // own range of each own row, row-local
    int32_t opre[kTileRows + 1];   // prefix of own counts over the own rows
    int32_t scan[kLinkBlock];
    int32_t item, nq, links, cpos, cend, pbase;
};
using TileShared = TileSharedT<kTileCap>;

// Best pair of one cluster at gap g (false: none). bu/bd are sorted positions.
template <class Rows, class TS>
__device__ inline bool best_pair(const Rows &A, const TileGeo &G, const TS &T, const KArgs &a, int j, int r,
                                 int g, float yi, float ti, int &bu, int &bd) {
    const int jd = j - g, ju = j + g;
    const float w = a.w_tab[r * kMaxGap + g - 1];
    const float wy = a.win_y[g - 1], wt = a.win_t[g - 1];
    bool found = false;
    float bc = 0.f;
    int bqu = 0, bqd = 0;
    visit_pairs(A, G, T.yc[jd], T.yc[ju], jd, ju, yi, ti, w, wy, wt, a.pair_c2,
                [&](int qd, float, float, int qu, float, float, float c) {
                    bool better = !found || c < bc;
                    if (found && c == bc) {
                        // exact tie of the score: compare input indices
                        const int idu = a.rec[A.pos(ju, qu)].id, idd = a.rec[A.pos(jd, qd)].id;
                        const int biu = a.rec[A.pos(ju, bqu)].id, bid = a.rec[A.pos(jd, bqd)].id;
                        better = idu < biu || (idu == biu && idd < bid);
                    }
                    if (better) {
                        found = true;
                        bc = c;
                        bqu = qu;
                        bqd = qd;
                    }
                });
    if (found) {
        bu = A.pos(ju, bqu);
        bd = A.pos(jd, bqd);
    }
    return found;
}

// Own cluster o of the tile -> staged row j and row-local index q.
template <class TS>
__device__ inline void own_locate(const TS &T, int jr0, int nown, int o, int &j, int &q) {
    int k = 0;
    while (k + 1 < nown && T.opre[k + 1] <= o) k++;
    j = jr0 + k;
    q = T.olo[j] + (o - T.opre[k]);
}

template <int Mode, bool InLds>
__device__ void tile_links(const KArgs &a, TileShared &T, const TileGeo &G, int si, int r0, int s0, int nown,
                           int own_total) {
    const int R = a.n_rows;
    const int tid = threadIdx.x;
    const int jr0 = r0 - s0;
    const int G2 = a.max_gap;
    LdsRows L{T.yt, T.cell, T.oq, T.base, T.plo, T.fs};
    GlbRows Gl{a.rec, T.plo, T.n, a.coff + ((int64_t)si * R + s0) * (kNcbMax + 1), G};
    int nl = 0;
    if (Mode == kPlain) {
        for (int o = tid; o < own_total; o += kLinkBlock) {
            int j, q;
            own_locate(T, jr0, nown, o, j, q);
            const int r = s0 + j;
            const float2 e = InLds ? L.at(j, q) : Gl.at(j, q);
            int bu = -1, bd = -1;
            bool done = true;
            if (r >= 1 && r + 1 <= R - 1) {
                const bool f = InLds ? best_pair(L, G, T, a, j, r, 1, e.x, e.y, bu, bd)
                                     : best_pair(Gl, G, T, a, j, r, 1, e.x, e.y, bu, bd);
                if (!f && G2 >= 2 && r >= 2 && r + 2 <= R - 1) {
                    const int slot = InLds ? atomicAdd(&T.nq, 1) : kQueueCap;
                    if (slot < kQueueCap) {
                        // searched by the whole workgroup after this pass
                        T.queue[slot] = (int16_t)o;
                        done = false;
                    } else if (InLds) {
                        best_pair(L, G, T, a, j, r, 2, e.x, e.y, bu, bd);
                    } else {
                        best_pair(Gl, G, T, a, j, r, 2, e.x, e.y, bu, bd);
                    }
                }
            }
            if (done) {
                a.link[InLds ? L.pos(j, q) : Gl.pos(j, q)] = make_int2(bu, bd);
                nl += (bu >= 0);
            }
        }
        __syncthreads();
        const int nq = InLds ? min(T.nq, kQueueCap) : 0;
        for (int k = tid; k < nq; k += kLinkBlock) {
            const int o = T.queue[k];
            int j, q;
            own_locate(T, jr0, nown, o, j, q);
            const int r = s0 + j;
            const float2 e = InLds ? L.at(j, q) : Gl.at(j, q);
            int bu = -1, bd = -1;
            best_pair(L, G, T, a, j, r, 2, e.x, e.y, bu, bd);
            a.link[L.pos(j, q)] = make_int2(bu, bd);
            nl += (bu >= 0);
        }
    } else {
        // every triplet of every gap goes to the pool; slots are reserved
        // per pass with a block scan and chunked grabs of the pool counter
        for (int base = 0; base < own_total; base += kLinkBlock) {
            const int o = base + tid;
            const bool act = o < own_total;
            int j = 0, q = 0, r = 0;
            float yi = 0.f, ti = 0.f;
            int ng[kMaxGap] = {}, nc[kMaxGap] = {};
            if (act) {
                own_locate(T, jr0, nown, o, j, q);
                r = s0 + j;
                const float2 e = InLds ? L.at(j, q) : Gl.at(j, q);
                yi = e.x;
                ti = e.y;
                for (int g = 1; g <= G2; g++) {
                    if (r - g < 0 || r + g > R - 1) continue;
                    const int jd = j - g, ju = j + g;
                    const float w = a.w_tab[r * kMaxGap + g - 1];
                    const float wy = a.win_y[g - 1], wt = a.win_t[g - 1];
                    int np = 0;
                    auto cnt = [&](int, float, float, int, float, float, float) { np++; };
                    if (InLds) visit_pairs(L, G, T.yc[jd], T.yc[ju], jd, ju, yi, ti, w, wy, wt, a.pair_c2, cnt, &nc[g - 1]);
                    else visit_pairs(Gl, G, T.yc[jd], T.yc[ju], jd, ju, yi, ti, w, wy, wt, a.pair_c2, cnt, &nc[g - 1]);
                    ng[g - 1] = np;
                }
            }
            int tot = 0;
#pragma unroll
            for (int g = 0; g < kMaxGap; g++) tot += ng[g];
            T.scan[tid] = tot;
            __syncthreads();
            for (int off = 1; off < kLinkBlock; off <<= 1) {
                const int xv = (tid >= off) ? T.scan[tid - off] : 0;
                __syncthreads();
                T.scan[tid] += xv;
                __syncthreads();
            }
            const int excl = T.scan[tid] - tot;
            if (tid == kLinkBlock - 1) {
                const int total = T.scan[tid];
                if (T.cpos + total > T.cend) {
                    const int grab = max(total, kPoolChunk);
                    T.cpos = atomicAdd(&a.cnt->pool_next, grab);
                    T.cend = T.cpos + grab;
                }
                T.pbase = T.cpos;
                T.cpos += total;
                if (total) atomicAdd(&a.cnt->pool_used, total);
            }
            __syncthreads();
            const int slot0 = T.pbase + excl;
            if (act) {
                const int p = InLds ? L.pos(j, q) : Gl.pos(j, q);
                const bool fits = (int64_t)slot0 + tot <= (int64_t)a.pool_cap;
                if (fits) {
                    int sl = slot0;
                    for (int g = 1; g <= G2; g++) {
                        if (ng[g - 1] == 0) continue;
                        const int jd = j - g, ju = j + g;
                        const float w = a.w_tab[r * kMaxGap + g - 1];
                        const float wy = a.win_y[g - 1], wt = a.win_t[g - 1];
                        const float xd = a.row_x[r - g], xi = a.row_x[r], xu = a.row_x[r + g];
                        const int ncd = nc[g - 1];
                        auto put = [&](int qd, float yd, float td, int qu, float yu, float tu, float c) {
                            uint16_t f[kMlpInP];
                            triplet_features(yd, td, xd, yi, ti, xi, yu, tu, xu, g, wy, wt, w, a.c2s, ncd, f);
                            uint4 *dst = reinterpret_cast<uint4 *>(a.pfeat + (int64_t)sl * kMlpInP);
                            dst[0] = make_uint4(f[0] | ((uint32_t)f[1] << 16), f[2] | ((uint32_t)f[3] << 16),
                                                f[4] | ((uint32_t)f[5] << 16), f[6] | ((uint32_t)f[7] << 16));
                            dst[1] = make_uint4(f[8] | ((uint32_t)f[9] << 16), f[10] | ((uint32_t)f[11] << 16), 0u, 0u);
                            a.pd[sl] = InLds ? L.pos(jd, qd) : Gl.pos(jd, qd);
                            a.pu[sl] = InLds ? L.pos(ju, qu) : Gl.pos(ju, qu);
                            a.pc[sl] = c;
                            sl++;
                        };
                        if (InLds) visit_pairs(L, G, T.yc[jd], T.yc[ju], jd, ju, yi, ti, w, wy, wt, a.pair_c2, put);
                        else visit_pairs(Gl, G, T.yc[jd], T.yc[ju], jd, ju, yi, ti, w, wy, wt, a.pair_c2, put);
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
    for (int off = 32; off > 0; off >>= 1) nl += __shfl_xor(nl, off);
    if ((tid & 63) == 0 && nl) atomicAdd(&T.links, nl);
}

// LDS written by lanes of one wave and read by others of the same wave:
// the wave's LDS operations complete in order; this keeps the compiler from
// moving them across.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------- plain search in LDS
// The plain search of a staged tile, 64 own clusters per wave and round, with
// loops whose trip counts are uniform over the wave (the maximum over its
// lanes; lanes past their own count are masked), so that control flow
// stays on the scalar unit once per step instead of once per lane branch:
//  1. each lane takes the staged positions of the fine bins its box overlaps
//     on the down and the up row (rows are staged in fine-bin order);
//  2. box tests over those ranges, 32 positions per step, give a bit mask of
//     the candidates on each row;
//  3. every (down, up) pair of set bits is scored, and the lexicographic
//     minimum of (c, up input index, down input index) kept.
// Clusters without a gap-1 pair wait in their wave's queue and are searched
// at gap 2, 64 at a time.
constexpr int kPlainWq = kQueueCap / (kLinkBlock / 64);    // gap-2 queue of a wave

// Maximum over the wave (every lane active): within each row of 16 lanes by
// cross-lane moves (swap neighbours, pairs, half-row mirror, row mirror),
// then over the four rows by lane reads.
__device__ inline int wave_max_u(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false));
    return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Staged fine-bin range of row j overlapped by [tlo, thi] (absolute LDS
// positions; lo == hi: empty).
__device__ inline void bin_range(const TileShared &T, const TileGeo &G, int j, int f0, int f1, int &lo, int &hi) {
    const int b = T.base[j];
    if (f1 < 0 || f0 >= G.nfb) {
        lo = hi = b;
        return;
    }
    lo = b + T.fs[j][max(f0, 0)];
    hi = b + T.fs[j][min(f1, G.nfb - 1) + 1];
}

// Bit mask of the positions lo + k0 + [0, 32) in [lo, hi) whose cluster lies
// in the box around (yi, ti) (down row: |yi - y| and |ti - t|; up row:
// |y - yi| and |t - ti|). nk: the wave-uniform number of positions to test.
// Branch-free: four staged (y, t) pairs are read before any is tested.
template <bool Down>
__device__ inline uint32_t box_mask(const TileShared &T, int lo, int hi, int k0, int nk, float yi, float ti, float wy,
                                    float wt) {
    uint32_t m = 0u;
    for (int k = 0; k < nk; k += 4) {
        float2 e[4];
        int p[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            p[u] = lo + k0 + k + u;
            e[u] = T.yt[p[u] < hi ? p[u] : 0];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const float dy = Down ? __fsub_rn(yi, e[u].x) : __fsub_rn(e[u].x, yi);
            const float dt = Down ? __fsub_rn(ti, e[u].y) : __fsub_rn(e[u].y, ti);
            const uint32_t in = (uint32_t)(p[u] < hi) & (uint32_t)(k + u < nk) & (uint32_t)(fabsf(dy) <= wy) &
                                (uint32_t)(fabsf(dt) <= wt);
            m |= in << (k + u);
        }
    }
    return m;
}

// Best pair of the lane's own cluster (yi, ti) on staged rows jd / ju at gap
// g (act: the lane has a cluster to search). bu/bd: sorted positions or -1.
// Exact ties of the score are resolved on the input indices as they occur.
__device__ void flat_pair_exact(const KArgs &a, const TileShared &T, const TileGeo &G, bool act, int jd, int ju, float yi,
                          float ti, float w, float wy, float wt, int &bu, int &bd) {
    const float st = slack(ti, wt);
    int dlo = 0, dhi = 0, ulo = 0, uhi = 0;
    if (act) {
        const int f0 = fine_bin(__fsub_rn(__fsub_rn(ti, wt), st), G.t0, G.inv_cbw, G.nf) - G.fb0;
        const int f1 = fine_bin(__fadd_rn(__fadd_rn(ti, wt), st), G.t0, G.inv_cbw, G.nf) - G.fb0;
        bin_range(T, G, jd, f0, f1, dlo, dhi);
        bin_range(T, G, ju, f0, f1, ulo, uhi);
    }
    const int maxd = wave_max_u(dhi - dlo), maxu = wave_max_u(uhi - ulo);
    const float c2 = a.pair_c2;
    bool found = false;
    float bc = 0.f;
    int bpu = 0, bpd = 0;
    for (int d0 = 0; d0 < maxd; d0 += 32) {
        const uint32_t dm = box_mask<true>(T, dlo, dhi, d0, min(32, maxd - d0), yi, ti, wy, wt);
        if (!__any(dm != 0u)) continue;
        for (int u0 = 0; u0 < maxu; u0 += 32) {
            const uint32_t um = dm ? box_mask<false>(T, ulo, uhi, u0, min(32, maxu - u0), yi, ti, wy, wt) : 0u;
            // every (down, up) pair of set bits, one pair per step: the wave
            // runs the largest pair count of its lanes
            const int nd = um ? __popc(dm) : 0, nu = __popc(um);
            const int tot = nd * nu;
            const int mt = wave_max_u(tot);
            uint32_t dd = um ? dm : 0u, uu = um;
            for (int k = 0; k < mt; k++) {
                const bool v = k < tot;
                const int pd = dlo + d0 + (v ? __builtin_ctz(dd) : 0);
                const int pu = ulo + u0 + (v ? __builtin_ctz(uu) : 0);
                const float2 ed = T.yt[v ? pd : 0];
                const float2 eu = T.yt[v ? pu : 0];
                const float c = pair_score(yi, ti, ed.x, ed.y, eu.x, eu.y, w);
                const bool acc = v && c <= c2;
                bool better = acc && (!found || c < bc);
                const bool tie = acc && found && c == bc;
                if (__any(tie)) {
                    if (tie) {
                        // exact tie of the score: compare input indices
                        const int idu = a.rec[T.plo[ju] + (pu - T.base[ju])].id;
                        const int idd = a.rec[T.plo[jd] + (pd - T.base[jd])].id;
                        const int biu = a.rec[T.plo[ju] + (bpu - T.base[ju])].id;
                        const int bid = a.rec[T.plo[jd] + (bpd - T.base[jd])].id;
                        better = idu < biu || (idu == biu && idd < bid);
                    }
                }
                found = found || acc;
                bc = better ? c : bc;
                bpu = better ? pu : bpu;
                bpd = better ? pd : bpd;
                // next pair: the next up bit, or the first up bit of the next down bit
                const uint32_t un = uu & (uu - 1u);
                const bool wrap = un == 0u;
                uu = wrap ? um : un;
                dd = wrap ? (dd & (dd - 1u)) : dd;
            }
        }
    }
    if (found) {
        bu = T.plo[ju] + (bpu - T.base[ju]);
        bd = T.plo[jd] + (bpd - T.base[jd]);
    }
}

// The same search without the tie resolution in the loop: a lane only notes
// (tied) that an accepted pair scored exactly its best so far. A lane that
// never notes one has a unique minimum (of two pairs with the final minimal
// score, the later visited finds the earlier as its best), so its result is
// the exact one; the others search again with flat_pair_exact.
__device__ void flat_pair_fast(const KArgs &a, const TileShared &T, const TileGeo &G, bool act, int jd, int ju,
                               float yi, float ti, float w, float wy, float wt, int &bu, int &bd, bool &tied) {
    const float st = slack(ti, wt);
    int dlo = 0, dhi = 0, ulo = 0, uhi = 0;
    if (act) {
        const int f0 = fine_bin(__fsub_rn(__fsub_rn(ti, wt), st), G.t0, G.inv_cbw, G.nf) - G.fb0;
        const int f1 = fine_bin(__fadd_rn(__fadd_rn(ti, wt), st), G.t0, G.inv_cbw, G.nf) - G.fb0;
        bin_range(T, G, jd, f0, f1, dlo, dhi);
        bin_range(T, G, ju, f0, f1, ulo, uhi);
    }
    const int maxd = wave_max_u(dhi - dlo), maxu = wave_max_u(uhi - ulo);
    const float c2 = a.pair_c2;
    bool found = false, tie = false;
    float bc = 0.f;
    int bpu = 0, bpd = 0;
    for (int d0 = 0; d0 < maxd; d0 += 32) {
        const uint32_t dm = box_mask<true>(T, dlo, dhi, d0, min(32, maxd - d0), yi, ti, wy, wt);
        if (!__any(dm != 0u)) continue;
        for (int u0 = 0; u0 < maxu; u0 += 32) {
            const uint32_t um = dm ? box_mask<false>(T, ulo, uhi, u0, min(32, maxu - u0), yi, ti, wy, wt) : 0u;
            const int nd = um ? __popc(dm) : 0, nu = __popc(um);
            const int tot = nd * nu;
            const int mt = wave_max_u(tot);
            uint32_t dd = um ? dm : 0u, uu = um;
            for (int k = 0; k < mt; k++) {
                const bool v = k < tot;
                const int pd = dlo + d0 + (v ? __builtin_ctz(dd) : 0);
                const int pu = ulo + u0 + (v ? __builtin_ctz(uu) : 0);
                const float2 ed = T.yt[v ? pd : 0];
                const float2 eu = T.yt[v ? pu : 0];
                const float c = pair_score(yi, ti, ed.x, ed.y, eu.x, eu.y, w);
                const bool acc = v && c <= c2;
                const bool better = acc && (!found || c < bc);
                tie = tie || (acc && found && c == bc);
                found = found || acc;
                bc = better ? c : bc;
                bpu = better ? pu : bpu;
                bpd = better ? pd : bpd;
                const uint32_t un = uu & (uu - 1u);
                const bool wrap = un == 0u;
                uu = wrap ? um : un;
                dd = wrap ? (dd & (dd - 1u)) : dd;
            }
        }
    }
    tied = tie;
    if (found) {
        bu = T.plo[ju] + (bpu - T.base[ju]);
        bd = T.plo[jd] + (bpd - T.base[jd]);
    }
}

__device__ void flat_pair(const KArgs &a, const TileShared &T, const TileGeo &G, bool act, int jd, int ju, float yi,
                          float ti, float w, float wy, float wt, int &bu, int &bd) {
    bool tied = false;
    flat_pair_fast(a, T, G, act, jd, ju, yi, ti, w, wy, wt, bu, bd, tied);
    if (__any(tied)) {
        int bu2 = -1, bd2 = -1;
        flat_pair_exact(a, T, G, tied, jd, ju, yi, ti, w, wy, wt, bu2, bd2);
        if (tied) {
            bu = bu2;
            bd = bd2;
        }
    }
}

__device__ void tile_links_flat(const KArgs &a, TileShared &T, const TileGeo &G, int r0, int s0, int nown,
                                int own_total) {
    const int R = a.n_rows;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int jr0 = r0 - s0;
    const int G2 = a.max_gap;
    int16_t *WQ = T.queue + wv * kPlainWq;
    int nq = 0, nl = 0;   // nq: wave-uniform
    int base = wv * 64;
    for (;;) {
        const bool drain = nq >= 64 || (base >= own_total && nq > 0);
        if (!drain && base >= own_total) break;
        int o;
        bool act;
        int g;
        if (drain) {
            const int take = min(nq, 64);
            act = lane < take;
            o = act ? (int)WQ[nq - take + lane] : -1;
            nq -= take;
            g = 2;
        } else {
            o = base + lane;
            act = o < own_total;
            if (!act) o = -1;
            base += kLinkBlock;
            g = 1;
        }
        int j = 0, q = 0, r = 0;
        float yi = 0.f, ti = 0.f, w = 0.f;
        if (act) {
            own_locate(T, jr0, nown, o, j, q);
            r = s0 + j;
            const float2 e = T.yt[T.base[j] + q];
            yi = e.x;
            ti = e.y;
            act = r - g >= 0 && r + g <= R - 1;
            if (act) w = a.w_tab[r * kMaxGap + g - 1];
        }
        int bu = -1, bd = -1;
        // g is the same for the whole wave (a fresh round or a gap-2 drain)
        const int gu = __builtin_amdgcn_readfirstlane(g);
        flat_pair(a, T, G, act, j - g, j + g, yi, ti, w, a.win_y[gu - 1], a.win_t[gu - 1], bu, bd);
        // gap 2 for the clusters without a gap-1 pair
        const bool g2 = o >= 0 && g == 1 && bu < 0 && G2 >= 2 && r >= 2 && r + 2 <= R - 1;
        const uint64_t m = __ballot(g2);
        const int ng2 = __popcll(m);
        if (ng2 && nq + ng2 > kPlainWq) {
            // the queue is full: search them now (rare)
            const bool act2 = g2;
            int bu2 = -1, bd2 = -1;
            float w2 = act2 ? a.w_tab[r * kMaxGap + 1] : 0.f;
            flat_pair(a, T, G, act2, j - 2, j + 2, yi, ti, w2, a.win_y[1], a.win_t[1], bu2, bd2);
            if (g2) {
                bu = bu2;
                bd = bd2;
            }
        } else if (g2) {
            WQ[nq + __popcll(m & ((1ull << lane) - 1ull))] = (int16_t)o;
        }
        const bool queued = g2 && !(ng2 && nq + ng2 > kPlainWq);
        if (ng2 && nq + ng2 <= kPlainWq) nq += ng2;
        if (o >= 0 && !queued) {
            a.link[T.plo[j] + q] = make_int2(bu, bd);
            nl += (bu >= 0);
        }
        wave_lds_sync();
    }
    for (int off = 32; off > 0; off >>= 1) nl += __shfl_xor(nl, off);
    if (lane == 0 && nl) atomicAdd(&T.links, nl);
}

// ---------------------------------------------------------------- pruned search
// The network scores the candidate triplets inside the search, one wave at
// a time (no workgroup barrier between the searches of a tile): per round,
// every lane enumerates the accepted pairs of one cluster at one gap (up to
// kPrK of them per round; a cluster with more takes further rounds of its
// wave), the wave packs them into its LDS list in lane order, computes their
// features one lane per pair, scores them in tiles of 16 on the matrix cores
// (the arithmetic of the stand-alone inference), and
// each lane keeps the best surviving pair of its cluster in the (c, up input
// index, down input index) order. Gap 2 is searched only for clusters with
// no surviving gap-1 pair, as in the plain finder: such clusters wait in
// their wave's queue until 64 of them (or the tile's end) fill a round.
constexpr int kWaves = kLinkBlock / 64;
constexpr int kPrEntW = 64 * kPrK;             // pairs of one wave's round
constexpr int kWq = 128;                       // gap-2 queue of a wave

// Lds: the tile is staged in LDS, so a row-local index and a box count are
// below kTileCap and travel in 16 bits (global-memory tiles: 32 bits).
template <bool Lds>
struct alignas(16) PruneSharedT {
    using Idx = std::conditional_t<Lds, uint16_t, int32_t>;
    static constexpr int kJqShift = Lds ? 12 : 24;   // staged row << shift | row-local index
    uint32_t ed[kWaves][kPrEntW];   // down candidate (row-local) | owner lane << 24
    uint32_t eu[kWaves][kPrEntW];   // up candidate (row-local) | pruned << 31
    uint32_t feat[kWaves][64][6];   // BF16 features (pairs) of the pairs being scored
    Idx jq[kLinkBlock];             // owner thread -> staged row and row-local index
    Idx nbox[kLinkBlock];           // owner thread -> clusters in its two boxes at this gap
    int32_t wnq[kWaves];            // queued clusters of each wave
};
static_assert(kTileCap <= (1 << 12) && kPrCap <= kTileCap, "16-bit LDS indices");
using TilePr = TileSharedT<kPrCap, kWaves * kWq>;


__device__ inline int wave_excl_scan(int v, int &total) {
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

// One round of a wave: lane searches cluster (j, q) of row r at gap g if
// act; bu/bd receive the best surviving pair (sorted positions) or stay -1.
// Every lane of the wave must call it.
template <class Rows, class PS>
__device__ void prune_round(const KArgs &a, const Rows &A, const TileGeo &G, const TilePr &T, PS &P,
                            int s0, bool act, int j, int q, int r, int g, int &bu, int &bd, int &scored,
                            int &pruned) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int jd = j - g, ju = j + g;
    const float wy = a.win_y[g - 1], wt = a.win_t[g - 1];
    uint32_t *ED = P.ed[wv], *EU = P.eu[wv];
    float yi = 0.f, ti = 0.f, w = 0.f;
    if (act) {
        const float2 e = A.at(j, q);
        yi = e.x;
        ti = e.y;
        w = a.w_tab[r * kMaxGap + g - 1];
        P.jq[tid] = (typename PS::Idx)((j << PS::kJqShift) | q);
    }
    bool found = false;
    float bc = 0.f;
    int bqu = 0, bqd = 0;
    int nbox = 0;
    for (int skip = 0;; skip += kPrK) {
        uint32_t kd[kPrK], ku[kPrK];
        int ntot = 0;
        if (act) {
            auto take = [&](int qd, float, float, int qu, float, float, float) {
                const int k = ntot - skip;
#pragma unroll
                for (int m = 0; m < kPrK; m++)
                    if (m == k) {
                        kd[m] = (uint32_t)qd;
                        ku[m] = (uint32_t)qu;
                    }
                ntot++;
            };
            visit_pairs(A, G, T.yc[jd], T.yc[ju], jd, ju, yi, ti, w, wy, wt, a.pair_c2, take,
                        skip == 0 ? &nbox : nullptr);
            if (skip == 0) P.nbox[tid] = (typename PS::Idx)nbox;
        }
        const int nk = act ? min(max(ntot - skip, 0), kPrK) : 0;
        int total;
        const int off = wave_excl_scan(nk, total);
        total = __builtin_amdgcn_readfirstlane(total);
#pragma unroll
        for (int m = 0; m < kPrK; m++)
            if (m < nk) {
                ED[off + m] = kd[m] | ((uint32_t)lane << 24);
                EU[off + m] = ku[m];
            }
        wave_lds_sync();
        for (int sub = 0; sub < total; sub += 64) {
            const int e = sub + lane;
            if (e < total) {
                const uint32_t ed = ED[e];
                const int own = (wv << 6) | (int)(ed >> 24), qd = ed & 0xffffff, qu = EU[e];
                const int jq = P.jq[own];
                const int oj = jq >> PS::kJqShift, oq = jq & ((1 << PS::kJqShift) - 1), orr = s0 + oj;
                const float2 ei = A.at(oj, oq), edn = A.at(oj - g, qd), eup = A.at(oj + g, qu);
                uint16_t f[kMlpInP];
                triplet_features(edn.x, edn.y, a.row_x[orr - g], ei.x, ei.y, a.row_x[orr], eup.x, eup.y,
                                 a.row_x[orr + g], g, wy, wt, a.w_tab[orr * kMaxGap + g - 1], a.c2s, P.nbox[own], f);
#pragma unroll
                for (int k = 0; k < 6; k++) P.feat[wv][lane][k] = f[2 * k] | ((uint32_t)f[2 * k + 1] << 16);
            }
            wave_lds_sync();
            const int nsub = min(total - sub, 64);
            const int c = lane & 15, qq = lane >> 4;
            // the weights are read once per step for its (up to 4) tiles;
            // the empty asm keeps the loads from being hoisted into the search
            MlpDev W = a.mlp;
            asm volatile("" : "+s"(W.w1), "+s"(W.w2), "+s"(W.w3), "+s"(W.b1), "+s"(W.b2), "+s"(W.b3));
            const int nt = (nsub + 15) >> 4;
            v4s bx[4];
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const int el = t * 16 + c;
                bx[t] = pack4(0, 0, 0, 0);
                if (el < nsub && qq < 3) bx[t] = pack4(make_uint2(P.feat[wv][el][2 * qq], P.feat[wv][el][2 * qq + 1]));
            }
            float z[4];
            mlp_logit4(MlpStream(W, lane), bx, nt, z);
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const int el = t * 16 + c;
                if (qq == 0 && el < nsub) {
                    scored++;
                    if (!(z[t] >= a.theta)) {
                        EU[sub + el] |= 0x80000000u;
                        pruned++;
                    }
                }
            }
            wave_lds_sync();
        }
#pragma unroll
        for (int m = 0; m < kPrK; m++) {
            if (m >= nk) break;
            const uint32_t u = EU[off + m];
            if (u & 0x80000000u) continue;
            const int qd = (int)kd[m], qu = (int)(u & 0x7fffffffu);
            const float2 ed = A.at(jd, qd), eu = A.at(ju, qu);
            const float cc = pair_score(yi, ti, ed.x, ed.y, eu.x, eu.y, w);
            bool better = !found || cc < bc;
            if (found && cc == bc) {
                const int idu = a.rec[A.pos(ju, qu)].id, idd = a.rec[A.pos(jd, qd)].id;
                const int biu = a.rec[A.pos(ju, bqu)].id, bid = a.rec[A.pos(jd, bqd)].id;
                better = idu < biu || (idu == biu && idd < bid);
            }
            if (better) {
                found = true;
                bc = cc;
                bqu = qu;
                bqd = qd;
            }
        }
        // the list is rewritten by the next round
        wave_lds_sync();
        if (!__any(act && ntot > skip + kPrK)) break;
    }
    if (found) {
        bu = A.pos(ju, bqu);
        bd = A.pos(jd, bqd);
    }
}

template <bool InLds>
__device__ void tile_prune(const KArgs &a, TilePr &T, PruneSharedT<InLds> &P, const TileGeo &G, int si, int r0, int s0,
                           int nsr, int nown, int own_total) {
    const int R = a.n_rows;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int jr0 = r0 - s0;
    const int G2 = a.max_gap;
    LdsRows L{T.yt, T.cell, T.oq, T.base, T.plo, T.fs};
    GlbRows Gl{a.rec, T.plo, T.n, a.coff + ((int64_t)si * R + s0) * (kNcbMax + 1), G};
    if (!InLds) {
        // row-local indices travel in 24 bits (an error of the run otherwise)
        bool big = false;
        for (int j = 0; j < nsr; j++) big |= T.n[j] >= (1 << 24);
        if (big) {
            if (tid == 0) atomicAdd(&a.cnt->pool_overflow, 1);
            return;
        }
    }
    int16_t *WQ = T.queue + wv * kWq;
    if (lane == 0) P.wnq[wv] = 0;
    wave_lds_sync();
    int nl = 0, scored = 0, pruned = 0;
    auto round = [&](bool act, int o, int g, bool queue_g2) {
        int j = 0, q = 0, r = 0;
        if (act) {
            own_locate(T, jr0, nown, o, j, q);
            r = s0 + j;
            act = r - g >= 0 && r + g <= R - 1;
        }
        int bu = -1, bd = -1;
        if (InLds) prune_round(a, L, G, T, P, s0, act, j, q, r, g, bu, bd, scored, pruned);
        else prune_round(a, Gl, G, T, P, s0, act, j, q, r, g, bu, bd, scored, pruned);
        const bool g2 = o >= 0 && queue_g2 && bu < 0 && G2 >= 2 && r >= 2 && r + 2 <= R - 1;
        const uint64_t m = __ballot(g2);
        if (g2) WQ[P.wnq[wv] + __popcll(m & ((1ull << lane) - 1ull))] = (int16_t)o;
        else if (o >= 0) {
            a.link[InLds ? L.pos(j, q) : Gl.pos(j, q)] = make_int2(bu, bd);
            nl += (bu >= 0);
        }
        wave_lds_sync();
        if (lane == 0) P.wnq[wv] += __popcll(m);
        wave_lds_sync();
    };
    // the waves take the tile's own clusters 64 at a time, round robin; a
    // full queue (64) is searched at gap 2 before the next 64 clusters, the
    // rest at the end (one call site: the round is inlined once)
    int base = wv * 64;
    for (;;) {
        const int nq = __builtin_amdgcn_readfirstlane(P.wnq[wv]);
        const bool drain = nq >= 64 || (base >= own_total && nq > 0);
        if (!drain && base >= own_total) break;
        int o;
        bool act;
        if (drain) {
            const int take = min(nq, 64);
            act = lane < take;
            o = act ? (int)WQ[nq - take + lane] : -1;
            wave_lds_sync();
            if (lane == 0) P.wnq[wv] = nq - take;
            wave_lds_sync();
        } else {
            o = base + lane;
            act = o < own_total;
            if (!act) o = -1;
            base += kLinkBlock;
        }
        round(act, o, drain ? 2 : 1, !drain);
    }
    for (int off = 32; off > 0; off >>= 1) {
        nl += __shfl_xor(nl, off);
        scored += __shfl_xor(scored, off);
        pruned += __shfl_xor(pruned, off);
    }
    if (lane == 0) {
        if (nl) atomicAdd(&T.links, nl);
        if (scored) atomicAdd(&a.cnt->pool_used, scored);
        if (pruned) atomicAdd(&a.cnt->n_pruned, pruned);
    }
}

// InLds: tiles from the work queue, searched in LDS; a tile over the LDS
// budget is appended to the overflow list. !InLds: the overflow tiles, one
// workgroup each, searched in global memory (a separate kernel, so that the
// common kernel keeps its register budget).
template <int Mode, bool InLds> struct ModeShared {};
template <bool InLds> struct ModeShared<kPrune, InLds> { PruneSharedT<InLds> P; };

template <int Mode, bool InLds>
__global__ __launch_bounds__(kLinkBlock, Mode == kPlain ? 4 : 3) void k_links(KArgs a) {
    using TS = std::conditional_t<Mode == kPrune, TilePr, TileShared>;
    __shared__ TS T;
    __shared__ ModeShared<Mode, InLds> X;
    const int R = a.n_rows;
    const int tid = threadIdx.x;
    const int n_tiles = InLds ? min(a.cnt->n_tiles, a.tile_cap) : min(a.cnt->n_glb_tiles, a.tile_cap);
    if (tid == 0) {
        T.cpos = 0;
        T.cend = 0;
    }
    for (int iter = 0;; iter++) {
        if (tid == 0) {
            int v = InLds ? atomicAdd(&a.cnt->tile_next, 1) : (int)blockIdx.x + iter * (int)gridDim.x;
            if ((iter & 15) == 0 && abort_requested(a)) v = n_tiles;
            T.item = v;
            T.nq = 0;
            T.links = 0;
        }
        __syncthreads();
        const int item = T.item;
        if (item >= n_tiles) break;
        const int2 tl = a.tiles[InLds ? item : a.glb_tiles[item]];
        const int w = tl.x;
        const int si = w / a.n_rb, rb = w - si * a.n_rb;
        const int cb0 = tl.y & 0xffff, cb1 = tl.y >> 16;
        const SiState S = a.st[si];
        const int r0 = rb * kTileRows, r1 = min(r0 + kTileRows, R);
        const int s0 = max(r0 - kMaxGap, 0), s1 = min(r1 + kMaxGap, R);
        const int nsr = s1 - s0, nown = r1 - r0;
        const int cb_lo = max(cb0 - 1, 0), cb_hi = min(cb1 + 1, S.ncb);
        TileGeo G;
        G.t0 = S.t0;
        G.inv_cbw = S.inv_cbw;
        G.nf = S.ncb * kFinePerCb;
        G.fb0 = cb_lo * kFinePerCb;
        G.nfb = (cb_hi - cb_lo) * kFinePerCb;
        const int32_t *co_s0 = a.coff + ((int64_t)si * R + s0) * (kNcbMax + 1);
        // wave 0: row ranges and their prefix sums (lane j: staged row j)
        if (tid < 64) {
            const int j = tid;
            int n = 0, own = 0;
            if (j < nsr) {
                const int32_t *co = co_s0 + (int64_t)j * (kNcbMax + 1);
                const int plo = co[cb_lo];
                n = co[cb_hi] - plo;
                T.plo[j] = plo;
                T.n[j] = n;
                T.olo[j] = co[cb0] - plo;
                T.yc[j] = a.ycell[s0 + j];
                if (j >= r0 - s0 && j < r1 - s0) own = co[cb1] - co[cb0];
            }
            int bs = n, os = own;
#pragma unroll
            for (int o = 1; o < 32; o <<= 1) {
                const int x = __shfl_up(bs, o), y = __shfl_up(os, o);
                if (j >= o) {
                    bs += x;
                    os += y;
                }
            }
            if (j < nsr) T.base[j] = bs - n;
            if (j == nsr - 1) T.base[nsr] = bs;
            const int k = j - (r0 - s0);
            if (k >= 0 && k < nown) T.opre[k] = os - own;
            if (k == nown - 1) T.opre[nown] = os;
        }
        __syncthreads();
        const int total = T.base[nsr];
        const int own_total = T.opre[nown];
        if (InLds && total > TS::kCap) {
            if constexpr (Mode == kPlain) {
                // searched at once from global memory by this workgroup, in
                // its place in the queue (the other workgroups go on)
                if (tid == 0) atomicAdd(&a.cnt->n_glb_inline, 1);
                tile_links<Mode, false>(a, T, G, si, r0, s0, nown, own_total);
                __syncthreads();
                if (tid == 0 && T.links) atomicAdd(&a.cnt->n_links, T.links);
            } else {
                if (tid == 0) a.glb_tiles[atomicAdd(&a.cnt->n_glb_tiles, 1)] = item;
            }
            continue;   // uniform: every thread leaves the tile
        }
        if (InLds) {
            // one wave per staged row, in four steps separated by the wave's
            // own LDS ordering (no workgroup barrier):
            //  A: fine bin starts of the row (the previous cluster's bin comes
            //     from the neighbouring lane), y cell and fine bin of every
            //     cluster in row order (the bin in the yt slot, as a temp);
            //  B: every cluster's rank inside its fine bin by (y cell, row
            //     order): a count over the bin, one lane per cluster;
            //  C: the row-local index of each rank (oq);
            //  D: (y, t) and y cell in rank order, read again from the row.
            // The plain search stages each row in its fine-bin order (step A
            // writes (y, t) directly; no ranking).
            {
                const int wv = tid >> 6, lane = tid & 63;
                int2 *yti = reinterpret_cast<int2 *>(T.yt);
                for (int j = wv; j < nsr; j += kLinkBlock / 64) {
                    const int n = T.n[j], bj = T.base[j], plo = T.plo[j];
                    const YCell yc = T.yc[j];
                    // fine-bin starts: every bin at or below the row's last
                    // bin is set by exactly one cluster below; the rest mark
                    // the row's end
                    for (int b = lane; b <= G.nfb; b += 64) T.fs[j][b] = (int16_t)n;
                    wave_lds_sync();
                    int carry = -1;
                    for (int q0 = 0; q0 < n; q0 += 64) {
                        const int q = q0 + lane;
                        int f = 0x7fffffff;
                        if (q < n) {
                            const float2 e = *reinterpret_cast<const float2 *>(a.rec + plo + q);
                            f = fine_bin(e.y, G.t0, G.inv_cbw, G.nf) - G.fb0;
                            if constexpr (Mode == kPlain) {
                                T.yt[bj + q] = e;
                            } else {
                                T.cell[bj + q] = (uint8_t)ycell_of(yc, e.x);
                                yti[bj + q].x = f;
                            }
                        }
                        int fp = __shfl_up(f, 1);
                        if (lane == 0) fp = carry;
                        if (q < n)
                            for (int b = max(fp + 1, 0); b <= min(f, G.nfb); b++) T.fs[j][b] = (int16_t)q;
                        carry = __shfl(f, 63);
                    }
                    if constexpr (Mode == kPlain) continue;   // the plain search takes rows in fine-bin order
                    wave_lds_sync();
                    for (int q = lane; q < n; q += 64) {
                        const int f = yti[bj + q].x;
                        const int lo = T.fs[j][f], hi = T.fs[j][f + 1];
                        const int c = T.cell[bj + q];
                        int rank = lo;
                        for (int m = lo; m < hi; m++) {
                            const int cm = T.cell[bj + m];
                            rank += (cm < c) || (cm == c && m < q);
                        }
                        yti[bj + q].y = rank;
                    }
                    wave_lds_sync();
                    for (int q = lane; q < n; q += 64) T.oq[bj + yti[bj + q].y] = (int16_t)q;
                    wave_lds_sync();
                    for (int s = lane; s < n; s += 64) {
                        const int q = T.oq[bj + s];
                        const float2 e = *reinterpret_cast<const float2 *>(a.rec + plo + q);
                        T.yt[bj + s] = e;
                        T.cell[bj + s] = (uint8_t)ycell_of(yc, e.x);
                    }
                }
            }
            __syncthreads();
            if constexpr (Mode == kPrune) tile_prune<InLds>(a, T, X.P, G, si, r0, s0, nsr, nown, own_total);
            else if constexpr (Mode == kPlain) tile_links_flat(a, T, G, r0, s0, nown, own_total);
            else tile_links<Mode, true>(a, T, G, si, r0, s0, nown, own_total);
        } else {
            if constexpr (Mode == kPrune) tile_prune<InLds>(a, T, X.P, G, si, r0, s0, nsr, nown, own_total);
            else tile_links<Mode, false>(a, T, G, si, r0, s0, nown, own_total);
        }
        __syncthreads();
        if (tid == 0 && T.links) atomicAdd(&a.cnt->n_links, T.links);
    }
}

void launch_links(const KArgs &a, Launch l, hipStream_t s) {
    // tiles too dense for LDS are searched inside the same launch
    hipLaunchKernelGGL((k_links<kPlain, true>), dim3(max(l.grid, 1)), dim3(kLinkBlock), 0, s, a);
}

void launch_links_enum(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL((k_links<kEnum, true>), dim3(max(l.grid, 1)), dim3(kLinkBlock), 0, s, a);
    hipLaunchKernelGGL((k_links<kEnum, false>), dim3(max(l.grid / 4, 1)), dim3(kLinkBlock), 0, s, a);
}

void launch_links_prune(const KArgs &a, Launch l, hipStream_t s) {
    // three workgroups per CU fit the LDS of a pruned search; dense tiles
    // are more frequent at its smaller tile size, so both launches are full
    const int grid = max(l.grid / 4 * 3, 1);
    hipLaunchKernelGGL((k_links<kPrune, true>), dim3(grid), dim3(kLinkBlock), 0, s, a);
    hipLaunchKernelGGL((k_links<kPrune, false>), dim3(grid), dim3(kLinkBlock), 0, s, a);
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
            for (int k = off; k < off + n1 + n2; k++) pruned += !(a.pz[k] >= th);
            for (int g = 0; g < 2 && bu < 0; g++) {
                const int k0 = off + (g ? n1 : 0), k1 = k0 + (g ? n2 : n1);
                bool found = false;
                float bc = 0.f;
                int biu = 0, bid = 0;
                for (int k = k0; k < k1; k++) {
                    if (!(a.pz[k] >= th)) continue;
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

// Training examples from the last pruned run: every triplet is kept with
// probability `keep` (a hash of (seed, sector instance, input index, rank of
// the triplet within its cluster), so the subset does not depend on
// scheduling) and labelled 1 if the run's cleaned links put its down and up
// clusters directly below and above its middle cluster and that cluster is
// on a track, else 0. Output order is arbitrary.
__device__ inline uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_samples(KArgs a, float keep, uint64_t seed, uint16_t *feat, float *label,
                                                 int64_t cap, unsigned long long *n_out) {
    const int n = min(a.cnt->n_valid_total, a.n_in);
    const uint64_t thr = keep >= 1.f ? ~0ull : (uint64_t)((double)keep * 18446744073709551616.0);
    const int lane = threadIdx.x & 63;
    for (int p0 = blockIdx.x * blockDim.x; p0 < n; p0 += gridDim.x * blockDim.x) {
        const int p = p0 + threadIdx.x;
        int off = -1, nt = 0;
        Rec e{};
        int2 l = make_int2(-1, -1);
        bool in_trk = false;
        if (p < n) {
            off = a.hoff[p];
            nt = off >= 0 ? a.hn1[p] + a.hn2[p] : 0;
            if (nt) {
                e = a.rec[p];
                l = a.link[p];
                in_trk = a.assign[a.si[e.sr >> 8].in_base + e.id] >= 0;
            }
        }
        // lanes walk their triplets in lock step; one atomic per wave and step
        int mx = nt;
        for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o));
        for (int j = 0; j < mx; j++) {
            bool take = false;
            float lab = 0.f;
            int k = 0;
            if (j < nt) {
                k = off + j;
                const uint64_t h = mix64(seed ^ mix64(((uint64_t)(e.sr >> 8) << 40) ^ ((uint64_t)e.id << 8) ^ (uint64_t)j));
                take = h < thr;
                if (take) {
                    const int d = a.pd[k], u = a.pu[k];
                    lab = (in_trk && l.y == d && l.x == u && a.link[d].x == p && a.link[u].y == p) ? 1.f : 0.f;
                }
            }
            const uint64_t m = __ballot(take);
            if (!m) continue;
            const int first = __ffsll((unsigned long long)m) - 1;
            unsigned long long base = 0;
            if (lane == first) base = atomicAdd(n_out, (unsigned long long)__popcll(m));
            base = __shfl(base, first);
            if (take) {
                const int64_t o = (int64_t)base + __popcll(m & ((1ull << lane) - 1ull));
                if (o < cap) {
                    const uint4 *src = reinterpret_cast<const uint4 *>(a.pfeat + (int64_t)k * kMlpInP);
                    uint4 *dst = reinterpret_cast<uint4 *>(feat + o * kMlpInP);
                    dst[0] = src[0];
                    dst[1] = src[1];
                    label[o] = lab;
                }
            }
        }
    }
}

void launch_samples(const KArgs &a, float keep, uint64_t seed, uint16_t *feat, float *label, int64_t cap,
                    unsigned long long *n_out, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_samples, dim3(max(grid, 1)), dim3(256), 0, s, a, keep, seed, feat, label, cap, n_out);
}

}  // namespace tpcca
