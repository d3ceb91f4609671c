// Track following and shared-cluster selection after the chains.
//
// The tracker the method derives from (Sec. 1) extends its seeds with a
// Kalman filter, and the capacity planning of Sec. 2 counts on more attached
// hits. Each chain is extended row by row beyond both of its ends with two
// linear 1-D filters (y against x and t against x, state value and slope),
// then every cluster goes to the longest extended track that contains it
// (ties to the smaller seed input index); tracks left with fewer than
// min_track_hits clusters are dropped. Every filter operation is one FP32
// rounding in a fixed order (this file is built without contraction), so
// the selection is the same on any device.
//
//   k_ford_*       the work order: chains by (sector instance, seed time)
//   k_follow       per chain end (4 lanes): filter the chain towards that end,
//                  extend beyond it, write the clusters found (sorted
//                  positions in ascending rows; the inward task adds the
//                  chain's) and claim them with one 32-bit atomicMax each;
//                  key = (length << 24) | (2^24 - 1 - seed input index)
//   k_follow_keep  per chain (4 lanes): clusters whose claim is its own key;
//                  a kept track's chain copy (a run of a multiple of 4
//                  records) and a keep flag per chain track number
//   k_si_follow,   after the scan of the keep flags: per sector instance the
//   k_follow_slots first kept track and count; per kept track its length,
//                  copy offset and seed under its new number
#include "tpcca_internal.h"

namespace tpcca {

namespace {

struct Kf1 {
    float a, b, p00, p01, p11;
};

__device__ inline Kf1 kf1_init(float m, float var, float var_slope0) { return Kf1{m, 0.0f, var, 0.0f, var_slope0}; }

// Prediction by dx: value moves along the slope; the slope variance grows by
// q |dx|.
__device__ inline void kf1_predict(Kf1 &f, float dx, float q) {
    f.a = __fadd_rn(f.a, __fmul_rn(f.b, dx));
    const float u = __fadd_rn(f.p01, __fmul_rn(dx, f.p11));
    const float s = __fadd_rn(f.p00, __fmul_rn(dx, f.p01));
    f.p00 = __fadd_rn(s, __fmul_rn(dx, u));
    f.p01 = u;
    f.p11 = __fadd_rn(f.p11, __fmul_rn(q, fabsf(dx)));
}

// Update with a measurement m of variance s2.
__device__ inline void kf1_update(Kf1 &f, float m, float s2) {
    const float S = __fadd_rn(f.p00, s2);
    const float iS = __fdiv_rn(1.0f, S);
    const float k0 = __fmul_rn(f.p00, iS);
    const float k1 = __fmul_rn(f.p01, iS);
    const float r = __fsub_rn(m, f.a);
    f.a = __fadd_rn(f.a, __fmul_rn(k0, r));
    f.b = __fadd_rn(f.b, __fmul_rn(k1, r));
    const float n00 = __fsub_rn(f.p00, __fmul_rn(k0, f.p00));
    const float n01 = __fsub_rn(f.p01, __fmul_rn(k0, f.p01));
    const float n11 = __fsub_rn(f.p11, __fmul_rn(k1, f.p01));
    f.p00 = n00;
    f.p01 = n01;
    f.p11 = n11;
}

// Bound on the rounding of the box predicate |fl(t - tp)| <= w (see the
// neighbour search): every admitted time lies within w + slack of tp.
__device__ inline float fslack(float v, float w) {
    return __fadd_rn(__fmul_rn(fabsf(v), 1.0e-6f), __fmul_rn(w, 1.0e-3f));
}

// Lanes per track: the G lanes of a group run the filters redundantly (same
// values, same branches), load the chain records and a row's candidates G at
// a time, and reduce the best candidate with shuffles inside the group.
constexpr int kFolG = 4;
constexpr int kFolPerWave = 64 / kFolG;
constexpr int kFolBlock = 256;

__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Sum over the G lanes of a group (all lanes get it).
__device__ inline int group_sum(int v) {
#pragma unroll
    for (int o = kFolG / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ inline int wave_prefix(int v, int &total) {
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

__device__ inline uint32_t claim_key(int T, int seed_id) {
    return ((uint32_t)T << 24) | (uint32_t)(0xFFFFFF - seed_id);
}

// Filter a chain copy (records ch[0..L), chain order ascending rows) through
// both filters, starting at record j_start and moving by dir, G records per
// load (the next chunk is loaded while the current one is filtered).
__device__ inline void filter_chain(const KArgs &a, const Rec *ch, int L, int dir, int gl, int gbase, Kf1 &fy,
                                    Kf1 &ft) {
    const int j_start = dir > 0 ? 0 : L - 1;
    auto load = [&](int c) {
        const int i = c * kFolG + gl;
        return i < L ? ch[j_start + dir * i] : Rec{0.f, 0.f, 0, 0};
    };
    Rec cur = load(0);
    float xq = 0.0f;
    for (int c = 0; c * kFolG < L; c++) {
        const Rec nxt = load(c + 1);
        const int n = min(kFolG, L - c * kFolG);
        for (int s = 0; s < n; s++) {
            const float y = __shfl(cur.y, gbase + s);
            const float t = __shfl(cur.t, gbase + s);
            const int sr = __shfl(cur.sr, gbase + s);
            const float xj = a.row_x[sr & 255];
            if (c == 0 && s == 0) {
                fy = kf1_init(y, a.f_var_y, a.f_var_s0);
                ft = kf1_init(t, a.f_var_t, a.f_var_s0);
            } else {
                const float dx = __fsub_rn(xj, xq);
                kf1_predict(fy, dx, a.f_q);
                kf1_predict(ft, dx, a.f_q);
                kf1_update(fy, y, a.f_var_y);
                kf1_update(ft, t, a.f_var_t);
            }
            xq = xj;
        }
        cur = nxt;
    }
}

// One extension from row r_end in direction dir (+1 outward, -1 inward), the
// filters already at x[r_end]. The sorted positions of the accepted clusters
// go to the chain's LDS staging row (written by the group's first lane): the
// outward ones to stg[0], stg[1], ..., the inward ones to stg[R - 1],
// stg[R - 2], ... (together at most R - L entries: the chain's own rows are
// never visited); returns their count.
__device__ int extend(const KArgs &a, int si, const SiState &S, int r_end, int dir, Kf1 &fy, Kf1 &ft, int gl,
                      int32_t *stg) {
    const int R = a.n_rows;
    const int nf = S.ncb * kFinePerCb;
    const float wy = a.f_win_y, wt = a.f_win_t;
    const int32_t *co_si = a.coff + (int64_t)si * R * (kNcbMax + 1);
    const uint32_t *fo_si = a.foff + (int64_t)si * R * kNcbMax;
    int n = 0, miss = 0;
    float xp = a.row_x[r_end];
    for (int r = r_end + dir; r >= 0 && r < R; r += dir) {
        const float xr = a.row_x[r];
        const float dx = __fsub_rn(xr, xp);
        kf1_predict(fy, dx, a.f_q);
        kf1_predict(ft, dx, a.f_q);
        xp = xr;
        const float vy = __fadd_rn(fy.p00, a.f_var_y), vt = __fadd_rn(ft.p00, a.f_var_t);
        const float ivy = __fdiv_rn(1.0f, vy), ivt = __fdiv_rn(1.0f, vt);
        const float yp = fy.a, tp = ft.a;
        const float st = fslack(tp, wt);
        const int f0 = fine_bin(__fsub_rn(__fsub_rn(tp, wt), st), S.t0, S.inv_cbw, nf);
        const int f1 = fine_bin(__fadd_rn(__fadd_rn(tp, wt), st), S.t0, S.inv_cbw, nf);
        // candidates: the fine bins f0..f1 (a fine-bin start that does not
        // fit its byte falls back to the coarse bin's bound: a superset)
        const int32_t *co = co_si + (int64_t)r * (kNcbMax + 1);
        const uint32_t *fo = fo_si + (int64_t)r * kNcbMax;
        const int cb0 = f0 / kFinePerCb, k0 = f0 % kFinePerCb;
        const int cb1 = (f1 + 1) / kFinePerCb, k1 = (f1 + 1) % kFinePerCb;
        const int c0s = co[cb0], c1s = co[cb1];
        const uint32_t w0 = fo[cb0], w1 = k1 ? fo[cb1] : 0u;
        const uint32_t b0 = k0 ? (w0 >> (8 * (k0 - 1))) & 255u : 0u;
        const uint32_t b1 = k1 ? (w1 >> (8 * (k1 - 1))) & 255u : 0u;
        const int lo = b0 == 255u ? c0s : c0s + (int)b0;
        const int hi = !k1 ? c1s : b1 == 255u ? co[cb1 + 1] : c1s + (int)b1;
        // each lane: the best of its candidates lo + gl, lo + gl + G, ...
        // (two loads in flight per lane)
        int bid = -1, bp = -1;
        float bchi = 0.0f, by = 0.0f, bt = 0.0f;
        auto consider = [&](const Rec &e, int p) {
            const float dy = __fsub_rn(e.y, yp), dt = __fsub_rn(e.t, tp);
            if (fabsf(dy) <= wy && fabsf(dt) <= wt) {
                const float chi = __fadd_rn(__fmul_rn(__fmul_rn(dy, dy), ivy), __fmul_rn(__fmul_rn(dt, dt), ivt));
                if (bid < 0 || chi < bchi || (chi == bchi && e.id < bid)) {
                    bid = e.id;
                    bp = p;
                    bchi = chi;
                    by = e.y;
                    bt = e.t;
                }
            }
        };
        for (int pb = lo; pb < hi; pb += 2 * kFolG) {
            const int p0 = pb + gl, p1 = pb + kFolG + gl;
            Rec e0{}, e1{};
            if (p0 < hi) e0 = a.rec[p0];
            if (p1 < hi) e1 = a.rec[p1];
            if (p0 < hi) consider(e0, p0);
            if (p1 < hi) consider(e1, p1);
        }
        // least (chi2, input index) over the group
#pragma unroll
        for (int o = kFolG / 2; o > 0; o >>= 1) {
            const int oid = __shfl_xor(bid, o), op = __shfl_xor(bp, o);
            const float ochi = __shfl_xor(bchi, o), oy = __shfl_xor(by, o), ot = __shfl_xor(bt, o);
            if (oid >= 0 && (bid < 0 || ochi < bchi || (ochi == bchi && oid < bid))) {
                bid = oid;
                bp = op;
                bchi = ochi;
                by = oy;
                bt = ot;
            }
        }
        if (bid >= 0 && bchi <= a.f_chi2) {
            kf1_update(fy, by, a.f_var_y);
            kf1_update(ft, bt, a.f_var_t);
            if (gl == 0) stg[dir > 0 ? n : a.n_rows - 1 - n] = bp;
            n++;
            miss = 0;
        } else if (++miss >= a.f_max_miss) {
            break;
        }
    }
    return n;
}

}  // namespace

// Work order. Chain tracks are taken in (sector instance, seed time) order
// (a counting sort on coarse time slabs), and the ordered list is cut into
// one contiguous share per XCD: workgroup i runs on XCD i mod 8, pops chains
// from its XCD's share and, once that is empty, from the next ones. The
// chains in flight on one XCD then cover a narrow time slab of one sector,
// whose records and coarse bin offsets stay in that XCD's L2.
constexpr int kFordSlab = 8;       // coarse time bins per slab of the order
constexpr int kXcd = 8;

__global__ __launch_bounds__(256) void k_ford_hist(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    const int nt = min(a.cnt->n_tseeds, a.tseed_cap);
    const int nb = kNcbMax / kFordSlab;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nt; k += gridDim.x * blockDim.x) {
        const Rec c0 = a.chain[a.tchoff[k]];
        const int si = c0.sr >> 8;
        const SiState S = a.st[si];
        const int f = fine_bin(c0.t, S.t0, S.inv_cbw, S.ncb * kFinePerCb) / kFinePerCb;
        const int key = si * nb + f / kFordSlab;
        atomicAdd(&a.fhist[key], 1);
    }
}

__global__ __launch_bounds__(256) void k_ford_scatter(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    const int nt = min(a.cnt->n_tseeds, a.tseed_cap);
    const int nb = kNcbMax / kFordSlab;
    int32_t *base = a.fhist + a.n_fbins + 1;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nt; k += gridDim.x * blockDim.x) {
        const Rec c0 = a.chain[a.tchoff[k]];
        const int si = c0.sr >> 8;
        const SiState S = a.st[si];
        const int f = fine_bin(c0.t, S.t0, S.inv_cbw, S.ncb * kFinePerCb) / kFinePerCb;
        a.ford[atomicAdd(&base[si * nb + f / kFordSlab], 1)] = k;
    }
}

// Next run of `count` ordered chains for a wave on XCD xcd: [c, hi), or
// false once every share is empty. q is the share being drained (lane 0).
__device__ inline bool next_chains(int32_t *heads, int nt, int xcd, int count, int &q, int &c, int &hi) {
    const int lane = threadIdx.x & 63;
    int ok = 0, cc = 0, hh = 0;
    if (lane == 0) {
        while (q < kXcd) {
            const int qq = (xcd + q) % kXcd;
            const int lo = (int)((int64_t)nt * qq / kXcd), up = (int)((int64_t)nt * (qq + 1) / kXcd);
            const int b = lo + atomicAdd(&heads[qq], count);
            if (b < up) {
                ok = 1;
                cc = b;
                hh = up;
                break;
            }
            q++;
        }
    }
    q = __shfl(q, 0);
    c = __shfl(cc, 0);
    hi = __shfl(hh, 0);
    return __shfl(ok, 0) != 0;
}

// With following on, the walk's chain copies carry the sorted position of
// each cluster in the id field; the extended tracks and the claims are in
// sorted positions too. A wave takes 8 chains, two groups each: the even
// group extends inward (filters from the outermost cluster down the chain,
// then beyond its innermost one), the odd group outward. The inward group
// writes its clusters in ascending rows followed by the chain's, the outward
// group its clusters in ascending rows: together the extended track. Both
// then claim their clusters with the key of the whole track.
// Dynamic LDS: n_rows staging entries per chain of the block.
__global__ __launch_bounds__(kFolBlock, 8) void k_follow(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    extern __shared__ int32_t fol_stage[];
    const int nt = min(a.cnt->n_tseeds, a.tseed_cap);
    const int R = a.n_rows;
    const int lane = threadIdx.x & 63;
    const int gl = lane & (kFolG - 1), gbase = lane & ~(kFolG - 1), grp = lane / kFolG;
    const bool inward = (grp & 1) == 0;
    // one staging row per chain, shared by its inward and outward group
    int32_t *stg = fol_stage + ((threadIdx.x >> 6) * (kFolPerWave / 2) + (grp >> 1)) * R;
    uint32_t *claim = reinterpret_cast<uint32_t *>(a.assign);
    const int xcd = blockIdx.x % kXcd;
    int q = 0, c = 0, hi = 0;
    int added = 0;
    while (next_chains(a.cnt->fq, nt, xcd, kFolPerWave / 2, q, c, hi)) {
        const int cj = c + (grp >> 1);
        const bool valid = cj < hi;
        const int k = valid ? a.ford[cj] : 0;
        int n = 0, L = 0, seed_id = 0;
        const Rec *ch = nullptr;
        if (valid) {
            L = a.tlen[k];
            ch = a.chain + a.tchoff[k];
            const Rec c0 = ch[0], cL = ch[L - 1];
            const int si = c0.sr >> 8;
            const SiState S = a.st[si];
            const int dir = inward ? -1 : 1;
            Kf1 fy, ft;
            filter_chain(a, ch, L, dir, gl, gbase, fy, ft);
            n = extend(a, si, S, (inward ? c0.sr : cL.sr) & 255, dir, fy, ft, gl, stg);
            seed_id = a.rec[c0.id].id;
            if (inward && gl == 0) {
                a.xseed[k] = seed_id;
                a.xsi[k] = si;
            }
        }
        const int m = valid ? n + (inward ? L : 0) : 0;
        const int T = m + __shfl_xor(m, kFolG);   // the partner group's segment
        int n_ent;
        const int r_ent = wave_prefix(gl == 0 ? m : 0, n_ent);
        int o0 = 0;
        if (lane == 0 && n_ent) o0 = atomicAdd(&a.cnt->ext_next, n_ent);
        o0 = __shfl(o0, 0);
        const int64_t off = (int64_t)o0 + __shfl(r_ent, gbase);
        wave_lds_sync();
        if (valid) {
            const int w = 2 * k + (inward ? 0 : 1);
            if (off >= 0 && off + m <= a.ext_cap) {
                int32_t *dst = a.ext + off;
                const uint32_t key = claim_key(T, seed_id);
                for (int i = gl; i < m; i += kFolG) {
                    // inward: staged downwards from the top of the row (so in
                    // ascending rows from R - n), then the chain
                    const int p = !inward ? stg[i] : i < n ? stg[R - n + i] : ch[i - n].id;
                    dst[i] = p;
                    atomicMax(&claim[p], key);
                }
                if (gl == 0) {
                    a.xoff[w] = (int32_t)off;
                    a.xlen[w] = m;
                    added += n;
                }
            } else if (gl == 0) {
                a.xlen[w] = -1;
                atomicAdd(&a.cnt->overflow, 1);
            }
        }
        wave_lds_sync();
    }
    for (int o = 32; o > 0; o >>= 1) added += __shfl_xor(added, o);
    if (lane == 0 && added) atomicAdd(&a.cnt->f_added, added);
}

// The two segments of chain track k's extended track: (inward + chain,
// outward) as (offset, count) pairs; false if either overflowed.
__device__ inline bool segments(const KArgs &a, int k, int &o1, int &n1, int &o2, int &n2) {
    n1 = a.xlen[2 * k];
    n2 = a.xlen[2 * k + 1];
    o1 = a.xoff[2 * k];
    o2 = a.xoff[2 * k + 1];
    return n1 >= 0 && n2 >= 0;
}

__device__ inline int seg_at(const KArgs &a, int o1, int n1, int o2, int i) {
    return a.ext[i < n1 ? o1 + i : o2 + (i - n1)];
}

// Per chain track: the clusters whose claim is its own key; a kept track
// (>= min_track_hits of them) gets its chain copy (records from the sorted
// space, in the extended track's order, padded to a multiple of 4) and a
// keep flag under its chain track number for the scan of the new numbers.
__global__ __launch_bounds__(kFolBlock) void k_follow_keep(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    const int nt = min(a.cnt->n_tseeds, a.tseed_cap);
    const uint32_t *claim = reinterpret_cast<const uint32_t *>(a.assign);
    const int lane = threadIdx.x & 63;
    const int gl = lane & (kFolG - 1), gbase = lane & ~(kFolG - 1), grp = lane / kFolG;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.cnt->n_chains = a.cnt->n_tracks;
    int dropped = 0;
    const int xcd = blockIdx.x % kXcd;
    int q = 0, c = 0, hi = 0;
    while (next_chains(a.cnt->fkq, nt, xcd, kFolPerWave, q, c, hi)) {
        const bool valid = c + grp < hi;
        const int k = valid ? a.ford[c + grp] : 0;
        int T = 0, kept = 0, o1 = 0, n1 = 0, o2 = 0, n2 = 0;
        uint32_t key = 0;
        const bool seg = valid && segments(a, k, o1, n1, o2, n2);
        if (seg) {
            T = n1 + n2;
            key = claim_key(T, a.xseed[k]);
            for (int i = gl; i < T; i += kFolG) kept += claim[seg_at(a, o1, n1, o2, i)] == key;
        }
        kept = group_sum(kept);
        const bool keep = seg && kept >= a.min_track_hits;
        const int len4 = keep ? (kept + 3) & ~3 : 0;
        int n_ent;
        const int r_ent = wave_prefix(gl == 0 ? len4 : 0, n_ent);
        int c0 = 0;
        if (lane == 0 && n_ent) c0 = atomicAdd(&a.cnt->f_chain_next, n_ent);
        c0 = __shfl(c0, 0);
        const int64_t off = (int64_t)c0 + __shfl(r_ent, gbase);
        bool ok = keep && off + len4 <= a.chain_cap;
        if (keep && !ok && gl == 0) atomicAdd(&a.cnt->overflow, 1);
        if (ok) {
            // the walk's chain copies are dead once k_follow has read them:
            // the kept tracks' copies take their place
            Rec *dst = a.chain + off;
            int m = 0;
            for (int i0 = 0; i0 < T; i0 += kFolG) {
                const int i = i0 + gl;
                const int p = i < T ? seg_at(a, o1, n1, o2, i) : -1;
                const bool own = p >= 0 && claim[p] == key;
                const uint32_t gm = (uint32_t)(__ballot(own) >> gbase) & ((1u << kFolG) - 1u);
                if (own) dst[m + __popc(gm & ((1u << gl) - 1u))] = a.rec[p];
                m += __popc(gm);
            }
            const int si = a.xsi[k];
            for (int i = m + gl; i < len4; i += kFolG) dst[i] = Rec{0.f, 0.f, -1, si << 8};
        }
        if (valid && gl == 0) {
            a.klen[k] = ok ? kept : 0;
            a.kchoff[k] = ok ? (int32_t)off : 0;
            dropped += !ok;
            const int g = a.tslot[k];
            if (g < a.trk_cap) a.trk_len[g] = ok ? 1 : 0;
        }
    }
    for (int o = 32; o > 0; o >>= 1) dropped += __shfl_xor(dropped, o);
    if (lane == 0 && dropped) atomicAdd(&a.cnt->f_dropped, dropped);
}

// After the scan of the keep flags (cl_off holds the new number of every
// chain track, cl_off[n_chains] the kept count): per sector instance the
// first kept track and count, per kept track its length, copy and seed.
__global__ void k_si_follow(KArgs a) {
    for (int si = blockIdx.x * blockDim.x + threadIdx.x; si < a.n_si; si += gridDim.x * blockDim.x) {
        const int b = a.st[si].trk_base, n = a.st[si].n_tracks;
        const int nb = a.cl_off[b];
        a.st[si].trk_base = nb;
        a.st[si].n_tracks = a.cl_off[b + n] - nb;
    }
}

__global__ __launch_bounds__(256) void k_follow_slots(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    const int nt = min(a.cnt->n_tseeds, a.tseed_cap);
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nt; k += gridDim.x * blockDim.x) {
        const int kept = a.klen[k];
        const int g = a.tslot[k];
        if (!kept || g >= a.trk_cap) continue;
        const int gn = a.cl_off[g];
        a.trk_len[gn] = kept;
        a.choff[gn] = a.kchoff[k];
        a.trk_seed[gn] = a.xseed[k];
    }
}

void launch_follow(const KArgs &a, Launch l, hipStream_t s) {
    const size_t lds = sizeof(int32_t) * (kFolBlock / 64) * (kFolPerWave / 2) * a.n_rows;
    const int nfb = a.n_fbins;
    hipLaunchKernelGGL(k_ford_hist, dim3(l.grid), dim3(256), 0, s, a);
    launch_scan_i32(a.fhist, nfb, a.fhist + nfb + 1, nullptr, a.scan_tmp, s);
    hipLaunchKernelGGL(k_ford_scatter, dim3(l.grid), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_follow, dim3(l.grid), dim3(kFolBlock), lds, s, a);
    hipLaunchKernelGGL(k_follow_keep, dim3(l.grid), dim3(kFolBlock), 0, s, a);
}

void launch_follow_slots(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL(k_si_follow, dim3((a.n_si + 255) / 256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_follow_slots, dim3(l.grid), dim3(256), 0, s, a);
}

}  // namespace tpcca
