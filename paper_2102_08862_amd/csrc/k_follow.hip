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
//   k_follow       per chain: filter the chain from each end, extend inward
//                  and outward, write the extended track (input indices in
//                  ascending rows) and claim its clusters with one 32-bit
//                  atomicMax each; key = (length << 24) | (2^24 - 1 - seed id)
//   k_follow_keep  per chain: clusters whose claim is its own key; a keep flag
//                  per canonical track number for the slot scan
//   k_si_follow    per sector instance: first kept track and count
//   k_follow_copy  per kept track: the chain copy of its kept clusters (a run
//                  of a multiple of 4 records), length and copy offset
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
    const float k0 = __fdiv_rn(f.p00, S);
    const float k1 = __fdiv_rn(f.p01, S);
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

__device__ inline int rec_row(const Rec &e) { return e.sr & 255; }

// Bound on the rounding of the box predicate |fl(t - tp)| <= w (see the
// neighbour search): every admitted time lies within w + slack of tp.
__device__ inline float fslack(float v, float w) {
    return __fadd_rn(__fmul_rn(fabsf(v), 1.0e-6f), __fmul_rn(w, 1.0e-3f));
}

// One extension from row r_end in direction dir (+1 outward, -1 inward), the
// filters already at x[r_end]. Accepted clusters (job input indices) go to
// the lane's staging column stg[j * stride], j = n0, n0 + 1, ...; returns
// their count.
__device__ int extend(const KArgs &a, int si, const SiState &S, int in_base, int r_end, int dir, Kf1 &fy, Kf1 &ft,
                      int32_t *stg, int stride, int n0) {
    const int R = a.n_rows;
    const int nf = S.ncb * kFinePerCb;
    const float wy = a.f_win_y, wt = a.f_win_t;
    int n = 0, miss = 0;
    float xp = a.row_x[r_end];
    for (int r = r_end + dir; r >= 0 && r < R; r += dir) {
        const float xr = a.row_x[r];
        const float dx = __fsub_rn(xr, xp);
        kf1_predict(fy, dx, a.f_q);
        kf1_predict(ft, dx, a.f_q);
        xp = xr;
        const float vy = __fadd_rn(fy.p00, a.f_var_y), vt = __fadd_rn(ft.p00, a.f_var_t);
        const float yp = fy.a, tp = ft.a;
        const float st = fslack(tp, wt);
        const int f0 = fine_bin(__fsub_rn(__fsub_rn(tp, wt), st), S.t0, S.inv_cbw, nf);
        const int f1 = fine_bin(__fadd_rn(__fadd_rn(tp, wt), st), S.t0, S.inv_cbw, nf);
        const int32_t *co = a.coff + ((int64_t)si * R + r) * (kNcbMax + 1);
        const int lo = co[f0 / kFinePerCb], hi = co[f1 / kFinePerCb + 1];
        int best = -1, bid = 0;
        float bchi = 0.0f, by = 0.0f, bt = 0.0f;
        for (int p = lo; p < hi; p++) {
            const Rec e = a.rec[p];
            const float dy = __fsub_rn(e.y, yp), dt = __fsub_rn(e.t, tp);
            if (!(fabsf(dy) <= wy && fabsf(dt) <= wt)) continue;
            const float chi = __fadd_rn(__fdiv_rn(__fmul_rn(dy, dy), vy), __fdiv_rn(__fmul_rn(dt, dt), vt));
            if (best < 0 || chi < bchi || (chi == bchi && e.id < bid)) {
                best = p;
                bid = e.id;
                bchi = chi;
                by = e.y;
                bt = e.t;
            }
        }
        if (best >= 0 && bchi <= a.f_chi2) {
            kf1_update(fy, by, a.f_var_y);
            kf1_update(ft, bt, a.f_var_t);
            stg[(int64_t)(n0 + n) * stride] = in_base + bid;
            n++;
            miss = 0;
        } else if (++miss >= a.f_max_miss) {
            break;
        }
    }
    return n;
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

}  // namespace

// Grid: exactly a.f_threads threads (the staging columns).
__global__ __launch_bounds__(256) void k_follow(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    const int nt = min(a.cnt->n_tseeds, a.tseed_cap);
    const int lane = threadIdx.x & 63;
    const int stride = a.f_threads;
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    int32_t *stg = a.fstage + gtid;
    uint32_t *claim = reinterpret_cast<uint32_t *>(a.assign);
    int added = 0;
    for (int base = blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < nt; base += stride) {
        const int k = base + lane;
        int T = 0, nin = 0, nout = 0, L = 0, in_base = 0;
        const Rec *ch = nullptr;
        Rec c0{};
        if (k < nt) {
            L = a.tlen[k];
            ch = a.chain + a.tchoff[k];
            c0 = ch[0];
            const int si = c0.sr >> 8;
            const SiState S = a.st[si];
            in_base = a.si[si].in_base;
            // inward: the filters start at the outermost cluster and take the
            // chain in descending rows
            Rec e = ch[L - 1];
            Kf1 fy = kf1_init(e.y, a.f_var_y, a.f_var_s0), ft = kf1_init(e.t, a.f_var_t, a.f_var_s0);
            float xq = a.row_x[rec_row(e)];
            for (int j = L - 2; j >= 0; j--) {
                e = ch[j];
                const float xj = a.row_x[rec_row(e)];
                const float dx = __fsub_rn(xj, xq);
                xq = xj;
                kf1_predict(fy, dx, a.f_q);
                kf1_predict(ft, dx, a.f_q);
                kf1_update(fy, e.y, a.f_var_y);
                kf1_update(ft, e.t, a.f_var_t);
            }
            nin = extend(a, si, S, in_base, rec_row(c0), -1, fy, ft, stg, stride, 0);
            // outward: from the innermost cluster, chain in ascending rows
            fy = kf1_init(c0.y, a.f_var_y, a.f_var_s0);
            ft = kf1_init(c0.t, a.f_var_t, a.f_var_s0);
            xq = a.row_x[rec_row(c0)];
            for (int j = 1; j < L; j++) {
                e = ch[j];
                const float xj = a.row_x[rec_row(e)];
                const float dx = __fsub_rn(xj, xq);
                xq = xj;
                kf1_predict(fy, dx, a.f_q);
                kf1_predict(ft, dx, a.f_q);
                kf1_update(fy, e.y, a.f_var_y);
                kf1_update(ft, e.t, a.f_var_t);
            }
            nout = extend(a, si, S, in_base, rec_row(e), 1, fy, ft, stg, stride, nin);
            T = nin + L + nout;
        }
        int n_ent;
        const int r_ent = wave_prefix(T, n_ent);
        int o0 = 0;
        if (lane == 0 && n_ent) o0 = atomicAdd(&a.cnt->ext_next, n_ent);
        o0 = __shfl(o0, 0);
        const int64_t off = (int64_t)o0 + r_ent;
        if (k < nt) {
            if (off >= 0 && off + T <= a.ext_cap) {
                int32_t *dst = a.ext + off;
                const uint32_t key = claim_key(T, c0.id);
                // inward entries were staged in descending rows
                for (int j = 0; j < nin; j++) {
                    const int gi = stg[(int64_t)(nin - 1 - j) * stride];
                    dst[j] = gi;
                    atomicMax(&claim[gi], key);
                }
                for (int j = 0; j < L; j++) {
                    const int gi = in_base + ch[j].id;
                    dst[nin + j] = gi;
                    atomicMax(&claim[gi], key);
                }
                for (int j = 0; j < nout; j++) {
                    const int gi = stg[(int64_t)(nin + j) * stride];
                    dst[nin + L + j] = gi;
                    atomicMax(&claim[gi], key);
                }
                a.xoff[k] = (int32_t)off;
                a.xlen[k] = T;
                a.xseed[k] = c0.id;
                a.xsi[k] = c0.sr >> 8;
                added += nin + nout;
            } else {
                a.xlen[k] = 0;
                atomicAdd(&a.cnt->overflow, 1);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) added += __shfl_xor(added, o);
    if (lane == 0 && added) atomicAdd(&a.cnt->f_added, added);
}

__global__ __launch_bounds__(256) void k_follow_keep(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    const int nt = min(a.cnt->n_tseeds, a.tseed_cap);
    const uint32_t *claim = reinterpret_cast<const uint32_t *>(a.assign);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.cnt->n_chains = a.cnt->n_tracks;
    int dropped = 0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nt; k += gridDim.x * blockDim.x) {
        const int T = a.xlen[k];
        int kept = 0;
        if (T > 0) {
            const int32_t *src = a.ext + a.xoff[k];
            const uint32_t key = claim_key(T, a.xseed[k]);
            for (int j = 0; j < T; j++) kept += claim[src[j]] == key;
        }
        const bool keep = kept >= a.min_track_hits;
        a.klen[k] = keep ? kept : 0;
        dropped += !keep;
        const int g = a.tslot[k];
        if (g < a.trk_cap) a.trk_len[g] = keep ? 1 : 0;
    }
    for (int o = 32; o > 0; o >>= 1) dropped += __shfl_xor(dropped, o);
    if ((threadIdx.x & 63) == 0 && dropped) atomicAdd(&a.cnt->f_dropped, dropped);
}

// After the scan of the keep flags (cl_off holds the new slot of every chain
// track, cl_off[n_chains] the kept count).
__global__ void k_si_follow(KArgs a) {
    for (int si = blockIdx.x * blockDim.x + threadIdx.x; si < a.n_si; si += gridDim.x * blockDim.x) {
        const int b = a.st[si].trk_base, n = a.st[si].n_tracks;
        const int nb = a.cl_off[b];
        a.st[si].trk_base = nb;
        a.st[si].n_tracks = a.cl_off[b + n] - nb;
    }
}

__global__ __launch_bounds__(256) void k_follow_copy(KArgs a) {
    TPCCA_ABORT_GUARD(a);
    const int nt = min(a.cnt->n_tseeds, a.tseed_cap);
    const uint32_t *claim = reinterpret_cast<const uint32_t *>(a.assign);
    const int lane = threadIdx.x & 63;
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < nt; base += stride) {
        const int k = base + lane;
        const int kept = k < nt ? a.klen[k] : 0;
        const int len4 = (kept + 3) & ~3;
        int n_ent;
        const int r_ent = wave_prefix(len4, n_ent);
        int c0 = 0;
        if (lane == 0 && n_ent) c0 = atomicAdd(&a.cnt->f_chain_next, n_ent);
        c0 = __shfl(c0, 0);
        if (!kept) continue;
        const int64_t off = (int64_t)c0 + r_ent;
        const int g = a.tslot[k];
        if (g >= a.trk_cap || off + len4 > a.chain_cap) {
            atomicAdd(&a.cnt->overflow, 1);
            continue;
        }
        const int gn = a.cl_off[g];
        const int T = a.xlen[k];
        const int32_t *src = a.ext + a.xoff[k];
        const int seed_id = a.xseed[k];
        const uint32_t key = claim_key(T, seed_id);
        const int si = a.xsi[k];
        const SiDesc d = a.si[si];
        // the chain copies of the walk are dead once k_follow has read them:
        // the kept tracks' copies take their place
        Rec *dst = a.chain + off;
        int m = 0;
        for (int j = 0; j < T; j++) {
            const int gi = src[j];
            if (claim[gi] != key) continue;
            const int id = gi - d.in_base;
            dst[m++] = Rec{d.y[id], d.t[id], id, (si << 8) | (int)d.row[id]};
        }
        for (; m < len4; m++) dst[m] = Rec{0.f, 0.f, -1, si << 8};
        a.trk_len[gn] = kept;
        a.trk_seed[gn] = seed_id;
        a.choff[gn] = (int32_t)off;
    }
}

void launch_follow(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL(k_follow, dim3(a.f_threads / 256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_follow_keep, dim3(l.grid), dim3(256), 0, s, a);
}

void launch_follow_slots(const KArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_si_follow, dim3((a.n_si + 255) / 256), dim3(256), 0, s, a);
}

void launch_follow_copy(const KArgs &a, Launch l, hipStream_t s) {
    hipLaunchKernelGGL(k_follow_copy, dim3(l.grid), dim3(256), 0, s, a);
}

}  // namespace tpcca
