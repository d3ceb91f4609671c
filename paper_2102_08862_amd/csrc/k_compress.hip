// Removal of the clusters of tracks not used for physics (Sec. 1: the
// compression of the synchronous phase drops TPC hits of such tracks, using
// the tracking's assignment). A cluster goes if its track has a successful
// fit and a transverse momentum below the threshold; clusters of no track,
// or of a track whose fit failed, stay. The kept clusters are listed by
// input index, ascending, sector after sector (the run's input chunks in
// order), so that the compressed sector is a plain subset of the input.
//
//   k_rm_flags   per removed track, its clusters' bits in a bitmap over the
//                run's inputs (few tracks go, so the per-cluster passes read
//                one bit per input instead of gathering track records)
//   k_rm_count   kept clusters per input chunk (one workgroup per chunk)
//   (scan)       chunk offsets in the output
//   k_rm_write   order-preserving compaction of each chunk: 32 rounds of
//                256 consecutive inputs; per round a ballot per wave, the
//                (round, wave) counts scanned in LDS, each kept input
//                written at its rank
// Both passes issue a thread's 32 bitmap loads before using any.
#include "compress_internal.h"

namespace tpcca {

namespace {

constexpr int kRmRounds = kChunk / 256;   // 32 rounds of 256 inputs per chunk
static_assert(kChunk % 256 == 0 && kRmRounds <= 32, "one mask bit per round");

// Bit k set: this thread's input of round k (st + 256 k + thread) is kept.
// The bitmap loads of all rounds are issued before any is used.
__device__ inline uint32_t chunk_mask(const RemoveArgs &r, const SiDesc &d, int st, int end) {
    uint32_t wd[kRmRounds];
#pragma unroll
    for (int k = 0; k < kRmRounds; k++) {
        const int c = st + k * 256 + (int)threadIdx.x;
        wd[k] = c < end ? r.bits[(d.in_base + c) >> 5] : 0xffffffffu;
    }
    uint32_t mask = 0;
#pragma unroll
    for (int k = 0; k < kRmRounds; k++) {
        const int c = st + k * 256 + (int)threadIdx.x;
        const bool kp = c < end && !((wd[k] >> ((d.in_base + c) & 31)) & 1u);
        mask |= (kp ? 1u : 0u) << k;
    }
    return mask;
}

}  // namespace

__global__ __launch_bounds__(256) void k_rm_flags(KArgs a, RemoveArgs r, int nt) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nt; g += gridDim.x * blockDim.x) {
        const tpcca_track &T = a.trk[g];
        if (!(T.status == 0 && fabsf(T.qpt) > r.qpt_max)) continue;
        // a removed track: mark its clusters (its list holds sector-local input indices)
        const int in_base = a.si[T.frame * r.n_sectors + T.sector].in_base;
        const int c0 = a.cl_off[g], L = a.trk_len[g];
        for (int j = 0; j < L; j++) {
            const int gi = in_base + a.clusters[c0 + j];
            atomicOr(&r.bits[gi >> 5], 1u << (gi & 31));
        }
    }
}

__global__ __launch_bounds__(256) void k_rm_count(KArgs a, RemoveArgs r) {
    __shared__ int s_w[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int ch = blockIdx.x; ch < a.n_chunks; ch += gridDim.x) {
        const int si = a.chunk[2 * ch], st = a.chunk[2 * ch + 1];
        const SiDesc d = a.si[si];
        const int end = min(st + kChunk, d.n);
        int cnt = __popc(chunk_mask(r, d, st, end));
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
        if (lane == 0) s_w[w] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) r.ccnt[ch] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_rm_write(KArgs a, RemoveArgs r) {
    __shared__ int s_cnt[kRmRounds * 4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int ch = blockIdx.x; ch < a.n_chunks; ch += gridDim.x) {
        const int si = a.chunk[2 * ch], st = a.chunk[2 * ch + 1];
        const SiDesc d = a.si[si];
        const int end = min(st + kChunk, d.n);
        const uint32_t mask = chunk_mask(r, d, st, end);
        for (int k = 0; k < kRmRounds; k++) {
            const uint64_t b = __ballot((mask >> k) & 1u);
            if (lane == 0) s_cnt[k * 4 + w] = __popcll(b);
        }
        __syncthreads();
        // exclusive prefix of the (round, wave) counts, in input order
        if (threadIdx.x < 64) {
            const int i0 = 2 * threadIdx.x;
            const int v0 = s_cnt[i0], v1 = s_cnt[i0 + 1];
            int x = v0 + v1;
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o);
                if (threadIdx.x >= o) x += y;
            }
            const int ex = x - v0 - v1;
            s_cnt[i0] = ex;
            s_cnt[i0 + 1] = ex + v0;
        }
        __syncthreads();
        const int64_t base = r.ccnt[ch];
        for (int k = 0; k < kRmRounds; k++) {
            const bool kp = (mask >> k) & 1u;
            const uint64_t b = __ballot(kp);
            if (kp) {
                const int64_t pos = base + s_cnt[k * 4 + w] + __popcll(b & below);
                if (pos < r.cap) r.out[pos] = st + k * 256 + threadIdx.x;
            }
        }
        __syncthreads();
    }
}

// Entropy reduction of the cluster properties: one thread per track walks
// its chain copy (16-byte records, rows ascending) and bins, per cluster
// after the first, the row step, the first differences of the quantised
// y and t (1/16 cm, FP32 product rounded to nearest even) and the
// track-model residuals: the first difference for the second cluster, then
// q_j dr_{j-1} - q_{j-1} (dr_{j-1} + dr_j) + q_{j-2} dr_j (exact in 64-bit
// integers). Histograms in LDS per workgroup, added to the global ones.
__device__ inline int ent_bin(long long v) { return (v >= -kEntH && v <= kEntH) ? (int)v + kEntH : kEntBins - 1; }

__global__ __launch_bounds__(256) void k_ent_hist(KArgs a, EntropyArgs e, int nt) {
    __shared__ int32_t h[kEntStreams * kEntBins];
    for (int i = threadIdx.x; i < kEntStreams * kEntBins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < nt; g += gridDim.x * blockDim.x) {
        const int L = a.trk_len[g];
        if (L < 2) continue;
        const Rec *ch = a.chain + a.choff[g];
        if (e.only_si >= 0 && (ch[0].sr >> 8) != e.only_si) continue;
        int r1 = 0, y1 = 0, t1 = 0, r2 = 0, y2 = 0, t2 = 0;   // clusters j - 1 and j - 2
        for (int j = 0; j < L; j++) {
            const Rec c = ch[j];
            const int r = c.sr & 255, qy = __float2int_rn(c.y * 16.f), qt = __float2int_rn(c.t * 16.f);
            if (j >= 1) {
                const int dr = r - r1;
                atomicAdd(&h[0 * kEntBins + ent_bin(dr)], 1);
                atomicAdd(&h[1 * kEntBins + ent_bin((long long)qy - y1)], 1);
                atomicAdd(&h[2 * kEntBins + ent_bin((long long)qt - t1)], 1);
                long long ry = (long long)qy - y1, rt = (long long)qt - t1;
                if (j >= 2) {
                    const long long dp = r1 - r2;
                    ry = (long long)qy * dp - (long long)y1 * (dp + dr) + (long long)y2 * dr;
                    rt = (long long)qt * dp - (long long)t1 * (dp + dr) + (long long)t2 * dr;
                }
                atomicAdd(&h[3 * kEntBins + ent_bin(ry)], 1);
                atomicAdd(&h[4 * kEntBins + ent_bin(rt)], 1);
            }
            r2 = r1; y2 = y1; t2 = t1;
            r1 = r; y1 = qy; t1 = qt;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kEntStreams * kEntBins; i += blockDim.x)
        if (h[i]) atomicAdd(&e.hist[i], h[i]);
}

void launch_entropy_hist(const KArgs &a, const EntropyArgs &e, int n_tracks, hipStream_t s) {
    if (n_tracks > 0)
        hipLaunchKernelGGL(k_ent_hist, dim3(min((n_tracks + 255) / 256, 4096)), dim3(256), 0, s, a, e, n_tracks);
}

// rANS coding of a sector's tracks (ANS coding after the entropy
// reduction, Sec. 1): one thread per track encodes its row steps and
// track-model residuals (streams 0, 3 and 4 of k_ent_hist) from the last
// cluster to the second and, within a cluster, from the last stream to the
// first, so that a decoder reads them in order; a symbol beyond +-kEntH goes as the escape bin followed by its 32
// bits as two uniform 16-bit parts. A first pass counts each track's bytes
// (final state included), a second writes them from the end of the track's
// range backwards, so that they lie in decoding order.
namespace {

__device__ inline void ans_put(uint32_t &x, uint32_t f, uint32_t c, uint8_t *out, int64_t &pos, int &nb) {
    // every coded symbol has f >= 1 (the model comes from the same symbols);
    // the clamp keeps the loop below finite (at most 3 bytes) whatever the table
    f = f ? f : 1u;
    const uint32_t xmax = ((kAnsL >> 16) << 8) * f;
    while (x >= xmax) {
        if (out) out[--pos] = (uint8_t)(x & 255u);
        nb++;
        x >>= 8;
    }
    x = ((x / f) << 16) + (x % f) + c;
}

__device__ inline void ans_sym(uint32_t &x, const AnsArgs &n, int k, long long v, uint8_t *out, int64_t &pos,
                               int &nb) {
    if (v >= -kEntH && v <= kEntH) {
        const int i = k * kEntBins + (int)v + kEntH;
        ans_put(x, n.freq[i], n.cum[i], out, pos, nb);
    } else {
        const uint32_t u = (uint32_t)(v & 0xffffffffll);
        ans_put(x, 1u, u & 0xffffu, out, pos, nb);
        ans_put(x, 1u, u >> 16, out, pos, nb);
        const int i = k * kEntBins + kEntBins - 1;
        ans_put(x, n.freq[i], n.cum[i], out, pos, nb);
    }
}

// Encodes track g; out == nullptr: count only. Returns the byte count.
__device__ inline int ans_track(const KArgs &a, const AnsArgs &n, int g, uint8_t *out, int64_t end) {
    const int L = a.trk_len[g];
    const Rec *ch = a.chain + a.choff[g];
    uint32_t x = kAnsL;
    int nb = 0;
    int64_t pos = end;
    for (int j = L - 1; j >= 1; j--) {
        const Rec c0 = ch[j], c1 = ch[j - 1];
        const int r = c0.sr & 255, r1 = c1.sr & 255;
        const int qy = __float2int_rn(c0.y * 16.f), qt = __float2int_rn(c0.t * 16.f);
        const int y1 = __float2int_rn(c1.y * 16.f), t1 = __float2int_rn(c1.t * 16.f);
        const int dr = r - r1;
        long long ry = (long long)qy - y1, rt = (long long)qt - t1;
        if (j >= 2) {
            const Rec c2 = ch[j - 2];
            const long long dp = r1 - (c2.sr & 255);
            const int y2 = __float2int_rn(c2.y * 16.f), t2 = __float2int_rn(c2.t * 16.f);
            ry = (long long)qy * dp - (long long)y1 * (dp + dr) + (long long)y2 * dr;
            rt = (long long)qt * dp - (long long)t1 * (dp + dr) + (long long)t2 * dr;
        }
        // coded: the row step and the track-model residuals (the first
        // differences follow from them)
        ans_sym(x, n, 4, rt, out, pos, nb);
        ans_sym(x, n, 3, ry, out, pos, nb);
        ans_sym(x, n, 0, dr, out, pos, nb);
    }
    for (int b = 0; b < 4; b++) {
        if (out) out[--pos] = (uint8_t)(x & 255u);
        nb++;
        x >>= 8;
    }
    return nb;
}

}  // namespace

__global__ __launch_bounds__(256) void k_ans_size(KArgs a, AnsArgs n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n.n_tracks; i += gridDim.x * blockDim.x)
        n.size[i] = ans_track(a, n, n.trk_base + i, nullptr, 0);
}

__global__ __launch_bounds__(256) void k_ans_write(KArgs a, AnsArgs n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n.n_tracks; i += gridDim.x * blockDim.x)
        ans_track(a, n, n.trk_base + i, n.out, n.size[i + 1]);
}

void launch_ans_size(const KArgs &a, const AnsArgs &n, hipStream_t s) {
    if (n.n_tracks > 0)
        hipLaunchKernelGGL(k_ans_size, dim3(min((n.n_tracks + 255) / 256, 4096)), dim3(256), 0, s, a, n);
}

void launch_ans_write(const KArgs &a, const AnsArgs &n, hipStream_t s) {
    if (n.n_tracks > 0)
        hipLaunchKernelGGL(k_ans_write, dim3(min((n.n_tracks + 255) / 256, 4096)), dim3(256), 0, s, a, n);
}

void launch_remove_flags(const KArgs &a, const RemoveArgs &r, int n_tracks, hipStream_t s) {
    if (n_tracks > 0)
        hipLaunchKernelGGL(k_rm_flags, dim3(min((n_tracks + 255) / 256, 65535)), dim3(256), 0, s, a, r, n_tracks);
}

void launch_remove_count(const KArgs &a, const RemoveArgs &r, hipStream_t s) {
    if (a.n_chunks > 0) hipLaunchKernelGGL(k_rm_count, dim3(min(a.n_chunks, 65535)), dim3(256), 0, s, a, r);
}

void launch_remove_write(const KArgs &a, const RemoveArgs &r, hipStream_t s) {
    if (a.n_chunks > 0) hipLaunchKernelGGL(k_rm_write, dim3(min(a.n_chunks, 65535)), dim3(256), 0, s, a, r);
}

}  // namespace tpcca
