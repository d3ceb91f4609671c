// Internal definitions shared by the HIP kernels and the host side of the
// tracker library. Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tpcca.h"

namespace tpcca {

constexpr int kMaxRows = 255;      // rows are uint8
constexpr int kMaxGap = 2;         // symmetric row gaps handled by the link kernel
constexpr int kNcbMax = 4096;      // coarse time bins per sector row (upper bound)
constexpr int kFinePerCb = 4;      // fine bins per coarse bin (row sort; at most 4: their
                                   // starts inside a coarse bin are packed in one word)
constexpr int kTileRows = 8;       // own pad rows of a neighbour-finding tile
constexpr int kMaxTileCb = 32;     // most own coarse bins of a tile
constexpr int kTileCap = 3072;     // clusters a tile stages in LDS (own rows, +-kMaxGap rows, time halo)
constexpr int kPrCap = 2944;       // the same for the pruned search (its LDS also holds the pair lists)
constexpr int kMaxYCells = 32;     // y cells per pad row in the row order
constexpr int kChunk = 8192;       // clusters per histogram / scatter work item
constexpr int kNSlabMax = 8;       // time slabs per pad row in the row sort's buckets
constexpr float kSlabW = 4096.0f;  // slab width in drift time (cm): slab = floor(t / kSlabW), clamped
constexpr int kSortBins = 2048;    // fine bins of one row-sort bucket: a slab holds kSlabW / cbw coarse
                                   // bins of width cbw >= 8; a row sorted as one bucket, at most this many
static_assert(kSortBins >= (int)kSlabW / 8 * kFinePerCb, "a slab's fine bins must fit the bucket histogram");
constexpr int kSortCap = 8192;     // most clusters a bucket sorts in registers (1024 threads x 8)
constexpr int kScanItems = 2048;   // elements per block of the device-wide scans
constexpr int kMaxStages = 16;
constexpr int kLenBins = 256;      // chain lengths are < 256 (rows are uint8)
constexpr int kMlpIn = 12;         // triplet features
constexpr int kMlpInP = 16;        // padded to the MFMA K of 16
constexpr int kMlpH = 64;          // hidden units per layer
constexpr int kMlpNParam = kMlpH * kMlpInP + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH + 1;
constexpr int kMlpMaxBatch = 8192; // largest training minibatch
constexpr int kPoolChunk = 1024;   // triplet-pool slots reserved per grab
constexpr int kPassBins = 16;      // fit pass histogram: 1..15 passes, the last bin 15 or more

// Device view of the triplet network (BF16 weights, FP32 biases).
struct MlpDev {
    const uint16_t *w1;  // [64][16]
    const uint16_t *w2;  // [64][64]
    const uint16_t *w3;  // [64]
    const float *b1;     // [64]
    const float *b2;     // [64]
    const float *b3;     // [1]
};

// Layout of the caller-owned network state buffer (byte offsets).
struct MlpState {
    static constexpr size_t w1 = 0;                        // BF16 [64][16]
    static constexpr size_t w2 = 2048;                     // BF16 [64][64]
    static constexpr size_t w3 = w2 + 8192;                // BF16 [64]
    static constexpr size_t b1 = w3 + 256;                 // FP32 [64]
    static constexpr size_t b2 = b1 + 256;                 // FP32 [64]
    static constexpr size_t b3 = b2 + 256;                 // FP32 [1]
    static constexpr size_t master = b3 + 256;             // FP32 [kMlpNParam]
    static constexpr size_t adam_m = master + 21504;       // FP32 [kMlpNParam]
    static constexpr size_t adam_v = adam_m + 21504;       // FP32 [kMlpNParam]
    static constexpr size_t step = adam_v + 21504;         // int32 step counter
    static constexpr size_t bytes = step + 256;
};

// Arguments of one training (or gradient-only) step.
struct MlpTrainArgs {
    uint16_t *w1, *w2, *w3;    // BF16 copies, rewritten after an update
    float *b1, *b2, *b3;
    float *master, *adam_m, *adam_v;
    int32_t *step;
    const uint16_t *X;         // [n][16] BF16
    const float *Y;            // [n]
    int32_t n;
    float pos_weight, lr, beta1, beta2, eps, weight_decay;
    int32_t update;            // 1: AdamW step, 0: gradient only
    float *grad_out;           // [kMlpNParam] (gradient-only mode)
    float *loss_out;           // [1] or null
};

// One sector of one frame ("sector instance"), uploaded by the host.
struct SiDesc {
    const uint8_t *row;
    const float *y;
    const float *t;
    int32_t n;          // input clusters
    int32_t in_base;    // offset of the sector's input indices in the job (assignment space)
    int32_t frame, sector;
    int32_t word_base;  // first word of the sector's track-seed bitmap
    int32_t nwords;
};

// Per sector instance, computed on the device during a run.
struct SiState {
    uint32_t tmin_key, tmax_key;   // order-preserving keys of the time range
    float t0;                      // time origin of the bins
    float inv_cbw;                 // 1 / coarse bin width
    int32_t ncb;                   // coarse bins per row
    int32_t n_valid;               // clusters that passed validation
    int32_t sbase;                 // first position of the sector in the sorted space
    int32_t trk_base, n_tracks;    // first global track slot, number of tracks
    int32_t cl_base, n_cl;         // first entry in the cluster lists, entries
    int32_t cps;                   // coarse bins per time slab (0: a coarse bin is wider than a slab,
                                   // every row is sorted as one bucket)
};

// Device counters of one run (zeroed at the start of the run).
struct Counters {
    unsigned long long n_samples;   // training examples written by the sampler (after a run)
    int32_t n_valid_total;
    int32_t n_tiles;
    int32_t tile_next;       // work queue of the neighbour-finding tiles
    int32_t fit_next;        // work queue of the fit (tracks in length order)
    int32_t n_glb_inline;    // dense tiles searched from global memory inside the plain launch
    int32_t n_links;
    int32_t n_seeds;
    int32_t n_tseeds;
    int32_t n_tracks;
    int32_t n_cl;
    int32_t n_invalid;
    int32_t overflow;
    int32_t n_glb_tiles;     // tiles that did not fit in LDS (served from L2)
    int32_t pool_next;       // triplet pool: slots handed out
    int32_t pool_used;       // triplet pool: slots holding triplets
    int32_t pool_overflow;   // triplets that did not fit the pool
    int32_t n_pruned;        // triplets below the logit threshold
    int32_t fit_passes[kPassBins + 1];  // tracks by fit passes taken; [kPassBins]: fits with halved steps
    int32_t chain_next;      // chain copy entries handed out by the walk
    // track following (runs with following only)
    int32_t n_chains;        // chain tracks before the selection
    int32_t ext_next;        // extended-track entries handed out
    int32_t f_added;         // clusters added by the extensions (all chains)
    int32_t f_dropped;       // chain tracks dropped by the selection
    int32_t f_chain_next;    // chain copy entries of the kept tracks handed out
    int32_t fq[8];           // following: per-XCD heads of the ordered chain shares
    int32_t fkq[8];          // the same for the selection
};
static_assert(sizeof(Counters) % 8 == 0 && offsetof(Counters, n_samples) == 0, "64-bit counter first");
static_assert(kFinePerCb >= 1 && kFinePerCb <= 4, "fine-bin starts packed in bytes 0..2 of a word");

// y cells of one pad row: cell = clamp(floor((y - ylo) * inv), 0, ny - 1).
// Within each fine time bin a row is ordered by (cell, t, id), so a box
// lookup binary-searches its first cell. Only the speed of the search
// depends on these values; any choice gives the same links.
struct YCell {
    float ylo, inv;
    int32_t ny, pad;
};

__device__ inline int ycell_of(const YCell &c, float y) {
    float v = __fmul_rn(__fsub_rn(y, c.ylo), c.inv);
    v = fminf(fmaxf(v, -1.0f), (float)c.ny);
    return min(max((int)floorf(v), 0), c.ny - 1);
}

// Fine time bin of a time (non-decreasing in t; the row sort and the
// neighbour tiles use this one definition).
__device__ inline int fine_bin(float t, float t0, float inv_cbw, int nf) {
    const float v = __fmul_rn(__fmul_rn(__fsub_rn(t, t0), inv_cbw), (float)kFinePerCb);
    const float c = fminf(fmaxf(v, -1.0f), (float)nf);
    return min(max((int)c, 0), nf - 1);
}

// Time slab of a cluster: floor(t / kSlabW) (exact: the width is a power of
// two) clamped to [0, kNSlabMax).
__device__ inline int slab_of_t(float t) {
    const float v = fminf(fmaxf(__fmul_rn(t, 1.0f / kSlabW), 0.0f), (float)(kNSlabMax - 1));
    return (int)v;
}

// A cluster in the sorted space: 16 bytes, one load per chain step.
struct Rec {
    float y, t;
    int32_t id;   // sector-local input index
    int32_t sr;   // (sector instance << 8) | row
};

// Everything a kernel needs, passed by value.
struct KArgs {
    // job shape
    int32_t n_si;
    int32_t n_rows;
    int32_t n_in;            // input clusters of the job (sum of n)
    int32_t n_chunks;
    int32_t n_words;
    int32_t seed_cap, tseed_cap, trk_cap;
    // constants of the method
    int32_t max_gap, min_track_hits, kf_passes;
    int32_t n_rb;            // row blocks per sector instance (ceil(n_rows / kTileRows))
    int32_t tile_budget;     // staged clusters a tile may hold (<= kTileCap)
    float win_y[kMaxGap], win_t[kMaxGap];   // (float)g * win, computed on the host
    float pair_c2;
    float cbw_min;
    float bz_kb;             // 2.99792458e-3 * Bz
    float sigma_y2, sigma_t2;
    float var_s, var_tau, var_k;
    float s_max;
    // track following
    int32_t follow;          // 1: extend the chains and resolve shared clusters before the fit
    float f_win_y, f_win_t;  // search box half widths around the prediction
    float f_chi2;            // gate
    float f_q;               // slope variance added per cm of |dx|
    float f_var_y, f_var_t;  // measurement variances
    float f_var_s0;          // initial slope variance
    int32_t f_max_miss;      // consecutive rows without a cluster that end an extension
    // tables
    const float *row_x;      // [n_rows]
    const float *w_tab;      // [n_rows * kMaxGap], (x_r - x_{r-g}) / (x_{r+g} - x_{r-g})
    const struct YCell *ycell; // [n_rows] y cells of the row order
    // buffers
    const SiDesc *si;
    SiState *st;
    Counters *cnt;
    const int32_t *chunk;    // [2 * n_chunks] (si, start)
    int32_t *bcnt;           // [n_si * n_rows * kNSlabMax] clusters per (row, time slab) bucket
    int32_t *bstart;         // [same] first position of the bucket within its sector
    int32_t *bcur;           // [same] scatter cursor
    int32_t sort_cap;        // buckets of at most this many clusters are sorted in registers
    int32_t *coff;           // [n_si * n_rows * (kNcbMax + 1)] global sorted positions
    int16_t *tstart;         // [n_si * n_rb * kNcbMax] first coarse bin of each tile
    int32_t *ntile;          // [n_si * n_rb + 1] tiles per (sector instance, row block)
    int32_t *tile_base;      // [n_si * n_rb + 1] exclusive prefix of ntile
    int2 *tiles;             // [tile_cap] (si * n_rb + rb, cb0 | cb1 << 16)
    int32_t *glb_tiles;      // [tile_cap] tiles over the LDS budget (searched in global memory)
    int32_t tile_cap;
    Rec *tmp;                // [n_in]
    Rec *rec;                // [n_in]
    int2 *link;              // [n_in] (up, dn) as sorted positions
    int32_t *upc;            // [n_in] cleaned up link (mutual), else -1
    int32_t *seeds;          // [seed_cap]
    int32_t *tseed;          // [tseed_cap]
    int32_t *tlen;           // [tseed_cap]
    int32_t *tslot;          // [tseed_cap]
    int32_t *tchoff;         // [tseed_cap] offset of the track's chain copy (per track seed)
    uint32_t *bits;          // [n_words]
    int32_t *wpre;           // [n_words + 1]
    int32_t *trk_len;        // [trk_cap + 1]
    int32_t *trk_seed;       // [trk_cap]
    int32_t *cl_off;         // [trk_cap + 1] offsets of the canonical cluster lists
    int32_t *choff;          // [trk_cap] offset of each track's chain copy (4-entry aligned)
    int32_t *perm;           // [trk_cap] track slots ordered by decreasing length
    int32_t *lhist;          // [kLenBins + 1] length histogram; after the sort: tracks with length >= b
    tpcca_track *trk;        // [trk_cap]
    float *trk_t0;           // [trk_cap] collision time of each track (drift cm; NaN if the fit failed)
    int32_t *clusters;       // [n_in]
    Rec *chain;              // [chain_cap] chain copies {y, t, id, (si << 8) | row}, a run of a multiple
                             // of 4 entries per track (the walk's copies, with following on, hold the
                             // sorted position in place of id)
    int64_t chain_cap;       // n_in + 3 * trk_cap
    int32_t *assign;         // [n_in]
    int2 *asg_pairs;         // [buckets * 16384] (input index, track number), in the dead staging buffer
    int32_t *asg_cnt;        // [buckets] pairs per bucket of 16384 input indices
    int32_t *scan_tmp;       // block sums of the scans
    // track following (per track seed k of the walk)
    int32_t *ext;            // [ext_cap] extended tracks: sorted positions in ascending rows
    int64_t ext_cap;
    int32_t *xoff, *xlen;    // [2 * tseed_cap] per extension task (2k inward + chain, 2k + 1
                             // outward): offset and count of its entries (-1: overflow)
    int32_t *xseed, *xsi;    // [tseed_cap] seed input index (sector-local) and sector instance
    int32_t *klen;           // [tseed_cap] clusters kept (0: dropped)
    int32_t *kchoff;         // [tseed_cap] the kept track's chain copy
    uint32_t *foff;          // [n_si * n_rows * kNcbMax] per coarse bin: starts of its fine bins 1..3
                             // relative to the bin's start, one byte each (255: not known)
    int32_t *ford;           // [tseed_cap] chain tracks in (sector instance, seed time) order
    int32_t *fhist;          // [2 * (n_fbins + 1)] slab counts, then their exclusive prefix
    int32_t n_fbins;         // n_si * (kNcbMax / 8) time slabs
    const volatile int32_t *abort_flag;  // host-mapped
    // learned pruning (pruned runs only)
    int32_t use_mlp;
    int32_t keep_pool;       // pruned run through the triplet pool (else scored in the search)
    float theta;             // prune triplets with logit < theta
    float c2s;               // sqrt(pair_c2), FP32
    int32_t pool_cap;
    uint16_t *pfeat;         // [pool_cap][16] BF16 features
    int32_t *pd, *pu;        // [pool_cap] down / up sorted positions
    float *pc;               // [pool_cap] pair score
    float *pz;               // [pool_cap] logit
    int32_t *hoff;           // [n_in] first pool slot of each cluster
    int32_t *hn1, *hn2;      // [n_in] triplets of gap 1 / gap 2
    MlpDev mlp;
};

// Arguments of the collision grouping (after a run; all but trk_group in the
// dead slot of the scratch region). A side is (frame, A or C): 2 per frame.
struct CollArgs {
    int32_t n_sectors;
    float gap;               // a group ends where t0 jumps by more than this (cm)
    float inv_w;             // 1 / bin width (bins of half the gap)
    int32_t min_len;         // anchors: tracks of at least this many clusters
    float window;            // other tracks join the nearest group within this (cm)
    uint32_t *range;         // [2 * sides] smallest, largest t0 (order-preserving keys)
    int32_t *nbins;          // [sides]
    int32_t *bin_base;       // [sides]
    uint32_t *bin_cnt, *bin_min, *bin_max;   // [bins]
    int32_t *bin_grp;        // [bins] group of a non-empty bin, -1 if empty
    int32_t *n_groups;       // [sides]
    int32_t *grp_base;       // [sides]
    double *grp_sum;         // [groups] sum of the t0 of its anchors (null: first pass)
    int32_t *grp_cnt;        // [groups] anchors
    int32_t *grp_att;        // [groups] other tracks attached
    double *grp_mean;        // [groups] mean t0 of the anchors
    int32_t *trk_group;      // [trk_cap] group within its side, -1: none
};

// Order-preserving map of a float to an unsigned key.
__host__ __device__ inline uint32_t fkey(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float fkey_inv(uint32_t k) {
    uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// The host's abort request (host-mapped memory, read with a system-scope
// load). It only goes from 0 to 1 during a run, so once a kernel sees it set
// every later kernel of the run sees it too: a kernel that checks it at block
// start therefore never consumes the output of a kernel that stopped early.
__device__ inline bool abort_requested(const KArgs &a) {
    return __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0;
}

// Block-uniform abort check at kernel start (uses one LDS word).
#define TPCCA_ABORT_GUARD(a)                                   \
    do {                                                       \
        __shared__ int s_abort_guard;                          \
        if (threadIdx.x == 0) s_abort_guard = abort_requested(a); \
        __syncthreads();                                       \
        if (s_abort_guard) return;                             \
    } while (0)

// Kernel launchers (one per stage); each enqueues on `s`.
struct Launch {
    int grid;    // persistent grid size (blocks)
    int block;   // threads per block
};

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
void launch_copy(const void *src, void *dst, int64_t n16, int grid, hipStream_t s);
void launch_grid_hist(const KArgs &a, Launch l, hipStream_t s);
void launch_grid_setup(const KArgs &a, hipStream_t s);
void launch_grid_scatter(const KArgs &a, Launch l, hipStream_t s);
void launch_grid_rowsort(const KArgs &a, Launch l, hipStream_t s);
void launch_tiles(const KArgs &a, hipStream_t s);
void launch_links(const KArgs &a, Launch l, hipStream_t s);
void launch_links_enum(const KArgs &a, Launch l, hipStream_t s);
void launch_links_prune(const KArgs &a, Launch l, hipStream_t s);
void launch_select(const KArgs &a, Launch l, hipStream_t s);
void launch_samples(const KArgs &a, float keep, uint64_t seed, uint16_t *feat, float *label, int64_t cap,
                    unsigned long long *n_out, int grid, hipStream_t s);
void launch_mlp_infer(const MlpDev &W, const uint16_t *X, const int32_t *n_dev, int32_t n_cap, float *z, int grid,
                      hipStream_t s);
void launch_mlp_train(const MlpTrainArgs &t, hipStream_t s);
void launch_seeds(const KArgs &a, Launch l, hipStream_t s);
void launch_walk(const KArgs &a, Launch l, hipStream_t s);
void launch_track_slots(const KArgs &a, Launch l, hipStream_t s);
void launch_lists(const KArgs &a, Launch l, hipStream_t s);
void launch_len_sort(const KArgs &a, Launch l, hipStream_t s);
void launch_follow(const KArgs &a, Launch l, hipStream_t s);
void launch_follow_slots(const KArgs &a, Launch l, hipStream_t s);
void launch_fit(const KArgs &a, Launch l, hipStream_t s);
// exclusive scans: out[i] = sum_{j<i} f(in[j]), out[n] = total, *total_dst = total
void launch_scan_popc(const uint32_t *in, int32_t n, int32_t *out, int32_t *total_dst, int32_t *tmp,
                      hipStream_t s);
void launch_scan_i32(const int32_t *in, int32_t n, int32_t *out, int32_t *total_dst, int32_t *tmp, hipStream_t s);
void launch_scan_i32_dev(const int32_t *in, const int32_t *n_dev, int32_t n_cap, int32_t *out,
                         int32_t *total_dst, int32_t *tmp, hipStream_t s);
void launch_si_tracks(const KArgs &a, hipStream_t s);
void launch_si_clusters(const KArgs &a, hipStream_t s);
void launch_t0_range(const KArgs &a, const CollArgs &c, hipStream_t s);
void launch_t0_bins(const KArgs &a, const CollArgs &c, int n_sides, hipStream_t s);
void launch_t0_group(const KArgs &a, const CollArgs &c, hipStream_t s);
void launch_t0_attach(const KArgs &a, const CollArgs &c, int n_groups_total, hipStream_t s);

}  // namespace tpcca
