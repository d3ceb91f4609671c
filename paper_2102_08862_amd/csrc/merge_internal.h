// Sector merging (after a run): device arguments and launchers. Not part of
// the C ABI.
#pragma once

#include "tpcca_internal.h"

namespace tpcca {

struct MergeArgs {
    int32_t n_sectors;       // sectors per frame (both sides)
    int32_t membrane;        // 0: adjacent sectors of one side; 1: sector k (A side) with k + n/2 (C side)
    int32_t min_len;         // eligible: at least this many clusters
    float window;            // collision-time window of a candidate pair (cm)
    float d2_cut;            // a pair is a candidate if D2 <= d2_cut
    float bin_w;             // time bin width: the smallest power of two >= window
    float inv_w;             // 1 / bin_w (exact)
    float lo;                // time of bin 0 (a multiple of bin_w)
    int32_t nb;              // bins per sector instance
    uint32_t *range;         // [2] smallest and largest eligible t0 (order-preserving keys)
    int32_t *start;          // [n_si * nb + 1] counts, then their exclusive prefix
    int32_t *cur;            // [n_si * nb] placement cursors
    int32_t *list;           // [tracks] eligible tracks grouped by (sector instance, bin)
    float4 *mst;             // [2 * tracks] their states in list order: (x, y, t, sin phi), (tau, q/pT, t0, phi)
    int32_t *best_next;      // [tracks] best candidate in the next sector (global slot, -1);
                             //   across the membrane: in the C-side sector (A-side tracks)
    int32_t *best_prev;      // [tracks] best candidate in the previous sector (across the
                             //   membrane: in the A-side sector, C-side tracks)
    int32_t *partner_next;   // [tracks] merged partner in the next sector (global slot, -1)
    int32_t *partner_prev;   // [tracks] merged partner in the previous sector
    int32_t *n_elig;         // [1] eligible tracks (the list's length)
    int32_t *n_pairs;        // [1]
};

// Refit of the merged pairs: each pair becomes one virtual track (the first
// track's clusters and its partner's rotated into the first track's frame,
// ordered by x), fitted by the fit kernel with the x carried by each record.
struct RefitArgs {
    int32_t n_sectors;
    int32_t *flags;          // [tracks + 1] 1 where the track has a partner in the next sector
    int32_t *pidx;           // [tracks + 1] exclusive prefix of flags: the pair index of a track
    int32_t *pa, *pb;        // [pairs] the pair's tracks (global slots), A in the lower sector
    int32_t *vlen;           // [pairs + 1] clusters of the virtual track, then (scan) their offsets
    int32_t *voff;           // [pairs + 1]
    int32_t *vseed;          // [pairs] seed of the first track (its tpcca_track.seed)
    int32_t *vperm;          // [pairs] fit order (identity)
    Rec *vchain;             // [entries] virtual chains {y, t, bits of x, (si << 8)}
    int64_t vcap;            // entries available
};

void launch_refit_flags(const KArgs &a, const MergeArgs &m, const RefitArgs &r, int n_tracks, hipStream_t s);
void launch_refit_pairs(const KArgs &a, const MergeArgs &m, const RefitArgs &r, int n_tracks, hipStream_t s);
void launch_refit_build(const KArgs &a, const RefitArgs &r, int n_pairs, hipStream_t s);
void launch_fit_x(const KArgs &a, Launch l, hipStream_t s);

void launch_merge_range(const KArgs &a, const MergeArgs &m, hipStream_t s);
void launch_merge_count(const KArgs &a, const MergeArgs &m, hipStream_t s);
void launch_merge_place(const KArgs &a, const MergeArgs &m, hipStream_t s);
void launch_merge_pairs(const KArgs &a, const MergeArgs &m, int n_tracks, int n_elig, hipStream_t s);

}  // namespace tpcca
