// Compression consumers of the assignment (after a run): device arguments
// and launchers. Not part of the C ABI.
#pragma once

#include "tpcca_internal.h"

namespace tpcca {

struct RemoveArgs {
    int32_t n_sectors;       // sectors per frame
    float qpt_max;           // a fitted track with |q/pT| above this is not used for physics (1 / pT_min)
    uint32_t *bits;          // [n_in / 32 + 2] 1: the cluster (job input index) is removed
    int32_t *ccnt;           // [chunks + 1] kept clusters per input chunk, then (scan) their offsets
    int32_t *out;            // [cap] kept input indices (sector-local), sector after sector, ascending
    int64_t cap;
};

// Entropy reduction: symbol histograms of the track clusters.
constexpr int kEntH = 255;                 // symbols in [-kEntH, kEntH] have a bin
constexpr int kEntBins = 2 * kEntH + 2;    // ... and the last bin holds the rest
constexpr int kEntStreams = 5;             // row step; y, t first differences; y, t track-model residuals

struct EntropyArgs {
    int32_t only_si;         // sector instance to take, -1: all
    int32_t *hist;           // [kEntStreams * kEntBins] counts
};

void launch_entropy_hist(const KArgs &a, const EntropyArgs &e, int n_tracks, hipStream_t s);

// rANS coding of one sector's tracks: one 32-bit state per track, 16-bit
// frequency models per stream.
constexpr uint32_t kAnsL = 1u << 23;
struct AnsArgs {
    int32_t trk_base, n_tracks;   // the sector's tracks: global slots [trk_base, trk_base + n_tracks)
    const uint32_t *freq;         // [kEntStreams * kEntBins]
    const uint32_t *cum;          // [kEntStreams * kEntBins]
    int32_t *size;                // [n_tracks + 1] bytes per track, then (scan) their offsets
    uint8_t *out;                 // caller's device buffer
};

void launch_ans_size(const KArgs &a, const AnsArgs &n, hipStream_t s);
void launch_ans_write(const KArgs &a, const AnsArgs &n, hipStream_t s);

void launch_remove_flags(const KArgs &a, const RemoveArgs &r, int n_tracks, hipStream_t s);
void launch_remove_count(const KArgs &a, const RemoveArgs &r, hipStream_t s);
void launch_remove_write(const KArgs &a, const RemoveArgs &r, hipStream_t s);

}  // namespace tpcca
