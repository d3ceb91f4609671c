/*
 * tpcca.h - C ABI of the MI355X TPC track finder.
 *
 * The library runs the track-finding step that the paper (Sec. 1) names as
 * the most compute-intensive part of ALICE's synchronous Run 3 processing:
 * full TPC tracking of whole continuous-readout time frames (~10 ms), with
 * the clusters kept in native coordinates (pad row, pad-direction y, drift
 * time) and track seeding that uses time, not z, as its coordinate, because
 * the collisions of a frame are not known before tracking (Sec. 1). A whole
 * frame is resident in GPU memory and device buffers are reused across the
 * sequential steps (Sec. 1). The paper prints no algorithm; the steps below
 * are the ones this library defines:
 *
 *   1. per sector, a per-row search grid ordered by drift time;
 *   2. neighbour links: for every cluster, the best (down, up) pair of
 *      clusters on rows r-g / r+g (g = 1, then 2) by the distance of the
 *      cluster from the straight line through the pair in (y, t), scored in
 *      FP32 with a fixed operation order (bit-reproducible);
 *   3. cleaning to mutual links, and cellular-automaton chains of mutual
 *      links; a chain of >= min_track_hits clusters is a track;
 *   4. an FP32 Kalman helix fit of every track, iterated (re-linearised)
 *      so that it converges to the maximum-a-posteriori helix.
 *
 * Optional inside a run: track following with shared-cluster selection
 * (config.follow), and pruning of candidate triplets by a small network
 * (config.use_mlp). After a run, on the resident results: collision times
 * and candidates (tpcca_find_collisions), merging across adjacent sectors
 * and across the central membrane (tpcca_merge_sectors,
 * tpcca_merge_membrane), the global refit of sector-merged pairs
 * (tpcca_refit_merged), and the compression consumers of the assignment:
 * removal of the clusters of tracks not used for physics
 * (tpcca_remove_clusters), the symbol histograms of the entropy reduction
 * (tpcca_entropy_histograms) and the rANS coding of a sector's track
 * clusters (tpcca_ans_encode).
 *
 * Conventions
 *   - Every function returns a tpcca_status; no exception crosses the ABI.
 *     tpcca_last_error() gives a message for the last failing call.
 *   - One context is used by one host thread at a time.
 *   - A cluster's identity is its index in the arrays passed to
 *     tpcca_load_sector (the sector-local input index). All tie-breaks and
 *     every output ordering use it, so results do not depend on the order
 *     in which the GPU processes anything.
 *   - Device memory: all working buffers of a run live in one caller-owned
 *     arena (tpcca_attach_arena); tpcca_required_arena says how large it
 *     must be for the frames currently loaded. The library itself allocates
 *     device memory only for a small per-context table block (sector
 *     descriptors, chunk list, row tables): 1 MiB in tpcca_create, grown only
 *     by tpcca_required_arena when the loaded frames need more. tpcca_run,
 *     tpcca_synchronize, the fetches and the network calls never allocate;
 *     a run whose tables would not fit fails with STATE instead.
 *     tpcca_run_noalloc runs without an attached arena, in a static device
 *     array owned by the library (TPCCA_NOALLOC_ARENA_BYTES per GPU).
 *   - All device work is enqueued on the caller's stream (tpcca_set_stream)
 *     and tpcca_run() does not wait for it; tpcca_synchronize() does.
 */
#ifndef TPCCA_H
#define TPCCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tpcca_ctx tpcca_ctx;

typedef enum {
    TPCCA_OK = 0,
    TPCCA_ERR_INVALID_ARG = -1, /* bad pointer, size, index or input value */
    TPCCA_ERR_NOMEM = -2,       /* arena missing or too small */
    TPCCA_ERR_CAPACITY = -3,    /* caller's output buffer too small; *n_out holds the size needed */
    TPCCA_ERR_STATE = -4,       /* call not valid in the context's current state */
    TPCCA_ERR_DEVICE = -5,      /* a HIP runtime call failed */
    TPCCA_ERR_ABORTED = -6      /* run stopped by tpcca_request_abort */
} tpcca_status;

/* Tracker constants. tpcca_config_default() fills the defaults listed. */
typedef struct {
    float bz_tesla;            /* solenoid field, 0.5 */
    int32_t n_sectors;         /* sectors per frame, 36 */
    int32_t n_rows;            /* pad rows per sector, 152 (at most 255) */
    const float *row_x;        /* host pointer, [n_rows] local x of each pad row (cm), strictly
                                  increasing; copied by tpcca_create. The default points to a
                                  built-in table x_r = 85 + r*160/151 cm, rounded to float */
    float sigma_y, sigma_t;    /* cluster resolution (cm), 0.1, 0.1 */
    float win_y, win_t;        /* neighbour box half widths per unit row gap (cm), 1.5, 2.0 */
    float pair_c2;             /* largest accepted pair score (cm^2), 0.2 */
    int32_t max_gap;           /* symmetric row gaps tried, 1..max_gap, 2 */
    int32_t min_track_hits;    /* shortest chain reported as a track, 10 */
    float prior_var_sinphi;    /* prior variances of the fit, centred on the three-point */
    float prior_var_tau;       /*   estimate: 1, 1, 100 (GeV^-2) */
    float prior_var_qpt;
    int32_t kf_passes;         /* most passes of the fit (each pass linearises the Kalman
                                  measurement updates about the previous pass's helix); passes
                                  stop once one moves no parameter by more than 3e-5 relative, 12 */
    float s_max;               /* |sin phi| at which a propagation fails, 0.999 */
    int32_t use_mlp;           /* 1: prune candidate triplets with the loaded network, 0 */
    float mlp_logit_threshold; /* triplets with logit below this are pruned, 0 */
    int32_t pool_per_cluster;  /* triplet-pool slots per input cluster (runs that keep the pool), 4 */
    /* Track following (Sec. 1: the tracker derives from one that extends its
       seeds with a Kalman filter; Sec. 2: more attached hits). With follow = 1
       every chain is extended row by row beyond both ends by two linear 1-D
       filters, y(x) and t(x) with state (value, slope), started at one chain
       end with variances (follow_var_y or _t, follow_var_slope0); a prediction
       by dx adds follow_q * |dx| to the slope variance. In each row the
       cluster inside the box |y - y_pred| <= follow_win_y,
       |t - t_pred| <= follow_win_t of least
       chi2 = dy^2 / (P_yy + follow_var_y) + dt^2 / (P_tt + follow_var_t)
       (ties: smaller input index) is taken if chi2 <= follow_chi2;
       follow_max_miss consecutive rows without one end the extension. Each
       cluster then goes to the longest extended track containing it (ties:
       smaller input index of the chain's innermost cluster, the seed); tracks
       keeping fewer than min_track_hits clusters are dropped. Kept tracks are
       numbered in ascending seed input index, list their clusters in
       ascending rows and are fitted; tpcca_track.seed is then the input
       index of the chain's seed. Needs sectors of fewer than 2^24 clusters. */
    int32_t follow;            /* 0 */
    float follow_win_y;        /* 1.5 (cm) */
    float follow_win_t;        /* 1.5 (cm) */
    float follow_chi2;         /* 16 */
    float follow_q;            /* 1e-4 (per cm) */
    float follow_var_y;        /* 0.01 (cm^2) */
    float follow_var_t;        /* 0.01 (cm^2) */
    float follow_var_slope0;   /* 1 */
    int32_t follow_max_miss;   /* 3 */
} tpcca_config;

/* One fitted track. Tracks of a sector are numbered 0..T-1 in ascending
   input index of their first (innermost) cluster. */
typedef struct {
    int32_t frame, sector;
    int32_t n_clusters;        /* clusters in the chain */
    int32_t status;            /* 0 ok; 2: propagation or initialisation failed;
                                  4: not converged within kf_passes passes */
    int64_t first;             /* offset of its clusters in the sector's cluster list */
    int32_t seed;              /* input index of its innermost cluster (with following: of the
                                  innermost cluster of the chain it grew from) */
    int32_t ndf;               /* 2*n_clusters - 5 */
    float x_ref;               /* x of the outermost cluster: parameters are given there */
    float y;                   /* local y (cm) */
    float t_base;              /* input time of the outermost cluster (cm of drift) */
    float dt;                  /* fitted time minus t_base (cm) */
    float sinphi;              /* sin of the transverse direction w.r.t. local x */
    float tau;                 /* d(time)/d(transverse arc length) */
    float qpt;                 /* q/pT (1/GeV) */
    float chi2;                /* data chi2 of the fitted helix over all clusters */
    float cov[15];             /* covariance of (y, t, sinphi, tau, qpt), lower triangle row-major */
} tpcca_track;

/* Figures filled by tpcca_get_stats. Counts are those of the last run.
   Stage times need the timing flag (tpcca_set_timing): each run records HIP
   events on the stream between its stages; stage_ms is the last timed run,
   stage_ms_total the sum over the n_timed_runs runs since timing was
   switched on (back-to-back runs need no synchronisation in between). */
typedef struct {
    int64_t n_clusters;        /* clusters in the run (all loaded frames) */
    int64_t n_links;           /* clusters with an (uncleaned) neighbour pair */
    int64_t n_seeds;           /* chain starts */
    int64_t n_tracks;          /* chains with >= min_track_hits clusters */
    int64_t n_track_clusters;  /* clusters assigned to tracks */
    int64_t n_invalid;         /* input clusters rejected on the device (row or value) */
    int64_t n_overflow_tiles;  /* neighbour-finding tiles too dense for LDS (searched in global memory) */
    int64_t n_triplets;        /* pruned runs: accepted candidate triplets scored by the network */
    int64_t n_pruned;          /* pruned runs: triplets below the threshold (among those examined) */
    int64_t n_pool_overflow;   /* pruned runs: triplets that did not fit the pool (run is invalid); without the
                                  pool, dense-tile pad rows of 2^24 or more clusters */
    int32_t mlp_used;          /* 1 if the last run pruned with the network */
    int64_t n_timed_runs;      /* runs summed in stage_ms_total */
    int32_t n_stages;          /* entries used in stage_ms / stage_name */
    float stage_ms[16];        /* device time per stage, last timed run */
    double stage_ms_total[16]; /* device time per stage summed over the timed runs */
    char stage_name[16][24];
    int64_t n_tiles;           /* neighbour-finding work items (sector, row block, time slab) */
    int64_t fit_passes[16];    /* tracks by fit passes taken: [k] = k passes (k = 1..14),
                                  [15] = 15 or more; [0]: fits that failed at the start */
    int64_t n_fit_restarts;    /* fits in which a step was halved (objective rose or the helix
                                  left the domain) */
    int64_t n_chains;          /* runs with following: chains before the selection (n_tracks: kept) */
    int64_t n_follow_added;    /* runs with following: clusters the extensions added, over all chains */
    int64_t n_follow_dropped;  /* runs with following: chains dropped by the selection */
} tpcca_stats;

/* Fill *out with the defaults above. The defaults are readings of the
   paper, which prints no tracker constants (geometry and field: the TPC of
   Sec. 1; windows, score cut and prior: this library's definition). */
tpcca_status tpcca_config_default(tpcca_config *out);

/* Create a context for one device (the current HIP device). Copies cfg and
   its row table; allocates the context's 1 MiB table block, a side stream
   and its events. Errors: INVALID_ARG for out-of-range constants, DEVICE if
   a HIP call fails. (Sec. 1: one tracker instance per GPU processing whole
   time frames.) */
tpcca_status tpcca_create(const tpcca_config *cfg, tpcca_ctx **out);

/* Release the context (not the arena or the stream, which the caller owns). */
void tpcca_destroy(tpcca_ctx *ctx);

/* Message for the last failing call on this context (never NULL). */
const char *tpcca_last_error(const tpcca_ctx *ctx);

/* Use `stream` (a hipStream_t; NULL = null stream) for all device work. */
tpcca_status tpcca_set_stream(tpcca_ctx *ctx, void *stream);

/* Open a new, empty time frame; *frame_id receives its index (0, 1, ...).
   The unit of work is a whole continuous-readout time frame of ~10 ms whose
   collisions are not separated before tracking (Sec. 1); several frames
   loaded together are tracked in one batched run. */
tpcca_status tpcca_add_frame(tpcca_ctx *ctx, int32_t *frame_id);

/* Drop all frames and their results. */
tpcca_status tpcca_clear_frames(tpcca_ctx *ctx);

/* Clusters are given in native TPC coordinates, pad row, pad direction and
   drift time, because without a collision assignment they cannot be turned
   into spatial coordinates before tracking (Sec. 1). Device pointers let
   clusters already on the GPU stay there (Sec. 3: data remain on the GPU
   between steps).
   Give the clusters of one sector of one frame: n entries of pad row
   (uint8, < n_rows), local y (cm) and drift time (cm). Arrays are SoA.
   is_device_ptr = 0: host arrays, copied before return (the caller may free
   them); they are staged into the arena by the next run. is_device_ptr = 1:
   device arrays, borrowed (not copied) until the next tpcca_synchronize
   after the last run that uses them. Host arrays are validated here
   (INVALID_ARG for a row >= n_rows or a non-finite value); device arrays
   are checked on the device and offending clusters are left out of the run
   and counted in tpcca_stats.n_invalid. A sector given twice for one frame:
   STATE. n = 0 is allowed. */
tpcca_status tpcca_load_sector(tpcca_ctx *ctx, int32_t frame, int32_t sector, int64_t n,
                               const uint8_t *row, const float *y, const float *t, int32_t is_device_ptr);

/* Arena bytes a run over the currently loaded frames needs (the whole
   frame must fit in GPU memory, Sec. 1). Grows the context's table block if
   the loaded frames need more (the only call besides tpcca_create that
   allocates). INVALID_ARG if a run over these frames would exceed the
   32-bit positions of the device buffers (about 1.2e9 clusters). */
tpcca_status tpcca_required_arena(tpcca_ctx *ctx, size_t *bytes);

/* The arena holds every working buffer of a run; buffers that are dead
   after a step are reused by later steps (Sec. 1: memory reuse for the
   sequential steps of the tracking).
   Use [device_ptr, device_ptr + bytes) as the arena (caller-owned device
   memory, e.g. a torch uint8 tensor; 256-byte aligned). Results of earlier
   runs live in the arena and stay valid until the next run or attach. One
   arena may serve several contexts whose runs are serialised on one stream
   (the per-run tables live in each context's own small device block); it
   then holds the results of the last run only, and every sector must have
   been loaded from device pointers (host-loaded sectors are staged in the
   arena). */
tpcca_status tpcca_attach_arena(tpcca_ctx *ctx, void *device_ptr, size_t bytes);

/* Enqueue the whole hot path over every loaded frame on the stream and
   return without waiting: full TPC track finding of the frames (Sec. 1,
   the most compute-intensive synchronous step), seeded with drift time in
   place of z (Sec. 1), derived from the HLT cellular-automaton tracker
   (Sec. 1). NOMEM if the arena is smaller than tpcca_required_arena; STATE
   if no frame is loaded or the frames changed since tpcca_required_arena in
   a way that needs a larger table block. Allocates nothing. */
tpcca_status tpcca_run(tpcca_ctx *ctx);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): tpcca_run
   with the run's working buffers in a library-owned static device array of
   TPCCA_NOALLOC_ARENA_BYTES bytes on the context's GPU instead of the
   attached arena (no arena needs to be attached). The run is eager (no
   graph capture) on the context's stream; it calls no hipMalloc, hipFree or
   other allocating routine. Returns CAPACITY if the loaded frames need more
   arena than the static array holds (tpcca_required_arena gives the size;
   about 130 MB go to the per-sector tables of one frame, the rest holds
   ~78 bytes per cluster), STATE if the context's table block is too small
   (call tpcca_required_arena once beforehand), DEVICE if the array is not
   available on this GPU. Every call on a GPU, from any context, shares that
   GPU's array: calls that overlap on one GPU race, and a call's results
   (read with the fetch functions) stay valid only until the next such call
   on that GPU. A later tpcca_run switches the context back to its attached
   arena. */
#define TPCCA_NOALLOC_ARENA_BYTES ((size_t)160 << 20)
tpcca_status tpcca_run_noalloc(tpcca_ctx *ctx);

/* Wait for the last run; DEVICE on a HIP error, ABORTED if it was aborted,
   CAPACITY if a pruned run overflowed its triplet pool. */
tpcca_status tpcca_synchronize(tpcca_ctx *ctx);

/* Ask a run in flight to stop early (checked between work items). The run's
   results are then undefined and tpcca_synchronize returns ABORTED.
   (Operational control of the online farm's processing, Sec. 2; not part
   of the method.) */
tpcca_status tpcca_request_abort(tpcca_ctx *ctx);

/* Batched, graph-replayed runs over many uneven frames are this library's
   extension of the whole-frame processing of Sec. 1 (the frames the farm
   replays from memory in a loop, Sec. 2).
   Replay runs from a captured HIP graph (1) or launch kernel by kernel (0,
   the default). With graphs on, the first run after a change of frames,
   arena, configuration or launch settings captures the whole kernel sequence
   on the stream; later runs launch that graph with one call. Per-stage
   timing is not recorded in graph mode. */
tpcca_status tpcca_set_graph(tpcca_ctx *ctx, int32_t on);

/* Set by the autotuner (this library's extension; the paper only asks for
   efficient use of the GPU, Sec. 1).
   Launch shape of one kernel group (1 histogram, 3 row scatter, 4 row sort,
   5 neighbour links, 6 seeds, 7 chain walk and copy, 8 track slots,
   9 selection after the track following, 10 cluster lists and assignment,
   11 fit): blocks_per_cu persistent
   workgroups per compute unit (0: keep).
   For stage 5, param sets how many clusters a neighbour-finding tile may
   stage in LDS (256..3072, 0: keep; smaller tiles give more work items).
   For stage 4, param sets how many clusters a (row, time slab) bucket of the
   row sort may hold to be sorted in registers (1..8192, 0: keep; larger
   buckets take a two-pass path through global memory).
   Results do not depend on these settings. */
tpcca_status tpcca_set_launch(tpcca_ctx *ctx, int32_t stage, int32_t blocks_per_cu, int32_t param);

/* Measurement helper (not part of the method): copy `bytes` (a multiple of
   16) from device src to device dst with a plain streaming kernel on the
   context's stream. Its hardware-counter readings for a known size calibrate
   the HBM traffic counters of the tracker's kernels. */
tpcca_status tpcca_copy(tpcca_ctx *ctx, const void *src, void *dst, size_t bytes);

/* Enable (1) or disable (0) per-stage device timing with HIP events; either
   call also resets the accumulated stage times. (Measurement of the
   tracking throughput that sizes the farm, Sec. 2.) */
tpcca_status tpcca_set_timing(tpcca_ctx *ctx, int32_t on);

/* Figures of the last run (synchronises first). */
tpcca_status tpcca_get_stats(tpcca_ctx *ctx, tpcca_stats *out);

/* Results of the last run for one (frame, sector), copied to host memory
   (each call synchronises first). CAPACITY if cap is too small; *n_out
   always receives the number of entries available. The tracks feed the
   calibration and the compression of the synchronous phase (Sec. 1). */
tpcca_status tpcca_get_tracks(tpcca_ctx *ctx, int32_t frame, int32_t sector, tpcca_track *out, int64_t cap,
                              int64_t *n_out);

/* Input indices of the clusters of every track of the sector, track after
   track, innermost cluster first (rows ascending). (The hits attached to
   tracks, Sec. 2.) */
tpcca_status tpcca_get_track_clusters(tpcca_ctx *ctx, int32_t frame, int32_t sector, int32_t *out, int64_t cap,
                                      int64_t *n_out);

/* Track number of every input cluster of the sector (-1: none); out[n]
   with n equal to the sector's cluster count. The compression removes hits
   of tracks not used for physics by this assignment (Sec. 1). */
tpcca_status tpcca_get_assignment(tpcca_ctx *ctx, int32_t frame, int32_t sector, int32_t *out, int64_t n);

/* Collision candidates (Sec. 1: with time as the seeding coordinate,
   collisions are separated only after tracking). Every fitted track carries
   its collision time t0 in drift cm: the drift time of its helix at the
   closest approach to the beam line in the transverse plane, minus the
   250 cm drift length (for a track of one side, v_d t_coll - z_vertex on the
   A side, + z_vertex on the C side). tpcca_find_collisions works per frame
   side (A: sectors 0 .. n_sectors/2 - 1, C: the rest) of every loaded frame:
     - anchors are the tracks of at least min_clusters (>= 0) clusters with a
       finite t0 (a short track extrapolates far to the beam line, so its t0
       is coarse);
     - the anchors in ascending t0 form a new group wherever t0 jumps by more
       than gap_cm (> 0); a group's time is the mean t0 of its anchors;
     - every other track with a finite t0 joins the group of nearest time (the
       earlier on a tie) if it lies within window_cm (>= 0) of it.
   Suggested values for 50 kHz Pb-Pb frames: gap 0.5, min_clusters 60,
   window 5. Call after a run (it synchronises; its working arrays take the
   arena's slot after the chain copies, so the result holds until the next
   run, and CAPACITY if a side's anchor t0 range needs more bins (of half the
   gap) than that slot holds: raise the gap); *n_groups_out = groups over all
   frames and sides. INVALID_ARG for a bad argument, STATE before a run.
   Tracks whose fit failed have t0 = NaN and no group. */
tpcca_status tpcca_find_collisions(tpcca_ctx *ctx, float gap_cm, int32_t min_clusters, float window_cm,
                                   int64_t *n_groups_out);

/* t0 (drift cm) and group of every track of the sector, in track order
   (group: within the frame side, in ascending t0; -1 if none or before
   tpcca_find_collisions); either pointer may be null. CAPACITY if cap is
   below the track count (*n_out holds it). */
tpcca_status tpcca_get_track_times(tpcca_ctx *ctx, int32_t frame, int32_t sector, float *t0, int32_t *group,
                                   int64_t cap, int64_t *n_out);

/* The groups of one frame side (0: A, 1: C) in ascending t0: time (mean t0
   of the anchors, rounded to FP32), tracks (anchors and attached) and
   anchors; any pointer may be null. STATE before tpcca_find_collisions,
   CAPACITY if cap is below the group count (*n_out holds it). */
tpcca_status tpcca_get_collisions(tpcca_ctx *ctx, int32_t frame, int32_t side, float *t0, int32_t *n_tracks,
                                  int32_t *n_anchors, int64_t cap, int64_t *n_out);

/* Sector merging (Sec. 1: time as the seeding coordinate defers the joining
   of a particle's pieces to after the tracking). A particle crossing the
   border between two adjacent sectors of one side leaves a track in each.
   tpcca_merge_sectors pairs them, for every loaded frame:
     - eligible tracks: fit ok (status 0), at least min_clusters clusters,
       finite collision time t0 (see tpcca_find_collisions);
     - a pair (A in sector s, B in the next sector of the same side, 360 /
       (n_sectors / 2) degrees further in azimuth) with |t0_A - t0_B| <=
       window_cm is scored from A's fitted helix: B's reference point and
       direction rotated into A's frame, the point of A's circle nearest to
       B's, and there the transverse miss, the direction and time differences
       and the difference of tau, D2 = sum of their squares over the scales
       0.5 cm, 0.02 rad, 0.5 cm and 0.01;
     - a pair is merged if D2 <= d2_cut and each track is the other's best
       candidate (least D2, then least track slot).
   Suggested values: min_clusters 30, window 8, d2_cut 25. Call after a run
   (it synchronises; its working arrays take the upper half of the arena's
   slot after the chain copies, so the result holds until the next run,
   beside the collision candidates); *n_pairs_out = merged pairs.
   INVALID_ARG for a bad argument, STATE before a run or with an odd number
   of sectors. */
tpcca_status tpcca_merge_sectors(tpcca_ctx *ctx, int32_t min_clusters, float window_cm, float d2_cut,
                                 int64_t *n_pairs_out);

/* Merged partners of every track of the sector, in track order: the index
   of its partner among the tracks of the next sector (next) and of the
   previous sector (prev) of its side, -1 if none; either pointer may be
   null. STATE before tpcca_merge_sectors, CAPACITY if cap is below the
   track count (*n_out holds it). */
tpcca_status tpcca_get_merges(tpcca_ctx *ctx, int32_t frame, int32_t sector, int32_t *next, int32_t *prev,
                              int64_t cap, int64_t *n_out);

/* Membrane merging (Sec. 1, as for tpcca_merge_sectors: seeding in time
   leaves z, and so the side a track crosses to, unknown until after the
   tracking). A particle crossing z = 0 inside the drift volume leaves a
   track in sector k of the A side and one in sector k + n_sectors / 2 of
   the C side, at the same azimuth. tpcca_merge_membrane pairs them, for
   every loaded frame:
     - eligible tracks as for tpcca_merge_sectors;
     - a pair (A in sector k < n_sectors / 2, B in sector k + n_sectors / 2)
       with |t0_A - t0_B| <= window_cm (the two pieces' collision times
       differ by twice the vertex z) whose time lines t0 + tau s, s the
       transverse arc from the beam line, meet within 1 cm at an s between
       the two tracks' reference arcs widened by 5 cm (the particle crosses
       z = 0 where one piece ends and the other starts) is scored from A's
       helix at
       B's reference point: the transverse miss and the direction
       difference, and tau_A + tau_B (drift time runs against z on the A
       side and with it on the C side), D2 = sum of their squares over 0.5
       cm, 0.02 rad and 0.01;
     - a pair is merged if D2 <= d2_cut and each track is the other's best
       candidate (least D2, then least track slot).
   Suggested values: min_clusters 30, window 30, d2_cut 25. Call after a run
   (it synchronises); its working arrays follow the sector merges' in the
   arena's slot (a refit made before is dropped), so the result holds until
   the next run or sector merge. *n_pairs_out = merged pairs. INVALID_ARG
   for a bad argument, STATE before a run or with an odd number of sectors,
   CAPACITY if the working arrays do not fit. */
tpcca_status tpcca_merge_membrane(tpcca_ctx *ctx, int32_t min_clusters, float window_cm, float d2_cut,
                                  int64_t *n_pairs_out);

/* Membrane partners of every track of the sector, in track order: the index
   of its partner among the tracks of the sector on the other side at the
   same azimuth (sector +- n_sectors / 2), -1 if none; partner may be null.
   STATE before tpcca_merge_membrane, CAPACITY if cap is below the track
   count (*n_out holds it). */
tpcca_status tpcca_get_membrane_merges(tpcca_ctx *ctx, int32_t frame, int32_t sector, int32_t *partner, int64_t cap,
                                       int64_t *n_out);

/* Removal of the clusters of tracks not used for physics (Sec. 1: the
   compression of the synchronous phase drops the TPC hits of tracks not
   used for physics, using the tracking's assignment). A cluster is removed
   if its track has a successful fit (status 0) and pT below pt_min (GeV),
   i.e. |q/pT| > 1 / pt_min; clusters of no track, and of tracks whose fit
   failed, are kept. kept: device pointer (caller-owned) to cap int32
   entries; receives the kept clusters' input indices (sector-local),
   ascending, sector after sector in (frame, sector) order of the run
   (tpcca_get_removal_range gives each sector's part). *n_kept = kept
   clusters of the whole run, also when cap is too small (then nothing is
   written and CAPACITY is returned: kept may be null with cap = 0 to
   query). Synchronises. INVALID_ARG for pt_min <= 0 or a null kept with
   cap > 0, STATE before a run. */
tpcca_status tpcca_remove_clusters(tpcca_ctx *ctx, float pt_min, int32_t *kept, int64_t cap, int64_t *n_kept);

/* The sector's part of the last tpcca_remove_clusters output: its first
   entry and its count. STATE before tpcca_remove_clusters (the ranges hold
   until the next run). */
tpcca_status tpcca_get_removal_range(tpcca_ctx *ctx, int32_t frame, int32_t sector, int64_t *begin,
                                     int64_t *count);

/* Entropy reduction of the cluster properties (Sec. 1: the compression
   reduces the entropy of the hit properties before the ANS coding), as
   symbol histograms of the track clusters. Per track (clusters in rows
   ascending), coordinates quantised to 1/16 cm (y * 16 and t * 16 in FP32,
   rounded to nearest even), every cluster after the first gives five
   symbols: the row step dr_j; the first differences of y and of t; and the
   track-model residuals of y and of t: the first difference for the second
   cluster, then q_j dr_{j-1} - q_{j-1} (dr_{j-1} + dr_j) + q_{j-2} dr_j
   (dr_{j-1} times the miss of the straight-line extrapolation in row
   number). hist: host pointer to 5 x 512 int64 counts, stream after
   stream; symbol s counts in bin s + 255 if |s| <= 255, else in bin 511.
   frame = sector = -1: every track of the run; otherwise the tracks of
   that sector. Synchronises. INVALID_ARG for a null hist or an unknown
   sector, STATE before a run. */
tpcca_status tpcca_entropy_histograms(tpcca_ctx *ctx, int32_t frame, int32_t sector, int64_t *hist);

/* ANS coding of one sector's track clusters (Sec. 1: entropy compression
   with ANS after the entropy reduction): of the symbols of
   tpcca_entropy_histograms, the row step and the track-model residuals of
   y and t (streams 0, 3, 4; the first differences follow from them), coded
   per track by rANS with one 32-bit state
   (kept in [2^23, 2^31), byte renormalisation) and, per stream, a 16-bit
   frequency model from the sector's histogram: f = max(1, floor(count *
   2^16 / total)) for counted bins (the escape bin counted at least once),
   the shortfall to 2^16 added to the bin of the largest count, an excess
   taken one unit at a time from the bin of the largest frequency (lowest
   index on ties). Per track the clusters' symbols are coded last to first
   and streams 4, 3, 0, so a decoder reads cluster 2 stream 0 first; an
   escape is the escape bin followed by the value's 32 bits as two uniform
   16-bit parts (high part first in decoding order). bytes: device pointer
   (caller-owned) to cap bytes; each track's bytes are in decoding order,
   the final state first (most significant byte first). offsets: host
   pointer to n_offsets int64 (at least the sector's track count + 1), or
   null: the start of every track's bytes, then the end. *n_bytes = the
   sector's bytes, also when cap is too small (then nothing is written and
   CAPACITY is returned; bytes may be null with cap = 0 to query).
   Synchronises. INVALID_ARG for a bad pointer, STATE before a run. */
tpcca_status tpcca_ans_encode(tpcca_ctx *ctx, int32_t frame, int32_t sector, uint8_t *bytes, int64_t cap,
                              int64_t *offsets, int64_t n_offsets, int64_t *n_bytes);

/* Global refit of the merged pairs (Sec. 1: the pieces of a particle found
   in two sectors joined after the tracking; the fit is the helix fit of
   tpcca_run, Sec. 3): every pair of tpcca_merge_sectors becomes one track
   whose clusters are those of the first track (sector s) and of its partner
   (next sector), the partner's rotated by the sector angle into sector s's
   frame, ordered by increasing local x (ties: the first track's before the
   partner's, each in its own order), and fitted like a track of sector s
   with the x each cluster carries. Call after tpcca_merge_sectors (it
   synchronises); the virtual tracks take the free part of the chain-copy
   region and the arena's slot after the merge arrays, so the result holds
   until the next run or merge (sector or membrane). *n_out = pairs refitted. STATE before
   tpcca_merge_sectors, CAPACITY if the virtual tracks do not fit. */
tpcca_status tpcca_refit_merged(tpcca_ctx *ctx, int64_t *n_out);

/* Refits whose first track lies in the sector, in the order of that track:
   the fitted track (frame and sector of the first track, n_clusters of
   both, x_ref the outermost cluster's x in that sector's frame, seed the
   first track's, first not meaningful), the first track's index among the
   sector's tracks (first_track) and its partner's among the next sector's
   (partner); any pointer may be null. STATE before tpcca_refit_merged,
   CAPACITY if cap is below the count (*n_out holds it). */
tpcca_status tpcca_get_refits(tpcca_ctx *ctx, int32_t frame, int32_t sector, tpcca_track *tracks,
                              int32_t *first_track, int32_t *partner, int64_t cap, int64_t *n_out);

/* The pad-row neighbour links of the cellular-automaton seeding (Sec. 1:
   HLT-derived tracker, seeding with time as a coordinate).
   Neighbour links of every input cluster of the sector, in input indices
   (-1: none): cleaned = 0 gives the best pair of step 2, cleaned = 1 keeps
   only mutual links. For checking and debugging. */
tpcca_status tpcca_get_links(tpcca_ctx *ctx, int32_t frame, int32_t sector, int32_t cleaned, int32_t *up,
                             int32_t *dn, int64_t n);

/* ---------------------------------------------------------------------
 * Learned triplet pruning: an extension of this library, not in the paper
 * (the paper names no network; the benchmark configuration that defines it
 * is learned pruning of the neighbour triplets with a 12-64-64-1 MLP). A
 * small network (12 features -> 64 -> 64 -> 1,
 * ReLU, BF16 weights and activations, FP32 biases and accumulation) scores
 * every accepted candidate triplet (down, cluster, up) of the neighbour
 * finder; with use_mlp = 1 triplets whose logit is below
 * mlp_logit_threshold are dropped before the best pair is chosen, i.e.
 * before the cellular automaton. Without loaded weights a run falls back to
 * the plain finder (tpcca_stats.mlp_used = 0).
 *
 * Parameters are exchanged as kMlpNParam = 5313 FP32 values in this order:
 * w1[64][16] (input columns 12..15 unused), b1[64], w2[64][64], b2[64],
 * w3[64], b3. The network's state (BF16 weights, FP32 master copy, AdamW
 * moments, gradient, training workspace) lives in one caller-owned device
 * buffer of tpcca_mlp_state_bytes() bytes.
 * --------------------------------------------------------------------- */

/* Bytes of the network state buffer. */
tpcca_status tpcca_mlp_state_bytes(size_t *bytes);

/* Use [device_ptr, device_ptr + bytes) (256-byte aligned, caller-owned) as
   the network state. Its contents are (re)initialised by tpcca_mlp_load. */
tpcca_status tpcca_mlp_attach(tpcca_ctx *ctx, void *device_ptr, size_t bytes);

/* Set the parameters from host FP32 values (weights are rounded to BF16 for
   use, the FP32 values become the training master copy); resets the AdamW
   state. STATE without an attached state buffer. Synchronous. */
tpcca_status tpcca_mlp_load(tpcca_ctx *ctx, const float *params);

/* Copy the FP32 master parameters to host memory (synchronous). */
tpcca_status tpcca_mlp_fetch(tpcca_ctx *ctx, float *params);

/* Switch pruning on (use_mlp = 1) or off (0) and set the logit threshold for
   the following runs, without reloading frames (the pool is sized at the
   next run, so the arena may need to grow: check tpcca_required_arena).
   A pruned run keeps, per cluster, the best (c, up id, down id) pair among
   its gap-1 triplets whose logit is >= the threshold, and among its gap-2
   triplets only if none survives (the pruning of the cellular automaton's
   candidates by a learned network). By default the network scores the
   triplets inside the neighbour search, gap 2 only where needed, and the
   stats count the triplets scored; see tpcca_set_triplet_pool for the
   variant that lists every triplet. INVALID_ARG for use_mlp outside {0, 1}
   or a NaN threshold. */
tpcca_status tpcca_set_pruning(tpcca_ctx *ctx, int32_t use_mlp, float logit_threshold);

/* keep = 1: pruned runs write every candidate triplet of every gap, with
   its features, positions, score and logit, to a pool in the arena
   (pool_per_cluster slots per cluster; CAPACITY at tpcca_synchronize if it
   overflows), then score and select in separate kernels; the links are the
   same as without the pool. tpcca_get_triplets and tpcca_triplet_samples
   need such a run (training data, inspection). keep = 0 (default): no pool.
   Takes effect at the next run; INVALID_ARG for keep outside {0, 1}. */
tpcca_status tpcca_set_triplet_pool(tpcca_ctx *ctx, int32_t keep);

/* Logits of n triplets: x_dev = device [n][16] BF16 features (columns
   12..15 zero), z_dev = device float[n]. Enqueued on the stream. */
tpcca_status tpcca_mlp_infer(tpcca_ctx *ctx, const uint16_t *x_dev, int64_t n, float *z_dev);

/* Hyper-parameters of one AdamW step on the weighted BCE-with-logits loss
   (positive examples weighted by pos_weight). */
typedef struct {
    float lr, beta1, beta2, eps, weight_decay, pos_weight;
} tpcca_mlp_hparams;

/* Gradient of the mean weighted BCE loss over the n (<= 8192) examples
   (x_dev [n][16] BF16, y_dev float[n] in {0,1}) with respect to the
   parameters, as FP32 in the parameter order, into grad_dev (device,
   5313 floats); loss_dev (device, 1 float) receives the loss. Forward and
   backward products run on the matrix cores with BF16 operands and FP32
   accumulation. Enqueued on the stream. */
tpcca_status tpcca_mlp_grad(tpcca_ctx *ctx, const uint16_t *x_dev, const float *y_dev, int64_t n, float pos_weight,
                            float *grad_dev, float *loss_dev);

/* One AdamW step on a minibatch (same inputs as tpcca_mlp_grad): updates
   the FP32 master parameters and their BF16 copies on the device. loss_dev
   may be NULL. Enqueued on the stream. */
tpcca_status tpcca_mlp_train_step(tpcca_ctx *ctx, const uint16_t *x_dev, const float *y_dev, int64_t n,
                                  const tpcca_mlp_hparams *hp, float *loss_dev);

/* Training examples from the last pruned run that kept its triplet pool
   (all loaded frames; STATE otherwise), built on
   the device: each triplet is kept with probability `keep` (decided by a
   hash of seed, sector, input index and the triplet's rank in its cluster,
   so the subset is reproducible) and labelled 1 if the run's cleaned links
   put its down and up clusters directly below and above its middle cluster
   and that cluster is on a track, else 0. feat_dev receives [n][16] BF16
   features (16-byte aligned), label_dev n floats, in arbitrary order;
   *n_out = kept triplets (CAPACITY if above cap). Synchronous. */
tpcca_status tpcca_triplet_samples(tpcca_ctx *ctx, float keep, uint64_t seed, uint16_t *feat_dev, float *label_dev,
                                   int64_t cap, int64_t *n_out);

/* Triplets of the last pruned run that kept its triplet pool (STATE
   otherwise) for one (frame, sector), ordered by the
   input index of the middle cluster, then gap, then down and up input index:
   tri[k] = (down, cluster, up, gap) input indices, feat[k] = 16 BF16
   features, z[k] = logit (any output pointer may be NULL). CAPACITY if cap
   is too small; *n_out receives the count. Synchronous. */
tpcca_status tpcca_get_triplets(tpcca_ctx *ctx, int32_t frame, int32_t sector, int32_t *tri, uint16_t *feat,
                                float *z, int64_t cap, int64_t *n_out);

#ifdef __cplusplus
}
#endif

#endif /* TPCCA_H */
