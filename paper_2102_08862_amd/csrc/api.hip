// Host side of the C ABI declared in include/tpcca.h: context, validation,
// the arena plan (every device buffer of a run is a sub-range of the
// caller's arena; buffers that are dead after a stage are reused by later
// stages), stage orchestration on the caller's stream and result fetches.
#include <algorithm>
#include <climits>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "compress_internal.h"
#include "merge_internal.h"
#include "tpcca_internal.h"

using namespace tpcca;

namespace {

struct SectorIn {
    int64_t n = 0;
    bool loaded = false;
    bool host = false;
    const uint8_t *drow = nullptr;
    const float *dy = nullptr;
    const float *dt = nullptr;
    std::vector<uint8_t> hrow;
    std::vector<float> hy, ht;
    size_t stage_off = 0;  // arena offset of staged host inputs
};

// Arena layout of one run.
struct Layout {
    size_t total = 0;
    size_t inputs, st, cnt;
    // tables in the context's own device block (not in the arena)
    size_t si, chunk, row_x, w_tab, ycell, tab_bytes;
    size_t bcnt, bstart, bcur, coff;
    size_t tstart, ntile, tile_base, tiles, glb_tiles;
    int64_t tile_cap = 0;
    size_t tmp, rec, link, upc;
    size_t rm_bits, rm_cnt;    // cluster removal: bitmap of removed inputs, per-chunk counts
    size_t ent_hist;           // entropy reduction: symbol histograms
    size_t ans_tab, ans_size;  // rANS: frequency tables, per-track byte counts
    size_t seeds, tseed, tlen, tslot, tchoff, choff;
    size_t bits, wpre;
    size_t trk_len, trk_seed, cl_off, trk, trk_t0, trk_group, slot_bytes;
    size_t clusters, assign, scan_tmp, asg_cnt;
    size_t perm, lhist, chain, chain_bytes, xslot;
    size_t pfeat, pd, pu, pc, pz, hoff, hn1, hn2;
    int64_t pool_cap = 0;
    size_t xoff, xlen, xseed, xsi, klen, kchoff, ford, fhist, foff;
    int64_t n_fbins = 0;
    int64_t ext_cap = 0;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Bump {
    size_t off = 0;
    size_t take(size_t bytes) {
        off = align_up(off, 256);
        const size_t r = off;
        off += align_up(bytes ? bytes : 1, 256);
        return r;
    }
};

const char *kStageNames[] = {"reset", "hist",  "setup",  "scatter", "rowsort", "links",
                             "seeds", "walk",  "slots",  "follow",  "clscan", "fit"};
constexpr int kNumStages = 12;
constexpr size_t kTabBlockDefault = 1 << 20;
constexpr int kEvRing = 64;

}  // namespace

// The library-owned run arena of tpcca_run_noalloc, for callers that cannot
// allocate device memory: a static device array (each GPU the library runs
// on holds its own copy until the process ends). Host code never passes the
// array's name to a kernel or a copy: the name is a host-side stand-in; the
// device address of each GPU's copy is taken once per device with
// hipGetSymbolAddress (in tpcca_create, with that device current) and used
// everywhere instead.
static __device__ __align__(256) char scratch[TPCCA_NOALLOC_ARENA_BYTES];
constexpr int kMaxDevices = 64;
static char *g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

static hipError_t scratch_setup(int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (g_scratch[dev]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch[dev] = (char *)p;
    return e;
}

static char *scratch_of(int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (dev >= 0 && dev < kMaxDevices) ? g_scratch[dev] : nullptr;
}

struct tpcca_ctx {
    tpcca_config cfg{};
    std::vector<float> row_x;
    int device = 0;
    int n_cu = 256;
    hipStream_t stream = nullptr;
    // the cluster lists and the assignment run on a side stream beside the
    // fit (they share no buffer with it); forked and joined with events
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::vector<std::vector<SectorIn>> frames;
    char *arena = nullptr;       // arena of the current (last) run
    size_t arena_bytes = 0;
    char *user_arena = nullptr;  // the caller's arena (tpcca_attach_arena)
    size_t user_arena_bytes = 0;
    bool plan_dirty = true;
    bool upload_dirty = true;
    bool have_results = false;
    bool ran = false;
    // collision candidates of the last tpcca_find_collisions (reset by a run)
    bool coll_valid = false;
    // sector merges of the last tpcca_merge_sectors (reset by a run): arena
    // offsets of the partner arrays (upper half of the post-run scratch slot)
    bool merge_valid = false;
    size_t merge_next_off = 0, merge_prev_off = 0;
    size_t merge_end = 0;   // first free byte after the merge arrays (offset in the arena)
    bool rm_valid = false;   // cluster removal's chunk offsets (reset by a run)
    // membrane merges (reset by a run or a new sector merge)
    bool mem_valid = false;
    size_t mem_a_off = 0, mem_c_off = 0, mem_end = 0;
    // refits of the merged pairs (reset by a run or a new merge)
    bool refit_valid = false;
    size_t refit_pidx_off = 0, refit_pa_off = 0, refit_pb_off = 0, refit_trk_off = 0;
    int64_t refit_n = 0;
    std::vector<int32_t> coll_n, coll_base;   // per side: groups, first group
    size_t coll_sum_off = 0, coll_cnt_off = 0, coll_att_off = 0;   // arena offsets: sums, anchors, attached
    Layout lay;
    KArgs args{};
    std::string err;
    int32_t *abort_host = nullptr;
    int32_t *abort_dev = nullptr;
    bool timing = false;
    bool events_ok = false;
    // ring of per-run event sets, so that back-to-back timed runs need no
    // host synchronisation; completed sets are folded into the totals
    hipEvent_t ev[kEvRing][kNumStages + 1];
    bool ev_pending[kEvRing] = {};
    int ev_next = 0;
    int64_t timed_runs = 0;
    double stage_ms_total[kNumStages] = {};
    float stage_ms_last[kNumStages] = {};
    std::vector<SiDesc> si_host;
    std::vector<int32_t> chunks;
    std::vector<float> wtab;
    std::vector<YCell> ycell;
    char *tab_dev = nullptr;     // device copy of the tables (SI descriptors, chunks, row tables)
    size_t tab_cap = 0;
    int64_t n_in = 0;
    int32_t n_words = 0;
    Launch lc[kMaxStages];   // launch shapes by stage index (1 hist .. 11 fit; see tpcca_set_launch)
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    bool graph_valid = false;
    int32_t tile_budget = kTileCap;  // clusters a neighbour tile may stage
    int32_t sort_cap = kSortCap;     // clusters a row-sort bucket may hold to be sorted in registers
    char *mlp = nullptr;       // caller-owned network state buffer
    bool mlp_loaded = false;
    bool keep_pool = false;    // pruned runs list every triplet in the pool
    bool pool_run = false;     // the plan includes the triplet pool
};

static void drop_graph(tpcca_ctx *c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    c->graph_valid = false;
}

static tpcca_status fail(tpcca_ctx *c, tpcca_status s, const std::string &m) {
    if (c) c->err = m;
    return s;
}

static tpcca_status hip_fail(tpcca_ctx *c, hipError_t e, const char *what) {
    return fail(c, TPCCA_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(c, call)                                             \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) return hip_fail((c), e_, #call);      \
    } while (0)

static const float *default_row_x() {
    static float tab[152];
    static bool init = false;
    if (!init) {
        for (int r = 0; r < 152; r++) tab[r] = (float)(85.0 + r * 160.0 / 151.0);
        init = true;
    }
    return tab;
}

extern "C" {

tpcca_status tpcca_config_default(tpcca_config *out) {
    if (!out) return TPCCA_ERR_INVALID_ARG;
    tpcca_config c{};
    c.bz_tesla = 0.5f;
    c.n_sectors = 36;
    c.n_rows = 152;
    c.row_x = default_row_x();
    c.sigma_y = 0.1f;
    c.sigma_t = 0.1f;
    c.win_y = 1.5f;
    c.win_t = 2.0f;
    c.pair_c2 = 0.2f;
    c.max_gap = 2;
    c.min_track_hits = 10;
    c.prior_var_sinphi = 1.0f;
    c.prior_var_tau = 1.0f;
    c.prior_var_qpt = 100.0f;
    c.kf_passes = 12;
    c.s_max = 0.999f;
    c.use_mlp = 0;
    c.mlp_logit_threshold = 0.0f;
    c.pool_per_cluster = 4;
    c.follow = 0;
    c.follow_win_y = 1.5f;
    c.follow_win_t = 1.5f;
    c.follow_chi2 = 16.0f;
    c.follow_q = 1.0e-4f;
    c.follow_var_y = 0.01f;
    c.follow_var_t = 0.01f;
    c.follow_var_slope0 = 1.0f;
    c.follow_max_miss = 3;
    *out = c;
    return TPCCA_OK;
}

tpcca_status tpcca_create(const tpcca_config *cfg, tpcca_ctx **out) {
    if (!cfg || !out) return TPCCA_ERR_INVALID_ARG;
    *out = nullptr;
    if (cfg->n_rows < 5 || cfg->n_rows > kMaxRows || cfg->n_sectors < 1 || cfg->n_sectors > 4096 || !cfg->row_x)
        return TPCCA_ERR_INVALID_ARG;
    if (cfg->max_gap < 1 || cfg->max_gap > kMaxGap || cfg->min_track_hits < 3 || cfg->kf_passes < 1 ||
        cfg->kf_passes > 64)
        return TPCCA_ERR_INVALID_ARG;
    if (cfg->pool_per_cluster < 1 || cfg->pool_per_cluster > 64 || !std::isfinite(cfg->mlp_logit_threshold) ||
        cfg->use_mlp < 0 || cfg->use_mlp > 1)
        return TPCCA_ERR_INVALID_ARG;
    if (!(cfg->win_y > 0) || !(cfg->win_t > 0) || !(cfg->pair_c2 >= 0) || !(cfg->sigma_y > 0) ||
        !(cfg->sigma_t > 0) || !(cfg->prior_var_sinphi > 0) || !(cfg->prior_var_tau > 0) ||
        !(cfg->prior_var_qpt > 0) || !(cfg->s_max > 0 && cfg->s_max < 1) || !std::isfinite(cfg->bz_tesla))
        return TPCCA_ERR_INVALID_ARG;
    if (cfg->follow < 0 || cfg->follow > 1 || !(cfg->follow_win_y > 0) || !(cfg->follow_win_t > 0) ||
        !(cfg->follow_chi2 >= 0) || !(cfg->follow_q >= 0) || !(cfg->follow_var_y > 0) ||
        !(cfg->follow_var_t > 0) || !(cfg->follow_var_slope0 > 0) || !std::isfinite(cfg->follow_win_y) ||
        !std::isfinite(cfg->follow_win_t) || !std::isfinite(cfg->follow_chi2) || !std::isfinite(cfg->follow_q) ||
        !std::isfinite(cfg->follow_var_y) || !std::isfinite(cfg->follow_var_t) ||
        !std::isfinite(cfg->follow_var_slope0) || cfg->follow_max_miss < 1 || cfg->follow_max_miss > 255)
        return TPCCA_ERR_INVALID_ARG;
    for (int r = 0; r < cfg->n_rows; r++) {
        if (!std::isfinite(cfg->row_x[r])) return TPCCA_ERR_INVALID_ARG;
        if (r && !(cfg->row_x[r] > cfg->row_x[r - 1])) return TPCCA_ERR_INVALID_ARG;
    }
    tpcca_ctx *c = new tpcca_ctx();
    c->cfg = *cfg;
    c->row_x.assign(cfg->row_x, cfg->row_x + cfg->n_rows);
    c->cfg.row_x = c->row_x.data();
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->abort_host, sizeof(int32_t), hipHostMallocMapped);
    if (e == hipSuccess) {
        *c->abort_host = 0;
        e = hipHostGetDevicePointer((void **)&c->abort_dev, c->abort_host, 0);
    }
    if (e != hipSuccess) {
        if (c->abort_host) (void)hipHostFree(c->abort_host);
        delete c;
        return TPCCA_ERR_DEVICE;
    }
    // the per-run tables (sector descriptors, chunk list, row tables) live in
    // a small device block of the context; 1 MiB holds those of about 1e9
    // clusters in ~100 frames, and only tpcca_required_arena grows it
    c->tab_cap = kTabBlockDefault;
    if (hipMalloc((void **)&c->tab_dev, c->tab_cap) != hipSuccess) {
        (void)hipHostFree(c->abort_host);
        delete c;
        return TPCCA_ERR_DEVICE;
    }
    // the no-allocation entry point's arena on this device (a failure only
    // disables that entry point)
    (void)scratch_setup(c->device);
    c->events_ok = true;
    for (int r = 0; r < kEvRing; r++)
        for (int i = 0; i <= kNumStages; i++)
            if (hipEventCreate(&c->ev[r][i]) != hipSuccess) c->events_ok = false;
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
        tpcca_destroy(c);
        return TPCCA_ERR_DEVICE;
    }
    const int cu = std::max(1, c->n_cu);
    for (int i = 0; i < kMaxStages; i++) c->lc[i] = Launch{cu * 8, 256};
    c->lc[3] = Launch{cu, 1024};      // scatter: 134 KB LDS, 1024 threads
    c->lc[4] = Launch{cu * 4, 1024};  // rowsort: 36 KB LDS, 1024 threads
    c->lc[5] = Launch{cu * 4, 256};  // links: 34 KB LDS -> 4 resident blocks per CU
    // decision-path constants, computed once on the host in FP32
    c->wtab.assign((size_t)cfg->n_rows * kMaxGap, 0.f);
    for (int r = 0; r < cfg->n_rows; r++)
        for (int g = 1; g <= kMaxGap; g++) {
            if (r - g < 0 || r + g >= cfg->n_rows) continue;
            volatile float num = c->row_x[r] - c->row_x[r - g];
            volatile float den = c->row_x[r + g] - c->row_x[r - g];
            volatile float w = num / den;
            c->wtab[(size_t)r * kMaxGap + g - 1] = w;
        }
    // y cells of the row order: about 2*win_y wide across the sector's width
    // at the row (clusters outside are clamped to the edge cells)
    c->ycell.assign((size_t)cfg->n_rows, YCell{0.f, 0.f, 1, 0});
    for (int r = 0; r < cfg->n_rows; r++) {
        const double half_angle = cfg->n_sectors >= 6 ? 2.0 * M_PI / cfg->n_sectors : 0.0;
        const double hw = std::fabs((double)c->row_x[r]) * std::tan(half_angle) + 2.0 * cfg->win_y;
        int ny = (int)std::floor(2.0 * hw / (2.0 * cfg->win_y));
        ny = std::min(std::max(ny, 1), kMaxYCells);
        YCell &yc = c->ycell[r];
        yc.ylo = (float)(-hw);
        yc.inv = (float)(ny / (2.0 * hw));
        yc.ny = ny;
    }
    *out = c;
    return TPCCA_OK;
}

void tpcca_destroy(tpcca_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->events_ok)
        for (int r = 0; r < kEvRing; r++)
            for (int i = 0; i <= kNumStages; i++) (void)hipEventDestroy(c->ev[r][i]);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamDestroy(c->side);
    }
    for (hipEvent_t e : {c->ev_fork, c->ev_join})
        if (e) (void)hipEventDestroy(e);
    if (c->abort_host) (void)hipHostFree(c->abort_host);
    if (c->tab_dev) (void)hipFree(c->tab_dev);
    delete c;
}

const char *tpcca_last_error(const tpcca_ctx *c) {
    if (!c) return "null context";
    return c->err.c_str();
}

tpcca_status tpcca_set_stream(tpcca_ctx *c, void *stream) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    c->stream = (hipStream_t)stream;
    return TPCCA_OK;
}

tpcca_status tpcca_set_timing(tpcca_ctx *c, int32_t on) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    if (on && !c->events_ok) return fail(c, TPCCA_ERR_DEVICE, "HIP events unavailable");
    (void)hipStreamSynchronize(c->stream);
    c->timing = on != 0;
    for (int r = 0; r < kEvRing; r++) c->ev_pending[r] = false;
    c->timed_runs = 0;
    for (int i = 0; i < kNumStages; i++) {
        c->stage_ms_total[i] = 0.0;
        c->stage_ms_last[i] = 0.f;
    }
    return TPCCA_OK;
}

tpcca_status tpcca_set_graph(tpcca_ctx *c, int32_t on) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(c->stream);
    c->use_graph = on != 0;
    drop_graph(c);
    return TPCCA_OK;
}

tpcca_status tpcca_set_launch(tpcca_ctx *c, int32_t stage, int32_t blocks_per_cu, int32_t param) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    static const int tunable[] = {1, 3, 4, 5, 6, 7, 8, 9, 10, 11};
    bool ok = false;
    for (int v : tunable) ok = ok || v == stage;
    if (!ok || blocks_per_cu < 0 || blocks_per_cu > 64) return fail(c, TPCCA_ERR_INVALID_ARG, "bad stage or blocks");
    if (param != 0 && !((stage == 5 && param >= 256 && param <= kTileCap) || (stage == 4 && param >= 1 && param <= kSortCap)))
        return fail(c, TPCCA_ERR_INVALID_ARG, "bad param");
    if (stage == 4 && blocks_per_cu > 4) return fail(c, TPCCA_ERR_INVALID_ARG, "rowsort: at most 4 blocks per CU");
    if (stage == 3 && blocks_per_cu > 4) return fail(c, TPCCA_ERR_INVALID_ARG, "scatter: at most 4 blocks per CU");
    if (stage == 5 && blocks_per_cu > 4) return fail(c, TPCCA_ERR_INVALID_ARG, "links: at most 4 blocks per CU");
    (void)hipStreamSynchronize(c->stream);
    if (blocks_per_cu) c->lc[stage].grid = std::max(1, c->n_cu) * blocks_per_cu;
    if (param && stage == 5) c->tile_budget = param;
    if (param && stage == 4) c->sort_cap = param;
    c->plan_dirty = true;  // the tile budget and the sort capacity are kernel arguments
    c->graph_valid = false;
    return TPCCA_OK;
}

tpcca_status tpcca_set_pruning(tpcca_ctx *c, int32_t use_mlp, float theta) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    if ((use_mlp != 0 && use_mlp != 1) || std::isnan(theta))
        return fail(c, TPCCA_ERR_INVALID_ARG, "use_mlp must be 0 or 1 and the threshold a number");
    (void)hipStreamSynchronize(c->stream);
    c->cfg.use_mlp = use_mlp;
    c->cfg.mlp_logit_threshold = theta;
    c->plan_dirty = true;  // pool size and threshold are part of the plan
    c->graph_valid = false;
    c->have_results = false;
    return TPCCA_OK;
}

tpcca_status tpcca_set_triplet_pool(tpcca_ctx *c, int32_t keep) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    if (keep != 0 && keep != 1) return fail(c, TPCCA_ERR_INVALID_ARG, "keep must be 0 or 1");
    (void)hipStreamSynchronize(c->stream);
    c->keep_pool = keep != 0;
    c->plan_dirty = true;  // the pool is part of the plan
    c->graph_valid = false;
    c->have_results = false;
    return TPCCA_OK;
}

tpcca_status tpcca_add_frame(tpcca_ctx *c, int32_t *frame_id) {
    if (!c || !frame_id) return TPCCA_ERR_INVALID_ARG;
    c->frames.emplace_back((size_t)c->cfg.n_sectors);
    *frame_id = (int32_t)c->frames.size() - 1;
    c->plan_dirty = true;
    c->graph_valid = false;
    c->have_results = false;
    return TPCCA_OK;
}

tpcca_status tpcca_clear_frames(tpcca_ctx *c) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(c->stream);
    c->frames.clear();
    c->plan_dirty = true;
    c->graph_valid = false;
    c->have_results = false;
    return TPCCA_OK;
}

tpcca_status tpcca_load_sector(tpcca_ctx *c, int32_t frame, int32_t sector, int64_t n, const uint8_t *row,
                               const float *y, const float *t, int32_t is_device_ptr) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    if (frame < 0 || frame >= (int32_t)c->frames.size())
        return fail(c, TPCCA_ERR_INVALID_ARG, "frame index out of range");
    if (sector < 0 || sector >= c->cfg.n_sectors) return fail(c, TPCCA_ERR_INVALID_ARG, "sector out of range");
    if (n < 0 || n > (int64_t)0x3fffffff) return fail(c, TPCCA_ERR_INVALID_ARG, "cluster count out of range");
    if (n > 0 && (!row || !y || !t)) return fail(c, TPCCA_ERR_INVALID_ARG, "null input array");
    SectorIn &s = c->frames[frame][sector];
    if (s.loaded) return fail(c, TPCCA_ERR_STATE, "sector already loaded for this frame");
    s = SectorIn();
    s.n = n;
    s.loaded = true;
    if (is_device_ptr) {
        s.host = false;
        s.drow = row;
        s.dy = y;
        s.dt = t;
    } else {
        for (int64_t i = 0; i < n; i++) {
            if (row[i] >= c->cfg.n_rows || !std::isfinite(y[i]) || !std::isfinite(t[i])) {
                s = SectorIn();
                return fail(c, TPCCA_ERR_INVALID_ARG,
                            "cluster " + std::to_string(i) + ": row out of range or non-finite value");
            }
        }
        s.host = true;
        s.hrow.assign(row, row + n);
        s.hy.assign(y, y + n);
        s.ht.assign(t, t + n);
    }
    c->plan_dirty = true;
    c->graph_valid = false;
    c->have_results = false;
    return TPCCA_OK;
}

}  // extern "C"

// Compute the arena layout and the host tables of the current frames. The
// per-context table block is (re)allocated only when may_alloc is set (the
// sizing call); a run whose tables no longer fit fails instead.
static tpcca_status plan(tpcca_ctx *c, bool may_alloc) {
    const int R = c->cfg.n_rows;
    const int NS = c->cfg.n_sectors;
    const int S = (int)c->frames.size() * NS;
    int64_t N = 0, W = 0, host_bytes = 0;
    c->si_host.assign((size_t)S, SiDesc{});
    c->chunks.clear();
    Bump b;
    Layout &L = c->lay;
    // staged host inputs first
    L.inputs = b.take(0);
    for (int f = 0; f < (int)c->frames.size(); f++)
        for (int s = 0; s < NS; s++) {
            SectorIn &x = c->frames[f][s];
            if (x.loaded && x.host && x.n > 0) {
                x.stage_off = b.take((size_t)x.n);
                b.take((size_t)x.n * 4);
                b.take((size_t)x.n * 4);
                host_bytes += x.n * 9;
            }
        }
    for (int f = 0; f < (int)c->frames.size(); f++)
        for (int s = 0; s < NS; s++) {
            const int si = f * NS + s;
            const SectorIn &x = c->frames[f][s];
            SiDesc &d = c->si_host[si];
            d.n = x.loaded ? (int32_t)x.n : 0;
            d.in_base = (int32_t)N;
            d.frame = f;
            d.sector = s;
            d.word_base = (int32_t)W;
            d.nwords = (d.n + 31) / 32;
            N += d.n;
            W += d.nwords;
            for (int64_t st = 0; st < d.n; st += kChunk) {
                c->chunks.push_back(si);
                c->chunks.push_back((int32_t)st);
            }
        }
    if (N > (int64_t)0x7fff0000 || W > (int64_t)0x7fff0000)
        return fail(c, TPCCA_ERR_INVALID_ARG, "too many clusters in one run");
    const int64_t seed_cap = N / 2 + 64;
    const int64_t tseed_cap = N / std::max(2, c->cfg.min_track_hits) + 64;
    const int64_t trk_cap = tseed_cap;
    // the chain copies: one run of a multiple of 4 entries per track
    const int64_t chain_cap = N + 3 * trk_cap;
    // every device buffer is indexed with 32-bit positions: the chain copies
    // hold up to N + 3 * trk_cap entries and the assignment buckets N rounded
    // up to a bucket plus one bucket; both must stay below 2^31
    if (chain_cap + 8 > (int64_t)INT32_MAX || (N / 16384 + 2) * (int64_t)16384 > (int64_t)INT32_MAX)
        return fail(c, TPCCA_ERR_INVALID_ARG,
                    "too many clusters in one run for 32-bit positions (" + std::to_string(N) + ")");
    const int64_t SR = (int64_t)S * R;
    {
        Bump t;
        L.si = t.take(sizeof(SiDesc) * S);
        L.chunk = t.take(sizeof(int32_t) * c->chunks.size());
        L.row_x = t.take(sizeof(float) * R);
        L.w_tab = t.take(sizeof(float) * R * kMaxGap);
        L.ycell = t.take(sizeof(YCell) * R);
        L.tab_bytes = t.off;
        if (L.tab_bytes > c->tab_cap) {
            if (!may_alloc)
                return fail(c, TPCCA_ERR_STATE,
                            "the loaded frames need a larger table block: call tpcca_required_arena before tpcca_run");
            (void)hipStreamSynchronize(c->stream);
            if (c->tab_dev) (void)hipFree(c->tab_dev);
            c->tab_dev = nullptr;
            c->tab_cap = 0;
            if (hipMalloc((void **)&c->tab_dev, L.tab_bytes) != hipSuccess)
                return fail(c, TPCCA_ERR_NOMEM, "device tables");
            c->tab_cap = L.tab_bytes;
        }
    }
    L.st = b.take(sizeof(SiState) * S);
    L.cnt = b.take(sizeof(Counters));
    L.bcnt = b.take(sizeof(int32_t) * SR * kNSlabMax);
    L.bstart = b.take(sizeof(int32_t) * SR * kNSlabMax);
    L.bcur = b.take(sizeof(int32_t) * SR * kNSlabMax);
    L.coff = b.take(sizeof(int32_t) * SR * (kNcbMax + 1));
    const int nrb = (R + kTileRows - 1) / kTileRows;
    const int64_t NW = (int64_t)S * nrb;
    L.tstart = b.take(sizeof(int16_t) * NW * kNcbMax);
    L.ntile = b.take(sizeof(int32_t) * (NW + 1));
    L.tile_base = b.take(sizeof(int32_t) * (NW + 1));
    // a (sector instance, row block) has at most one tile per coarse bin
    L.tile_cap = NW * kNcbMax;
    if (L.tile_cap > (int64_t)0x7fff0000) return fail(c, TPCCA_ERR_INVALID_ARG, "too many sectors in one run");
    L.tiles = b.take(sizeof(int2) * L.tile_cap);
    L.glb_tiles = b.take(sizeof(int32_t) * L.tile_cap);
    // Scratch region reused across the sequential steps:
    //   scatter -> row sort:        tmp, the row-grouped records (16 B/cluster)
    //   seeds -> walk:              cleaned up links and the seed list (slot)
    //   walk -> fit:                the chain copies
    //   lists -> assignment (side): the (input, track) pairs per bucket (slot)
    // tmp and the chain copies share the region's start (tmp is dead after
    // the row sort, before the walk writes the copies); the slot after the
    // chain copies holds the cleaned links and seeds, then the pairs.
    L.chain_bytes = sizeof(Rec) * (size_t)chain_cap;
    const size_t slot_bytes = std::max(align_up(sizeof(int32_t) * (size_t)N, 256) + sizeof(int32_t) * (size_t)seed_cap,
                                       sizeof(int2) * (size_t)(N + 2 * 16384));
    L.chain = b.take(L.chain_bytes + 256 + slot_bytes);
    L.tmp = L.chain;
    L.xslot = L.chain + align_up(L.chain_bytes, 256);
    L.upc = L.xslot;
    L.seeds = L.xslot + align_up(sizeof(int32_t) * (size_t)N, 256);
    L.rec = b.take(sizeof(Rec) * N);
    L.link = b.take(sizeof(int2) * N);
    L.tseed = b.take(sizeof(int32_t) * tseed_cap);
    L.tlen = b.take(sizeof(int32_t) * tseed_cap);
    L.tslot = b.take(sizeof(int32_t) * tseed_cap);
    L.tchoff = b.take(sizeof(int32_t) * tseed_cap);
    L.bits = b.take(sizeof(uint32_t) * (W + 1));
    L.wpre = b.take(sizeof(int32_t) * (W + 1));
    L.trk_len = b.take(sizeof(int32_t) * (trk_cap + 1));
    L.trk_seed = b.take(sizeof(int32_t) * trk_cap);
    L.cl_off = b.take(sizeof(int32_t) * (trk_cap + 1));
    L.trk = b.take(sizeof(tpcca_track) * trk_cap);
    L.trk_t0 = b.take(sizeof(float) * trk_cap);
    L.trk_group = b.take(sizeof(int32_t) * trk_cap);
    L.slot_bytes = slot_bytes;
    L.choff = b.take(sizeof(int32_t) * trk_cap);
    L.perm = b.take(sizeof(int32_t) * trk_cap);
    L.lhist = b.take(sizeof(int32_t) * (kLenBins + 1));
    L.clusters = b.take(sizeof(int32_t) * N);
    L.assign = b.take(sizeof(int32_t) * N);
    L.asg_cnt = b.take(sizeof(int32_t) * (N / 16384 + 2));
    L.rm_bits = b.take(sizeof(uint32_t) * (size_t)(N / 32 + 2));
    L.rm_cnt = b.take(sizeof(int32_t) * (c->chunks.size() / 2 + 1));
    L.ent_hist = b.take(sizeof(int32_t) * kEntStreams * kEntBins);
    L.ans_tab = b.take(2 * sizeof(uint32_t) * kEntStreams * kEntBins);
    L.ans_size = b.take(sizeof(int32_t) * (size_t)(trk_cap + 1));
    c->pool_run = c->cfg.use_mlp != 0 && c->keep_pool;
    // every workgroup of the neighbour search may leave up to one partly used
    // chunk of the pool behind
    L.pool_cap = c->pool_run ? (int64_t)c->cfg.pool_per_cluster * N + (int64_t)(c->lc[5].grid + 1) * kPoolChunk : 0;
    if (L.pool_cap > (int64_t)0x7fff0000) L.pool_cap = 0x7fff0000;
    L.pfeat = b.take(sizeof(uint16_t) * kMlpInP * L.pool_cap);
    L.pd = b.take(sizeof(int32_t) * L.pool_cap);
    L.pu = b.take(sizeof(int32_t) * L.pool_cap);
    L.pc = b.take(sizeof(float) * L.pool_cap);
    L.pz = b.take(sizeof(float) * L.pool_cap);
    L.hoff = b.take(c->pool_run ? sizeof(int32_t) * N : 0);
    L.hn1 = b.take(c->pool_run ? sizeof(int32_t) * N : 0);
    L.hn2 = b.take(c->pool_run ? sizeof(int32_t) * N : 0);
    // track following: the per-chain figures; the extended tracks take the
    // slot after the chain copies (dead between the walk and the lists) and
    // the claims the assignment (written afterwards)
    const bool fol = c->cfg.follow != 0;
    if (fol) {
        for (int si = 0; si < S; si++)
            if (c->si_host[si].n >= (1 << 24))
                return fail(c, TPCCA_ERR_INVALID_ARG, "track following needs sectors of fewer than 2^24 clusters");
    }
    L.xoff = b.take(fol ? sizeof(int32_t) * 2 * tseed_cap : 0);
    L.xlen = b.take(fol ? sizeof(int32_t) * 2 * tseed_cap : 0);
    L.xseed = b.take(fol ? sizeof(int32_t) * tseed_cap : 0);
    L.xsi = b.take(fol ? sizeof(int32_t) * tseed_cap : 0);
    L.klen = b.take(fol ? sizeof(int32_t) * tseed_cap : 0);
    L.kchoff = b.take(fol ? sizeof(int32_t) * tseed_cap : 0);
    L.ford = b.take(fol ? sizeof(int32_t) * tseed_cap : 0);
    L.foff = b.take(fol ? sizeof(uint32_t) * SR * kNcbMax : 0);
    L.n_fbins = fol ? (int64_t)S * (kNcbMax / 8) : 0;
    L.fhist = b.take(fol ? sizeof(int32_t) * 2 * (L.n_fbins + 1) : 0);
    L.ext_cap = fol ? std::min<int64_t>((int64_t)(slot_bytes / sizeof(int32_t)), INT32_MAX - 1024) : 0;
    const int64_t nblk =
        (std::max<int64_t>(std::max<int64_t>(std::max<int64_t>(W, trk_cap), NW), L.n_fbins) + kScanItems - 1) /
            kScanItems +
        2;
    L.scan_tmp = b.take(sizeof(int32_t) * nblk);
    L.total = align_up(b.off, 256);
    c->n_in = N;
    c->n_words = (int32_t)W;

    KArgs &a = c->args;
    a = KArgs{};
    a.n_si = S;
    a.n_rows = R;
    a.n_in = (int32_t)N;
    a.n_chunks = (int32_t)(c->chunks.size() / 2);
    a.n_words = (int32_t)W;
    a.seed_cap = (int32_t)seed_cap;
    a.tseed_cap = (int32_t)tseed_cap;
    a.chain_cap = chain_cap;
    a.trk_cap = (int32_t)trk_cap;
    a.max_gap = c->cfg.max_gap;
    a.n_rb = nrb;
    // the pruned search without the pool stages smaller tiles
    a.tile_budget = std::min(c->tile_budget, (c->cfg.use_mlp && !c->keep_pool) ? kPrCap : kTileCap);
    a.sort_cap = c->sort_cap;
    a.tile_cap = (int32_t)L.tile_cap;
    a.min_track_hits = c->cfg.min_track_hits;
    a.kf_passes = c->cfg.kf_passes;
    for (int g = 1; g <= kMaxGap; g++) {
        volatile float gy = (float)g * c->cfg.win_y;
        volatile float gt = (float)g * c->cfg.win_t;
        a.win_y[g - 1] = gy;
        a.win_t[g - 1] = gt;
    }
    a.pair_c2 = c->cfg.pair_c2;
    // a coarse bin must be at least the widest time window (half width
    // max_gap * win_t) twice over, so that every candidate of a cluster lies
    // in its own or an adjacent bin with room for the predicates' slack
    a.cbw_min = std::max(8.0f, 2.0f * (float)c->cfg.max_gap * c->cfg.win_t);
    a.bz_kb = (float)(2.99792458e-3 * (double)c->cfg.bz_tesla);
    a.sigma_y2 = c->cfg.sigma_y * c->cfg.sigma_y;
    a.sigma_t2 = c->cfg.sigma_t * c->cfg.sigma_t;
    a.var_s = c->cfg.prior_var_sinphi;
    a.var_tau = c->cfg.prior_var_tau;
    a.var_k = c->cfg.prior_var_qpt;
    a.s_max = c->cfg.s_max;
    a.follow = fol ? 1 : 0;
    a.f_win_y = c->cfg.follow_win_y;
    a.f_win_t = c->cfg.follow_win_t;
    a.f_chi2 = c->cfg.follow_chi2;
    a.f_q = c->cfg.follow_q;
    a.f_var_y = c->cfg.follow_var_y;
    a.f_var_t = c->cfg.follow_var_t;
    a.f_var_s0 = c->cfg.follow_var_slope0;
    a.f_max_miss = c->cfg.follow_max_miss;
    a.ext_cap = L.ext_cap;
    a.n_fbins = (int32_t)L.n_fbins;
    a.theta = c->cfg.mlp_logit_threshold;
    {
        volatile float c2 = c->cfg.pair_c2;
        a.c2s = sqrtf(c2);
    }
    a.pool_cap = (int32_t)L.pool_cap;
    (void)host_bytes;
    c->plan_dirty = false;
    c->upload_dirty = true;
    return TPCCA_OK;
}

static void bind_pointers(tpcca_ctx *c) {
    KArgs &a = c->args;
    const Layout &L = c->lay;
    char *A = c->arena;
    char *D = c->tab_dev;
    a.row_x = (const float *)(D + L.row_x);
    a.w_tab = (const float *)(D + L.w_tab);
    a.ycell = (const YCell *)(D + L.ycell);
    a.tstart = (int16_t *)(A + L.tstart);
    a.ntile = (int32_t *)(A + L.ntile);
    a.tile_base = (int32_t *)(A + L.tile_base);
    a.tiles = (int2 *)(A + L.tiles);
    a.glb_tiles = (int32_t *)(A + L.glb_tiles);
    a.si = (const SiDesc *)(D + L.si);
    a.st = (SiState *)(A + L.st);
    a.cnt = (Counters *)(A + L.cnt);
    a.chunk = (const int32_t *)(D + L.chunk);
    a.bcnt = (int32_t *)(A + L.bcnt);
    a.bstart = (int32_t *)(A + L.bstart);
    a.bcur = (int32_t *)(A + L.bcur);
    a.coff = (int32_t *)(A + L.coff);
    a.tmp = (Rec *)(A + L.tmp);
    a.rec = (Rec *)(A + L.rec);
    a.link = (int2 *)(A + L.link);
    a.upc = (int32_t *)(A + L.upc);
    a.seeds = (int32_t *)(A + L.seeds);
    a.tseed = (int32_t *)(A + L.tseed);
    a.tlen = (int32_t *)(A + L.tlen);
    a.tslot = (int32_t *)(A + L.tslot);
    a.tchoff = (int32_t *)(A + L.tchoff);
    a.bits = (uint32_t *)(A + L.bits);
    a.wpre = (int32_t *)(A + L.wpre);
    a.trk_len = (int32_t *)(A + L.trk_len);
    a.trk_seed = (int32_t *)(A + L.trk_seed);
    a.cl_off = (int32_t *)(A + L.cl_off);
    a.trk = (tpcca_track *)(A + L.trk);
    a.trk_t0 = (float *)(A + L.trk_t0);
    a.clusters = (int32_t *)(A + L.clusters);
    a.choff = (int32_t *)(A + L.choff);
    a.perm = (int32_t *)(A + L.perm);
    a.lhist = (int32_t *)(A + L.lhist);
    a.chain = (Rec *)(A + L.chain);
    a.assign = (int32_t *)(A + L.assign);
    a.asg_pairs = (int2 *)(A + L.xslot);
    a.asg_cnt = (int32_t *)(A + L.asg_cnt);
    a.scan_tmp = (int32_t *)(A + L.scan_tmp);
    a.abort_flag = c->abort_dev;
    a.pfeat = (uint16_t *)(A + L.pfeat);
    a.pd = (int32_t *)(A + L.pd);
    a.pu = (int32_t *)(A + L.pu);
    a.pc = (float *)(A + L.pc);
    a.pz = (float *)(A + L.pz);
    a.hoff = (int32_t *)(A + L.hoff);
    a.hn1 = (int32_t *)(A + L.hn1);
    a.hn2 = (int32_t *)(A + L.hn2);
    a.ext = (int32_t *)(A + L.xslot);
    a.xoff = (int32_t *)(A + L.xoff);
    a.xlen = (int32_t *)(A + L.xlen);
    a.xseed = (int32_t *)(A + L.xseed);
    a.xsi = (int32_t *)(A + L.xsi);
    a.klen = (int32_t *)(A + L.klen);
    a.kchoff = (int32_t *)(A + L.kchoff);
    a.ford = (int32_t *)(A + L.ford);
    a.foff = c->cfg.follow ? (uint32_t *)(A + L.foff) : nullptr;
    a.fhist = (int32_t *)(A + L.fhist);
    a.use_mlp = (c->cfg.use_mlp && c->mlp_loaded) ? 1 : 0;
    a.keep_pool = (a.use_mlp && c->pool_run) ? 1 : 0;
    if (c->mlp) {
        a.mlp.w1 = (const uint16_t *)(c->mlp + MlpState::w1);
        a.mlp.w2 = (const uint16_t *)(c->mlp + MlpState::w2);
        a.mlp.w3 = (const uint16_t *)(c->mlp + MlpState::w3);
        a.mlp.b1 = (const float *)(c->mlp + MlpState::b1);
        a.mlp.b2 = (const float *)(c->mlp + MlpState::b2);
        a.mlp.b3 = (const float *)(c->mlp + MlpState::b3);
    }
}

// Enqueue the kernels of one run on s (events into ring slot `slot` if tm).
static void enqueue_run(tpcca_ctx *c, hipStream_t s, bool tm, int slot) {
    const KArgs &a = c->args;
    const Layout &L = c->lay;
    char *A = c->arena;
    Counters *cnt = (Counters *)(A + L.cnt);
    int st = 0;
    auto mark = [&](int i) {
        if (tm) (void)hipEventRecord(c->ev[slot][i], s);
    };
    mark(st++);
    // reset: row counts, bitmap, assignment (fill kernels: graph-safe)
    launch_fill_i32(a.bcnt, (int64_t)a.n_si * a.n_rows * kNSlabMax, 0, s);
    launch_fill_i32((int32_t *)a.bits, (int64_t)a.n_words + 1, 0, s);
    launch_fill_i32(a.asg_cnt, (int64_t)a.n_in / 16384 + 2, 0, s);
    mark(st++);
    launch_grid_hist(a, c->lc[1], s);  // also resets per-sector state and counters
    mark(st++);
    launch_grid_setup(a, s);
    mark(st++);
    launch_grid_scatter(a, c->lc[3], s);
    mark(st++);
    launch_grid_rowsort(a, c->lc[4], s);
    launch_tiles(a, s);  // tile partition of the neighbour search (part of the search grid)
    mark(st++);
    if (a.use_mlp && a.keep_pool) {
        launch_links_enum(a, c->lc[5], s);
        launch_mlp_infer(a.mlp, a.pfeat, &cnt->pool_next, a.pool_cap, a.pz, c->n_cu * 8, s);
        launch_select(a, c->lc[6], s);
    } else if (a.use_mlp) {
        launch_links_prune(a, c->lc[5], s);
    } else {
        launch_links(a, c->lc[5], s);
    }
    mark(st++);
    launch_seeds(a, c->lc[6], s);
    mark(st++);
    launch_walk(a, c->lc[7], s);
    mark(st++);
    launch_scan_popc(a.bits, a.n_words, a.wpre, &cnt->n_tracks, a.scan_tmp, s);
    launch_track_slots(a, c->lc[8], s);
    launch_si_tracks(a, s);
    mark(st++);
    if (a.follow) {
        // claims go into the assignment (rebuilt whole by the lists)
        launch_fill_i32(a.assign, a.n_in, 0, s);
        launch_fill_i32(a.fhist, a.n_fbins + 1, 0, s);
        launch_follow(a, c->lc[9], s);
        // keep flags (in trk_len by chain track number) -> new track numbers
        launch_scan_i32_dev(a.trk_len, &cnt->n_chains, a.trk_cap, a.cl_off, &cnt->n_tracks, a.scan_tmp, s);
        launch_follow_slots(a, c->lc[9], s);
    }
    mark(st++);
    launch_scan_i32_dev(a.trk_len, &cnt->n_tracks, a.trk_cap, a.cl_off, &cnt->n_cl, a.scan_tmp, s);
    launch_si_clusters(a, s);
    mark(st++);
    // side stream: the cluster lists and the assignment, beside the length
    // order and the fit on the main stream (they share no buffer)
    (void)hipEventRecord(c->ev_fork, s);
    (void)hipStreamWaitEvent(c->side, c->ev_fork, 0);
    launch_lists(a, c->lc[10], c->side);
    (void)hipEventRecord(c->ev_join, c->side);
    launch_len_sort(a, c->lc[11], s);
    launch_fit(a, c->lc[11], s);
    (void)hipStreamWaitEvent(s, c->ev_join, 0);   // join
    mark(st++);
}

// Fold one completed ring slot into the totals (waits for its last event).
static void fold_slot(tpcca_ctx *c, int r) {
    if (!c->ev_pending[r]) return;
    (void)hipEventSynchronize(c->ev[r][kNumStages]);
    for (int i = 0; i < kNumStages; i++) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev[r][i], c->ev[r][i + 1]) != hipSuccess) ms = 0.f;
        c->stage_ms_total[i] += ms;
        c->stage_ms_last[i] = ms;
    }
    c->timed_runs++;
    c->ev_pending[r] = false;
}

extern "C" {

tpcca_status tpcca_required_arena(tpcca_ctx *c, size_t *bytes) {
    if (!c || !bytes) return TPCCA_ERR_INVALID_ARG;
    if (c->plan_dirty || c->lay.tab_bytes > c->tab_cap) {
        tpcca_status s = plan(c, true);
        if (s != TPCCA_OK) return s;
    }
    *bytes = c->lay.total;
    return TPCCA_OK;
}

tpcca_status tpcca_attach_arena(tpcca_ctx *c, void *ptr, size_t bytes) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    if (ptr && ((uintptr_t)ptr & 255)) return fail(c, TPCCA_ERR_INVALID_ARG, "arena must be 256-byte aligned");
    (void)hipStreamSynchronize(c->stream);
    c->arena = c->user_arena = (char *)ptr;
    c->arena_bytes = c->user_arena_bytes = ptr ? bytes : 0;
    c->upload_dirty = true;
    c->graph_valid = false;
    c->have_results = false;
    return TPCCA_OK;
}

tpcca_status tpcca_request_abort(tpcca_ctx *c) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    __atomic_store_n(c->abort_host, 1, __ATOMIC_SEQ_CST);
    return TPCCA_OK;
}

}  // extern "C"

// Make `ptr` the arena of the next run (a change of arena re-uploads the
// tables and staged inputs and drops a captured graph).
static void use_arena(tpcca_ctx *c, char *ptr, size_t bytes) {
    if (c->arena != ptr) {
        c->upload_dirty = true;
        c->graph_valid = false;
    }
    c->arena = ptr;
    c->arena_bytes = bytes;
}

static tpcca_status run_on_arena(tpcca_ctx *c, bool graphs);

extern "C" {

tpcca_status tpcca_run(tpcca_ctx *c) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    if (c->frames.empty()) return fail(c, TPCCA_ERR_STATE, "no frame loaded");
    if (c->plan_dirty) {
        tpcca_status s = plan(c, false);
        if (s != TPCCA_OK) return s;
    }
    use_arena(c, c->user_arena, c->user_arena_bytes);
    if (!c->arena || c->arena_bytes < c->lay.total)
        return fail(c, TPCCA_ERR_NOMEM, "arena of " + std::to_string(c->arena_bytes) + " bytes, run needs " +
                                            std::to_string(c->lay.total));
    return run_on_arena(c, c->use_graph);
}

tpcca_status tpcca_run_noalloc(tpcca_ctx *c) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    if (c->frames.empty()) return fail(c, TPCCA_ERR_STATE, "no frame loaded");
    char *A = scratch_of(c->device);
    if (!A) return fail(c, TPCCA_ERR_DEVICE, "the static run arena of this device is unavailable");
    if (c->plan_dirty) {
        tpcca_status s = plan(c, false);
        if (s != TPCCA_OK) return s;
    }
    if (c->lay.total > TPCCA_NOALLOC_ARENA_BYTES)
        return fail(c, TPCCA_ERR_CAPACITY, "the run needs " + std::to_string(c->lay.total) +
                                               " bytes of arena, the static arena holds " +
                                               std::to_string((size_t)TPCCA_NOALLOC_ARENA_BYTES));
    use_arena(c, A, TPCCA_NOALLOC_ARENA_BYTES);
    return run_on_arena(c, false);
}

}  // extern "C"

static tpcca_status run_on_arena(tpcca_ctx *c, bool graphs) {
    hipStream_t s = c->stream;
    bind_pointers(c);
    const Layout &L = c->lay;
    char *A = c->arena;
    if (c->upload_dirty) {
        const int NS = c->cfg.n_sectors;
        for (int f = 0; f < (int)c->frames.size(); f++)
            for (int k = 0; k < NS; k++) {
                SectorIn &x = c->frames[f][k];
                SiDesc &d = c->si_host[(size_t)f * NS + k];
                if (!x.loaded || x.n == 0) {
                    d.row = nullptr;
                    d.y = d.t = nullptr;
                    continue;
                }
                if (x.host) {
                    char *p = A + x.stage_off;
                    const size_t o1 = align_up((size_t)x.n, 256), o2 = o1 + align_up((size_t)x.n * 4, 256);
                    HIPCHK(c, hipMemcpyAsync(p, x.hrow.data(), (size_t)x.n, hipMemcpyHostToDevice, s));
                    HIPCHK(c, hipMemcpyAsync(p + o1, x.hy.data(), (size_t)x.n * 4, hipMemcpyHostToDevice, s));
                    HIPCHK(c, hipMemcpyAsync(p + o2, x.ht.data(), (size_t)x.n * 4, hipMemcpyHostToDevice, s));
                    d.row = (const uint8_t *)p;
                    d.y = (const float *)(p + o1);
                    d.t = (const float *)(p + o2);
                } else {
                    d.row = x.drow;
                    d.y = x.dy;
                    d.t = x.dt;
                }
            }
        char *D = c->tab_dev;
        HIPCHK(c, hipMemcpyAsync(D + L.si, c->si_host.data(), sizeof(SiDesc) * c->si_host.size(),
                                 hipMemcpyHostToDevice, s));
        if (!c->chunks.empty())
            HIPCHK(c, hipMemcpyAsync(D + L.chunk, c->chunks.data(), sizeof(int32_t) * c->chunks.size(),
                                     hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemcpyAsync(D + L.row_x, c->row_x.data(), sizeof(float) * c->row_x.size(),
                                 hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemcpyAsync(D + L.w_tab, c->wtab.data(), sizeof(float) * c->wtab.size(),
                                 hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemcpyAsync(D + L.ycell, c->ycell.data(), sizeof(YCell) * c->ycell.size(),
                                 hipMemcpyHostToDevice, s));
        HIPCHK(c, hipStreamSynchronize(s));
        c->upload_dirty = false;
    }
    const bool tm = c->timing && c->events_ok && !graphs;
    const int slot = c->ev_next;
    if (tm) {
        fold_slot(c, slot);  // the slot is reused: fold its previous run first
        c->ev_next = (slot + 1) % kEvRing;
    }
    if (graphs) {
        if (!c->graph_valid) {
            // capture on an idle stream (earlier work of this or another
            // context on the stream finishes first)
            HIPCHK(c, hipStreamSynchronize(s));
            drop_graph(c);
            HIPCHK(c, hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
            enqueue_run(c, s, false, slot);
            hipGraph_t g = nullptr;
            hipError_t ec = hipStreamEndCapture(s, &g);
            if (ec != hipSuccess) return hip_fail(c, ec, "hipStreamEndCapture (graph mode needs a non-default stream)");
            c->graph = g;
            HIPCHK(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
            c->graph_valid = true;
        }
        HIPCHK(c, hipGraphLaunch(c->graph_exec, s));
    } else {
        enqueue_run(c, s, tm, slot);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
    if (tm) c->ev_pending[slot] = true;
    c->ran = true;
    c->have_results = true;
    c->coll_valid = false;
    c->merge_valid = false;
    c->rm_valid = false;
    c->mem_valid = false;
    c->refit_valid = false;
    return TPCCA_OK;
}

extern "C" {

tpcca_status tpcca_synchronize(tpcca_ctx *c) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->have_results && c->arena) {
        int32_t ovf = 0;
        HIPCHK(c, hipMemcpy(&ovf, c->arena + c->lay.cnt + offsetof(Counters, overflow), sizeof(ovf),
                            hipMemcpyDeviceToHost));
        if (ovf > 0) {
            c->have_results = false;
            return fail(c, TPCCA_ERR_CAPACITY, "track buffers overflowed (extended tracks of the following)");
        }
    }
    if (c->have_results && c->args.use_mlp && c->arena) {
        int32_t ovf = 0;
        HIPCHK(c, hipMemcpy(&ovf, c->arena + c->lay.cnt + offsetof(Counters, pool_overflow), sizeof(ovf),
                            hipMemcpyDeviceToHost));
        if (ovf > 0) {
            c->have_results = false;
            return fail(c, TPCCA_ERR_CAPACITY, c->args.keep_pool
                                                   ? "triplet pool overflow: raise pool_per_cluster"
                                                   : "a pad row of a dense tile holds 2^24 or more clusters");
        }
    }
    if (__atomic_load_n(c->abort_host, __ATOMIC_SEQ_CST)) {
        __atomic_store_n(c->abort_host, 0, __ATOMIC_SEQ_CST);
        c->have_results = false;
        return fail(c, TPCCA_ERR_ABORTED, "run aborted");
    }
    return TPCCA_OK;
}

tpcca_status tpcca_get_stats(tpcca_ctx *c, tpcca_stats *out) {
    if (!c || !out) return TPCCA_ERR_INVALID_ARG;
    tpcca_stats z{};
    *out = z;
    if (!c->ran) return fail(c, TPCCA_ERR_STATE, "no run yet");
    tpcca_status ss = tpcca_synchronize(c);
    if (ss != TPCCA_OK) return ss;
    Counters k;
    HIPCHK(c, hipMemcpy(&k, c->arena + c->lay.cnt, sizeof(k), hipMemcpyDeviceToHost));
    out->n_clusters = c->n_in;
    out->n_links = k.n_links;
    out->n_seeds = k.n_seeds;
    out->n_tracks = k.n_tracks;
    out->n_track_clusters = k.n_cl;
    out->n_invalid = k.n_invalid;
    out->n_overflow_tiles = k.n_glb_tiles + k.n_glb_inline;
    out->n_tiles = k.n_tiles;
    out->n_triplets = c->args.use_mlp ? k.pool_used : 0;
    out->n_pruned = k.n_pruned;
    out->n_pool_overflow = k.pool_overflow;
    out->mlp_used = c->args.use_mlp;
    for (int i = 0; i < 16 && i < kPassBins; i++) out->fit_passes[i] = k.fit_passes[i];
    out->n_fit_restarts = k.fit_passes[kPassBins];
    if (c->args.follow) {
        out->n_chains = k.n_chains;
        out->n_follow_added = k.f_added;
        out->n_follow_dropped = k.f_dropped;
    }
    out->n_stages = 0;
    if (c->timing && c->events_ok) {
        for (int r = 0; r < kEvRing; r++) fold_slot(c, (c->ev_next + r) % kEvRing);
        for (int i = 0; i < kNumStages; i++) {
            out->stage_ms[i] = c->stage_ms_last[i];
            out->stage_ms_total[i] = c->stage_ms_total[i];
            std::snprintf(out->stage_name[i], sizeof(out->stage_name[i]), "%s", kStageNames[i]);
        }
        out->n_stages = kNumStages;
        out->n_timed_runs = c->timed_runs;
    }
    return TPCCA_OK;
}

}  // extern "C"

static tpcca_status locate(tpcca_ctx *c, int32_t frame, int32_t sector, int &si, SiState &st) {
    if (frame < 0 || frame >= (int32_t)c->frames.size() || sector < 0 || sector >= c->cfg.n_sectors)
        return fail(c, TPCCA_ERR_INVALID_ARG, "frame or sector out of range");
    if (!c->have_results) return fail(c, TPCCA_ERR_STATE, "no results (run first)");
    tpcca_status s = tpcca_synchronize(c);
    if (s != TPCCA_OK) return s;
    si = frame * c->cfg.n_sectors + sector;
    HIPCHK(c, hipMemcpy(&st, c->arena + c->lay.st + sizeof(SiState) * si, sizeof(SiState), hipMemcpyDeviceToHost));
    return TPCCA_OK;
}

extern "C" {

tpcca_status tpcca_get_tracks(tpcca_ctx *c, int32_t frame, int32_t sector, tpcca_track *out, int64_t cap,
                              int64_t *n_out) {
    if (!c || !n_out) return TPCCA_ERR_INVALID_ARG;
    int si;
    SiState st;
    tpcca_status s = locate(c, frame, sector, si, st);
    if (s != TPCCA_OK) return s;
    *n_out = st.n_tracks;
    if (cap < st.n_tracks) return fail(c, TPCCA_ERR_CAPACITY, "track buffer too small");
    if (st.n_tracks > 0) {
        if (!out) return TPCCA_ERR_INVALID_ARG;
        HIPCHK(c, hipMemcpy(out, c->arena + c->lay.trk + sizeof(tpcca_track) * (size_t)st.trk_base,
                            sizeof(tpcca_track) * (size_t)st.n_tracks, hipMemcpyDeviceToHost));
    }
    return TPCCA_OK;
}

tpcca_status tpcca_get_track_clusters(tpcca_ctx *c, int32_t frame, int32_t sector, int32_t *out, int64_t cap,
                                      int64_t *n_out) {
    if (!c || !n_out) return TPCCA_ERR_INVALID_ARG;
    int si;
    SiState st;
    tpcca_status s = locate(c, frame, sector, si, st);
    if (s != TPCCA_OK) return s;
    *n_out = st.n_cl;
    if (cap < st.n_cl) return fail(c, TPCCA_ERR_CAPACITY, "cluster buffer too small");
    if (st.n_cl > 0) {
        if (!out) return TPCCA_ERR_INVALID_ARG;
        HIPCHK(c, hipMemcpy(out, c->arena + c->lay.clusters + sizeof(int32_t) * (size_t)st.cl_base,
                            sizeof(int32_t) * (size_t)st.n_cl, hipMemcpyDeviceToHost));
    }
    return TPCCA_OK;
}

tpcca_status tpcca_find_collisions(tpcca_ctx *c, float gap_cm, int32_t min_clusters, float window_cm,
                                   int64_t *n_groups_out) {
    if (!c || !n_groups_out || !(gap_cm > 0.f) || !std::isfinite(gap_cm) || min_clusters < 0 ||
        !(window_cm >= 0.f) || !std::isfinite(window_cm))
        return TPCCA_ERR_INVALID_ARG;
    *n_groups_out = 0;
    if (!c->have_results) return fail(c, TPCCA_ERR_STATE, "no results (run first)");
    tpcca_status ss = tpcca_synchronize(c);
    if (ss != TPCCA_OK) return ss;
    const int sides = 2 * (int)c->frames.size();
    char *A = c->arena;
    const Layout &L = c->lay;
    // working arrays in the slot after the chain copies (dead after a run)
    Bump b;
    const size_t o_range = b.take(sizeof(uint32_t) * 2 * sides), o_nb = b.take(sizeof(int32_t) * sides),
                 o_bb = b.take(sizeof(int32_t) * sides), o_ng = b.take(sizeof(int32_t) * sides),
                 o_gb = b.take(sizeof(int32_t) * sides);
    CollArgs ca{};
    ca.n_sectors = c->cfg.n_sectors;
    ca.gap = gap_cm;
    ca.min_len = min_clusters;
    ca.window = window_cm;
    {
        volatile float w = 0.5f * gap_cm;
        ca.inv_w = 1.0f / w;
    }
    char *X = A + L.xslot;
    ca.range = (uint32_t *)(X + o_range);
    ca.nbins = (int32_t *)(X + o_nb);
    ca.bin_base = (int32_t *)(X + o_bb);
    ca.n_groups = (int32_t *)(X + o_ng);
    ca.grp_base = (int32_t *)(X + o_gb);
    ca.trk_group = (int32_t *)(A + L.trk_group);
    std::vector<uint32_t> rng(2 * (size_t)sides);
    for (int h = 0; h < sides; h++) {
        rng[2 * h] = 0xffffffffu;
        rng[2 * h + 1] = 0u;
    }
    HIPCHK(c, hipMemcpyAsync(ca.range, rng.data(), sizeof(uint32_t) * rng.size(), hipMemcpyHostToDevice, c->stream));
    launch_t0_range(c->args, ca, c->stream);
    HIPCHK(c, hipMemcpyAsync(rng.data(), ca.range, sizeof(uint32_t) * rng.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // bins of half the gap per side, over its t0 range (the same FP32
    // arithmetic as the kernels' bin index)
    std::vector<int32_t> nb(sides, 0), bb(sides, 0);
    int64_t total = 0;
    for (int h = 0; h < sides; h++) {
        if (rng[2 * h] > rng[2 * h + 1]) continue;
        const float lo = fkey_inv(rng[2 * h]), hi = fkey_inv(rng[2 * h + 1]);
        volatile float d = hi - lo;
        volatile float v = d * ca.inv_w;
        const double bmax = std::floor((double)v);
        if (!(bmax >= 0.0) || bmax > 1e9) return fail(c, TPCCA_ERR_CAPACITY, "collision-time range too wide");
        nb[h] = (int32_t)bmax + 1;
        bb[h] = (int32_t)total;
        total += nb[h];
    }
    const size_t o_cnt = b.take(sizeof(uint32_t) * total), o_min = b.take(sizeof(uint32_t) * total),
                 o_max = b.take(sizeof(uint32_t) * total), o_grp = b.take(sizeof(int32_t) * total);
    if (b.off > L.slot_bytes / 2 || total > (int64_t)0x7fff0000)
        return fail(c, TPCCA_ERR_CAPACITY, "collision-time bins exceed the scratch slot (raise the gap)");
    ca.bin_cnt = (uint32_t *)(X + o_cnt);
    ca.bin_min = (uint32_t *)(X + o_min);
    ca.bin_max = (uint32_t *)(X + o_max);
    ca.bin_grp = (int32_t *)(X + o_grp);
    HIPCHK(c, hipMemcpyAsync(ca.nbins, nb.data(), sizeof(int32_t) * sides, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(ca.bin_base, bb.data(), sizeof(int32_t) * sides, hipMemcpyHostToDevice, c->stream));
    launch_fill_i32((int32_t *)ca.bin_cnt, total, 0, c->stream);
    launch_fill_i32((int32_t *)ca.bin_min, total, -1, c->stream);
    launch_fill_i32((int32_t *)ca.bin_max, total, 0, c->stream);
    launch_t0_bins(c->args, ca, sides, c->stream);
    std::vector<int32_t> ng(sides, 0), gb(sides, 0);
    HIPCHK(c, hipMemcpyAsync(ng.data(), ca.n_groups, sizeof(int32_t) * sides, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int64_t groups = 0;
    for (int h = 0; h < sides; h++) {
        if (!nb[h]) ng[h] = 0;
        gb[h] = (int32_t)groups;
        groups += ng[h];
    }
    // group sums and counts after the bins
    const size_t o_sum = b.take(sizeof(double) * groups), o_gc = b.take(sizeof(int32_t) * groups),
                 o_ga = b.take(sizeof(int32_t) * groups), o_gm = b.take(sizeof(double) * groups);
    if (b.off > L.slot_bytes / 2) return fail(c, TPCCA_ERR_CAPACITY, "collision groups exceed the scratch slot");
    ca.grp_sum = (double *)(X + o_sum);
    ca.grp_cnt = (int32_t *)(X + o_gc);
    ca.grp_att = (int32_t *)(X + o_ga);
    ca.grp_mean = (double *)(X + o_gm);
    HIPCHK(c, hipMemcpyAsync(ca.grp_base, gb.data(), sizeof(int32_t) * sides, hipMemcpyHostToDevice, c->stream));
    launch_fill_i32((int32_t *)ca.grp_sum, 2 * groups, 0, c->stream);
    launch_fill_i32(ca.grp_cnt, groups, 0, c->stream);
    launch_fill_i32(ca.grp_att, groups, 0, c->stream);
    launch_t0_group(c->args, ca, c->stream);
    launch_t0_attach(c->args, ca, (int)groups, c->stream);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "collision kernels");
    c->coll_n = ng;
    c->coll_base = gb;
    c->coll_sum_off = L.xslot + o_sum;
    c->coll_cnt_off = L.xslot + o_gc;
    c->coll_att_off = L.xslot + o_ga;
    c->coll_valid = true;
    *n_groups_out = groups;
    return TPCCA_OK;
}

tpcca_status tpcca_get_track_times(tpcca_ctx *c, int32_t frame, int32_t sector, float *t0, int32_t *group, int64_t cap,
                                   int64_t *n_out) {
    if (!c || !n_out) return TPCCA_ERR_INVALID_ARG;
    int si;
    SiState st;
    tpcca_status s = locate(c, frame, sector, si, st);
    if (s != TPCCA_OK) return s;
    *n_out = st.n_tracks;
    if (cap < st.n_tracks) return fail(c, TPCCA_ERR_CAPACITY, "buffer too small");
    if (st.n_tracks > 0) {
        if (t0)
            HIPCHK(c, hipMemcpy(t0, c->arena + c->lay.trk_t0 + sizeof(float) * (size_t)st.trk_base,
                                sizeof(float) * (size_t)st.n_tracks, hipMemcpyDeviceToHost));
        if (group) {
            if (c->coll_valid)
                HIPCHK(c, hipMemcpy(group, c->arena + c->lay.trk_group + sizeof(int32_t) * (size_t)st.trk_base,
                                    sizeof(int32_t) * (size_t)st.n_tracks, hipMemcpyDeviceToHost));
            else
                for (int64_t k = 0; k < st.n_tracks; k++) group[k] = -1;
        }
    }
    return TPCCA_OK;
}

tpcca_status tpcca_get_collisions(tpcca_ctx *c, int32_t frame, int32_t side, float *t0, int32_t *n_tracks,
                                  int32_t *n_anchors, int64_t cap, int64_t *n_out) {
    if (!c || !n_out) return TPCCA_ERR_INVALID_ARG;
    if (frame < 0 || frame >= (int32_t)c->frames.size() || side < 0 || side > 1)
        return fail(c, TPCCA_ERR_INVALID_ARG, "frame or side out of range");
    if (!c->coll_valid) return fail(c, TPCCA_ERR_STATE, "no collision candidates (call tpcca_find_collisions)");
    const int h = 2 * frame + side;
    const int n = c->coll_n[h];
    *n_out = n;
    if (cap < n) return fail(c, TPCCA_ERR_CAPACITY, "buffer too small");
    if (n > 0) {
        std::vector<double> sum(n);
        std::vector<int32_t> cnt(n), att(n);
        HIPCHK(c, hipMemcpy(sum.data(), c->arena + c->coll_sum_off + sizeof(double) * (size_t)c->coll_base[h],
                            sizeof(double) * (size_t)n, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(cnt.data(), c->arena + c->coll_cnt_off + sizeof(int32_t) * (size_t)c->coll_base[h],
                            sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(att.data(), c->arena + c->coll_att_off + sizeof(int32_t) * (size_t)c->coll_base[h],
                            sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));
        for (int k = 0; k < n; k++) {
            if (t0) t0[k] = cnt[k] ? (float)(sum[k] / cnt[k]) : 0.f;
            if (n_tracks) n_tracks[k] = cnt[k] + att[k];
            if (n_anchors) n_anchors[k] = cnt[k];
        }
    }
    return TPCCA_OK;
}

// The merge pipeline (range, bins, placement, best candidates, mutual bests)
// with its working arrays in [region, region + room) of the arena; used =
// bytes taken.
static tpcca_status run_merge(tpcca_ctx *c, int32_t membrane, int32_t min_clusters, float window_cm, float d2_cut,
                              size_t region, size_t room, MergeArgs &m, size_t &used, int64_t *n_pairs_out) {
    char *A = c->arena;
    char *X = A + region;
    const int64_t trk_cap = c->args.trk_cap;
    Bump b;
    const size_t o_rng = b.take(sizeof(uint32_t) * 2), o_np = b.take(sizeof(int32_t));
    m = MergeArgs{};
    m.n_sectors = c->cfg.n_sectors;
    m.membrane = membrane;
    m.min_len = min_clusters;
    m.window = window_cm;
    m.d2_cut = d2_cut;
    m.range = (uint32_t *)(X + o_rng);
    m.n_pairs = (int32_t *)(X + o_np);
    uint32_t rng[2] = {0xffffffffu, 0u};
    HIPCHK(c, hipMemcpyAsync(m.range, rng, sizeof(rng), hipMemcpyHostToDevice, c->stream));
    launch_merge_range(c->args, m, c->stream);
    HIPCHK(c, hipMemcpyAsync(rng, m.range, sizeof(rng), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int n_si = c->args.n_si;
    int64_t nt = 0;
    {
        int32_t v = 0;
        HIPCHK(c, hipMemcpy(&v, &c->args.cnt->n_tracks, sizeof(int32_t), hipMemcpyDeviceToHost));
        nt = std::min<int64_t>(v, trk_cap);
    }
    // time bins: the smallest power of two >= the window, from a multiple
    // of the width (exact bin indices); wider if the bins would not fit the
    // scan
    double w = 1.0;
    while (w < (double)window_cm) w *= 2.0;
    double lo = 0.0;
    int64_t nb = 1;
    for (;;) {
        if (rng[0] <= rng[1]) {
            const double tmin = fkey_inv(rng[0]), tmax = fkey_inv(rng[1]);
            lo = std::floor(tmin / w) * w;
            nb = (int64_t)std::floor((tmax - lo) / w) + 1;
        }
        if ((int64_t)n_si * nb + 1 <= trk_cap || w > 1e30) break;
        w *= 2.0;
    }
    m.bin_w = (float)w;
    m.inv_w = (float)(1.0 / w);
    m.lo = (float)lo;
    m.nb = (int32_t)nb;
    const int64_t nbins = (int64_t)n_si * nb;
    const int64_t ntr = std::max<int64_t>(nt, 1);
    const size_t o_bn = b.take(sizeof(int32_t) * ntr), o_bp = b.take(sizeof(int32_t) * ntr),
                 o_pn = b.take(sizeof(int32_t) * ntr), o_pp = b.take(sizeof(int32_t) * ntr),
                 o_list = b.take(sizeof(int32_t) * ntr), o_mst = b.take(2 * sizeof(float4) * ntr),
                 o_start = b.take(sizeof(int32_t) * (nbins + 1)), o_cur = b.take(sizeof(int32_t) * nbins);
    if (b.off > room) return fail(c, TPCCA_ERR_CAPACITY, "merge arrays exceed the scratch slot");
    m.best_next = (int32_t *)(X + o_bn);
    m.best_prev = (int32_t *)(X + o_bp);
    m.partner_next = (int32_t *)(X + o_pn);
    m.partner_prev = (int32_t *)(X + o_pp);
    m.list = (int32_t *)(X + o_list);
    m.mst = (float4 *)(X + o_mst);
    m.start = (int32_t *)(X + o_start);
    m.cur = (int32_t *)(X + o_cur);
    m.n_elig = m.start + nbins;   // the scan's total
    launch_fill_i32(m.start, nbins + 1, 0, c->stream);
    launch_fill_i32(m.cur, nbins, 0, c->stream);
    launch_fill_i32(m.n_pairs, 1, 0, c->stream);
    launch_fill_i32(m.best_next, ntr, -1, c->stream);
    launch_fill_i32(m.best_prev, ntr, -1, c->stream);
    launch_fill_i32(m.partner_next, ntr, -1, c->stream);
    launch_fill_i32(m.partner_prev, ntr, -1, c->stream);
    launch_merge_count(c->args, m, c->stream);
    launch_scan_i32(m.start, (int32_t)nbins, m.start, nullptr, c->args.scan_tmp, c->stream);   // nbins + 1 entries
    launch_merge_place(c->args, m, c->stream);
    launch_merge_pairs(c->args, m, (int)nt, (int)nt, c->stream);
    int32_t np = 0;
    HIPCHK(c, hipMemcpyAsync(&np, m.n_pairs, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "merge kernels");
    used = align_up(b.off, 256);
    *n_pairs_out = np;
    return TPCCA_OK;
}

static tpcca_status merge_check(tpcca_ctx *c, int32_t min_clusters, float window_cm, float d2_cut,
                                int64_t *n_pairs_out) {
    if (!c || !n_pairs_out || min_clusters < 0 || !(window_cm > 0.f) || !std::isfinite(window_cm) ||
        !(d2_cut >= 0.f) || !std::isfinite(d2_cut))
        return TPCCA_ERR_INVALID_ARG;
    *n_pairs_out = 0;
    if (!c->have_results) return fail(c, TPCCA_ERR_STATE, "no results (run first)");
    if (c->cfg.n_sectors < 2 || (c->cfg.n_sectors & 1))
        return fail(c, TPCCA_ERR_STATE, "merging needs an even number of sectors (two sides)");
    return tpcca_synchronize(c);
}

tpcca_status tpcca_merge_sectors(tpcca_ctx *c, int32_t min_clusters, float window_cm, float d2_cut,
                                 int64_t *n_pairs_out) {
    tpcca_status ss = merge_check(c, min_clusters, window_cm, d2_cut, n_pairs_out);
    if (ss != TPCCA_OK) return ss;
    const Layout &L = c->lay;
    // working arrays in the upper half of the slot after the chain copies
    // (the lower half keeps the collision candidates); the membrane merges
    // and the refits come after them
    const size_t region = L.xslot + align_up(L.slot_bytes / 2, 256);
    const size_t room = L.slot_bytes - align_up(L.slot_bytes / 2, 256);
    c->merge_valid = c->mem_valid = c->refit_valid = false;
    MergeArgs m;
    size_t used = 0;
    ss = run_merge(c, 0, min_clusters, window_cm, d2_cut, region, room, m, used, n_pairs_out);
    if (ss != TPCCA_OK) return ss;
    c->merge_next_off = (size_t)((char *)m.partner_next - c->arena);
    c->merge_prev_off = (size_t)((char *)m.partner_prev - c->arena);
    c->merge_end = region + used;
    c->merge_valid = true;
    return TPCCA_OK;
}

tpcca_status tpcca_merge_membrane(tpcca_ctx *c, int32_t min_clusters, float window_cm, float d2_cut,
                                  int64_t *n_pairs_out) {
    tpcca_status ss = merge_check(c, min_clusters, window_cm, d2_cut, n_pairs_out);
    if (ss != TPCCA_OK) return ss;
    const Layout &L = c->lay;
    // after the sector merges (if any) in the upper half of the slot; a
    // refit placed there before is overwritten
    const size_t region = c->merge_valid ? c->merge_end : L.xslot + align_up(L.slot_bytes / 2, 256);
    const size_t room = L.xslot + L.slot_bytes - region;
    c->mem_valid = c->refit_valid = false;
    MergeArgs m;
    size_t used = 0;
    ss = run_merge(c, 1, min_clusters, window_cm, d2_cut, region, room, m, used, n_pairs_out);
    if (ss != TPCCA_OK) return ss;
    c->mem_a_off = (size_t)((char *)m.partner_next - c->arena);
    c->mem_c_off = (size_t)((char *)m.partner_prev - c->arena);
    c->mem_end = region + used;
    c->mem_valid = true;
    return TPCCA_OK;
}

tpcca_status tpcca_refit_merged(tpcca_ctx *c, int64_t *n_out) {
    if (!c || !n_out) return TPCCA_ERR_INVALID_ARG;
    *n_out = 0;
    if (!c->merge_valid) return fail(c, TPCCA_ERR_STATE, "no merges (call tpcca_merge_sectors)");
    tpcca_status ss = tpcca_synchronize(c);
    if (ss != TPCCA_OK) return ss;
    char *A = c->arena;
    const Layout &L = c->lay;
    const KArgs &a = c->args;
    Counters k{};
    HIPCHK(c, hipMemcpy(&k, a.cnt, sizeof(Counters), hipMemcpyDeviceToHost));
    const int64_t nt = std::min<int64_t>(k.n_tracks, a.trk_cap);
    // the pair arrays after the merge arrays and the membrane merges (upper
    // half of the slot)
    const size_t end = L.xslot + L.slot_bytes;
    Bump b;
    b.off = c->mem_valid ? std::max(c->merge_end, c->mem_end) : c->merge_end;
    const size_t o_flags = b.take(sizeof(int32_t) * (nt + 1)), o_pidx = b.take(sizeof(int32_t) * (nt + 1));
    if (b.off > end) return fail(c, TPCCA_ERR_CAPACITY, "refit arrays exceed the scratch slot");
    RefitArgs r{};
    r.n_sectors = c->cfg.n_sectors;
    r.flags = (int32_t *)(A + o_flags);
    r.pidx = (int32_t *)(A + o_pidx);
    MergeArgs m{};
    m.partner_next = (int32_t *)(A + c->merge_next_off);
    launch_refit_flags(a, m, r, (int)nt, c->stream);
    launch_scan_i32(r.flags, (int32_t)nt, r.pidx, nullptr, a.scan_tmp, c->stream);
    int32_t np = 0;
    HIPCHK(c, hipMemcpyAsync(&np, r.pidx + nt, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int64_t npr = std::max<int64_t>(np, 1);
    const size_t o_pa = b.take(sizeof(int32_t) * npr), o_pb = b.take(sizeof(int32_t) * npr),
                 o_vlen = b.take(sizeof(int32_t) * (npr + 1)), o_voff = b.take(sizeof(int32_t) * (npr + 1)),
                 o_vseed = b.take(sizeof(int32_t) * npr), o_vperm = b.take(sizeof(int32_t) * npr),
                 o_vt0 = b.take(sizeof(float) * npr), o_vtrk = b.take(sizeof(tpcca_track) * npr),
                 o_vcnt = b.take(sizeof(Counters));
    if (b.off > end) return fail(c, TPCCA_ERR_CAPACITY, "refit arrays exceed the scratch slot");
    r.pa = (int32_t *)(A + o_pa);
    r.pb = (int32_t *)(A + o_pb);
    r.vlen = (int32_t *)(A + o_vlen);
    r.voff = (int32_t *)(A + o_voff);
    r.vseed = (int32_t *)(A + o_vseed);
    r.vperm = (int32_t *)(A + o_vperm);
    launch_refit_pairs(a, m, r, (int)nt, c->stream);
    launch_scan_i32(r.vlen, np, r.voff, nullptr, a.scan_tmp, c->stream);
    int32_t n_ent = 0;
    HIPCHK(c, hipMemcpyAsync(&n_ent, r.voff + np, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // the virtual chains take the chain-copy region after the copies in use
    const int64_t used = std::max<int64_t>(k.chain_next, k.f_chain_next);
    r.vchain = a.chain + used;
    r.vcap = std::max<int64_t>(a.chain_cap - used, 0);
    if (n_ent > r.vcap) return fail(c, TPCCA_ERR_CAPACITY, "merged tracks exceed the free chain-copy space");
    launch_refit_build(a, r, np, c->stream);
    // the fit over the virtual tracks: its own track arrays and counters
    KArgs va = a;
    va.chain = r.vchain;
    va.choff = r.voff;
    va.trk_len = r.vlen;
    va.perm = r.vperm;
    va.trk_seed = r.vseed;
    va.cl_off = r.voff;   // no cluster lists for refits: 'first' is not meaningful
    va.trk = (tpcca_track *)(A + o_vtrk);
    va.trk_t0 = (float *)(A + o_vt0);
    va.cnt = (Counters *)(A + o_vcnt);
    va.trk_cap = (int32_t)npr;
    Counters z{};
    z.n_tracks = np;
    HIPCHK(c, hipMemcpyAsync(va.cnt, &z, sizeof(Counters), hipMemcpyHostToDevice, c->stream));
    // vlen was scanned into voff; the lengths themselves are still in vlen
    if (np > 0) launch_fit_x(va, c->lc[11], c->stream);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "refit kernels");
    c->refit_pidx_off = o_pidx;
    c->refit_pa_off = o_pa;
    c->refit_pb_off = o_pb;
    c->refit_trk_off = o_vtrk;
    c->refit_n = np;
    c->refit_valid = true;
    *n_out = np;
    return TPCCA_OK;
}

tpcca_status tpcca_get_refits(tpcca_ctx *c, int32_t frame, int32_t sector, tpcca_track *tracks, int32_t *first_track,
                              int32_t *partner, int64_t cap, int64_t *n_out) {
    if (!c || !n_out) return TPCCA_ERR_INVALID_ARG;
    if (!c->refit_valid) return fail(c, TPCCA_ERR_STATE, "no refits (call tpcca_refit_merged)");
    int si;
    SiState st;
    tpcca_status s = locate(c, frame, sector, si, st);
    if (s != TPCCA_OK) return s;
    const int half = c->cfg.n_sectors / 2, side = sector / half, k = sector % half;
    int si_n;
    SiState stn;
    s = locate(c, frame, side * half + (k + 1) % half, si_n, stn);
    if (s != TPCCA_OK) return s;
    int32_t r0 = 0, r1 = 0;
    const int32_t *pidx = (const int32_t *)(c->arena + c->refit_pidx_off);
    HIPCHK(c, hipMemcpy(&r0, pidx + st.trk_base, sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(&r1, pidx + st.trk_base + st.n_tracks, sizeof(int32_t), hipMemcpyDeviceToHost));
    const int64_t n = r1 - r0;
    *n_out = n;
    if (cap < n) return fail(c, TPCCA_ERR_CAPACITY, "buffer too small");
    if (n == 0) return TPCCA_OK;
    if (tracks)
        HIPCHK(c, hipMemcpy(tracks, c->arena + c->refit_trk_off + sizeof(tpcca_track) * (size_t)r0,
                            sizeof(tpcca_track) * (size_t)n, hipMemcpyDeviceToHost));
    for (int dir = 0; dir < 2; dir++) {
        int32_t *out = dir == 0 ? first_track : partner;
        if (!out) continue;
        HIPCHK(c, hipMemcpy(out, c->arena + (dir == 0 ? c->refit_pa_off : c->refit_pb_off) + sizeof(int32_t) * (size_t)r0,
                            sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));
        const int32_t base = dir == 0 ? st.trk_base : stn.trk_base;
        for (int64_t i = 0; i < n; i++) out[i] -= base;
    }
    return TPCCA_OK;
}

tpcca_status tpcca_get_merges(tpcca_ctx *c, int32_t frame, int32_t sector, int32_t *next, int32_t *prev, int64_t cap,
                              int64_t *n_out) {
    if (!c || !n_out) return TPCCA_ERR_INVALID_ARG;
    if (!c->merge_valid) return fail(c, TPCCA_ERR_STATE, "no merges (call tpcca_merge_sectors)");
    int si;
    SiState st;
    tpcca_status s = locate(c, frame, sector, si, st);
    if (s != TPCCA_OK) return s;
    *n_out = st.n_tracks;
    if (cap < st.n_tracks) return fail(c, TPCCA_ERR_CAPACITY, "buffer too small");
    if (st.n_tracks == 0) return TPCCA_OK;
    const int half = c->cfg.n_sectors / 2, side = sector / half, k = sector % half;
    int si_n, si_p;
    SiState stn, stp;
    s = locate(c, frame, side * half + (k + 1) % half, si_n, stn);
    if (s != TPCCA_OK) return s;
    s = locate(c, frame, side * half + (k + half - 1) % half, si_p, stp);
    if (s != TPCCA_OK) return s;
    for (int dir = 0; dir < 2; dir++) {
        int32_t *out = dir == 0 ? next : prev;
        if (!out) continue;
        HIPCHK(c, hipMemcpy(out, c->arena + (dir == 0 ? c->merge_next_off : c->merge_prev_off) +
                                     sizeof(int32_t) * (size_t)st.trk_base,
                            sizeof(int32_t) * (size_t)st.n_tracks, hipMemcpyDeviceToHost));
        const int32_t base = dir == 0 ? stn.trk_base : stp.trk_base;
        for (int64_t i = 0; i < st.n_tracks; i++)
            if (out[i] >= 0) out[i] -= base;
    }
    return TPCCA_OK;
}

tpcca_status tpcca_remove_clusters(tpcca_ctx *c, float pt_min, int32_t *kept, int64_t cap, int64_t *n_kept) {
    if (!c || !n_kept || !(pt_min > 0.f) || !std::isfinite(pt_min) || cap < 0 || (cap > 0 && !kept))
        return TPCCA_ERR_INVALID_ARG;
    *n_kept = 0;
    if (!c->have_results) return fail(c, TPCCA_ERR_STATE, "no results (run first)");
    tpcca_status ss = tpcca_synchronize(c);
    if (ss != TPCCA_OK) return ss;
    const KArgs &a = c->args;
    const Layout &L = c->lay;
    c->rm_valid = false;
    RemoveArgs r{};
    r.n_sectors = c->cfg.n_sectors;
    r.qpt_max = 1.f / pt_min;
    r.bits = (uint32_t *)(c->arena + L.rm_bits);
    r.ccnt = (int32_t *)(c->arena + L.rm_cnt);
    r.out = kept;
    r.cap = cap;
    int32_t nt = 0;
    HIPCHK(c, hipMemcpy(&nt, &a.cnt->n_tracks, sizeof(int32_t), hipMemcpyDeviceToHost));
    nt = std::min(nt, a.trk_cap);
    launch_fill_i32((int32_t *)r.bits, (int64_t)(a.n_in / 32 + 2), 0, c->stream);
    launch_remove_flags(a, r, nt, c->stream);
    launch_remove_count(a, r, c->stream);
    launch_scan_i32(r.ccnt, a.n_chunks, r.ccnt, nullptr, a.scan_tmp, c->stream);   // n_chunks + 1 entries
    int32_t total = 0;
    HIPCHK(c, hipMemcpyAsync(&total, r.ccnt + a.n_chunks, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *n_kept = total;
    c->rm_valid = true;
    if (cap < total) return fail(c, TPCCA_ERR_CAPACITY, "kept-cluster buffer too small");
    launch_remove_write(a, r, c->stream);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "removal kernels");
    return TPCCA_OK;
}

tpcca_status tpcca_entropy_histograms(tpcca_ctx *c, int32_t frame, int32_t sector, int64_t *hist) {
    if (!c || !hist) return TPCCA_ERR_INVALID_ARG;
    if (!c->have_results) return fail(c, TPCCA_ERR_STATE, "no results (run first)");
    tpcca_status ss = tpcca_synchronize(c);
    if (ss != TPCCA_OK) return ss;
    EntropyArgs e{};
    e.only_si = -1;
    if (frame >= 0 || sector >= 0) {
        int si;
        SiState st;
        ss = locate(c, frame, sector, si, st);
        if (ss != TPCCA_OK) return ss;
        e.only_si = si;
    }
    e.hist = (int32_t *)(c->arena + c->lay.ent_hist);
    const KArgs &a = c->args;
    int32_t nt = 0;
    HIPCHK(c, hipMemcpy(&nt, &a.cnt->n_tracks, sizeof(int32_t), hipMemcpyDeviceToHost));
    nt = std::min(nt, a.trk_cap);
    launch_fill_i32(e.hist, kEntStreams * kEntBins, 0, c->stream);
    launch_entropy_hist(a, e, nt, c->stream);
    int32_t h[kEntStreams * kEntBins];
    HIPCHK(c, hipMemcpyAsync(h, e.hist, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return hip_fail(c, err, "entropy kernel");
    for (int i = 0; i < kEntStreams * kEntBins; i++) hist[i] = h[i];
    return TPCCA_OK;
}

// rANS frequency model of one stream: f = max(1, floor(count 2^16 / total))
// for counted bins (the escape bin counted at least once), the shortfall to
// 2^16 added to the bin of the largest count, an excess taken one unit at a
// time from the bin of the largest frequency (lowest index on ties).
static void ans_model(const int64_t *hin, uint32_t *f, uint32_t *c) {
    int64_t h[kEntBins];
    int64_t tot = 0;
    for (int i = 0; i < kEntBins; i++) h[i] = hin[i];
    h[kEntBins - 1] = std::max<int64_t>(h[kEntBins - 1], 1);
    for (int i = 0; i < kEntBins; i++) tot += h[i];
    const int64_t M = 1 << 16;
    int64_t sum = 0;
    for (int i = 0; i < kEntBins; i++) {
        f[i] = h[i] > 0 ? (uint32_t)std::max<int64_t>(1, h[i] * M / tot) : 0u;
        sum += f[i];
    }
    int64_t d = M - sum;
    if (d > 0) {
        int im = 0;
        for (int i = 1; i < kEntBins; i++)
            if (h[i] > h[im]) im = i;
        f[im] += (uint32_t)d;
    }
    while (d < 0) {
        int im = 0;
        for (int i = 1; i < kEntBins; i++)
            if (f[i] > f[im]) im = i;
        f[im]--;
        d++;
    }
    c[0] = 0;
    for (int i = 1; i < kEntBins; i++) c[i] = c[i - 1] + f[i - 1];
}

tpcca_status tpcca_ans_encode(tpcca_ctx *c, int32_t frame, int32_t sector, uint8_t *bytes, int64_t cap,
                              int64_t *offsets, int64_t n_offsets, int64_t *n_bytes) {
    if (!c || !n_bytes || cap < 0 || (cap > 0 && !bytes)) return TPCCA_ERR_INVALID_ARG;
    *n_bytes = 0;
    if (!c->have_results) return fail(c, TPCCA_ERR_STATE, "no results (run first)");
    tpcca_status ss = tpcca_synchronize(c);
    if (ss != TPCCA_OK) return ss;
    int si;
    SiState st;
    ss = locate(c, frame, sector, si, st);
    if (ss != TPCCA_OK) return ss;
    const KArgs &a = c->args;
    const Layout &L = c->lay;
    // the sector's symbol histograms, then the models
    EntropyArgs e{};
    e.only_si = si;
    e.hist = (int32_t *)(c->arena + L.ent_hist);
    int32_t nt = 0;
    HIPCHK(c, hipMemcpy(&nt, &a.cnt->n_tracks, sizeof(int32_t), hipMemcpyDeviceToHost));
    nt = std::min(nt, a.trk_cap);
    launch_fill_i32(e.hist, kEntStreams * kEntBins, 0, c->stream);
    launch_entropy_hist(a, e, nt, c->stream);
    int32_t h32[kEntStreams * kEntBins];
    HIPCHK(c, hipMemcpyAsync(h32, e.hist, sizeof(h32), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    uint32_t tab[2 * kEntStreams * kEntBins];
    for (int k = 0; k < kEntStreams; k++) {
        int64_t h[kEntBins];
        for (int i = 0; i < kEntBins; i++) h[i] = h32[k * kEntBins + i];
        ans_model(h, tab + k * kEntBins, tab + kEntStreams * kEntBins + k * kEntBins);
    }
    AnsArgs n{};
    n.trk_base = st.trk_base;
    n.n_tracks = st.n_tracks;
    n.freq = (const uint32_t *)(c->arena + L.ans_tab);
    n.cum = n.freq + kEntStreams * kEntBins;
    n.size = (int32_t *)(c->arena + L.ans_size);
    n.out = bytes;
    HIPCHK(c, hipMemcpyAsync(c->arena + L.ans_tab, tab, sizeof(tab), hipMemcpyHostToDevice, c->stream));
    launch_ans_size(a, n, c->stream);
    launch_scan_i32(n.size, st.n_tracks, n.size, nullptr, a.scan_tmp, c->stream);   // n_tracks + 1 entries
    int32_t total = 0;
    HIPCHK(c, hipMemcpyAsync(&total, n.size + st.n_tracks, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *n_bytes = total;
    if (cap < total) return fail(c, TPCCA_ERR_CAPACITY, "byte buffer too small");
    if (offsets && n_offsets < (int64_t)st.n_tracks + 1) return fail(c, TPCCA_ERR_CAPACITY, "offset array too small");
    launch_ans_write(a, n, c->stream);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return hip_fail(c, err, "rANS kernels");
    if (offsets) {
        std::vector<int32_t> o((size_t)st.n_tracks + 1);
        HIPCHK(c, hipMemcpy(o.data(), n.size, sizeof(int32_t) * o.size(), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < o.size(); i++) offsets[i] = o[i];
    }
    return TPCCA_OK;
}

tpcca_status tpcca_get_removal_range(tpcca_ctx *c, int32_t frame, int32_t sector, int64_t *begin, int64_t *count) {
    if (!c || !begin || !count) return TPCCA_ERR_INVALID_ARG;
    if (!c->rm_valid) return fail(c, TPCCA_ERR_STATE, "no removal (call tpcca_remove_clusters)");
    int si;
    SiState st;
    tpcca_status s = locate(c, frame, sector, si, st);
    if (s != TPCCA_OK) return s;
    // the sector's chunks are consecutive in the chunk table
    const int nch = (int)(c->chunks.size() / 2);
    int k0 = 0;
    while (k0 < nch && c->chunks[2 * k0] < si) k0++;
    int k1 = k0;
    while (k1 < nch && c->chunks[2 * k1] == si) k1++;
    int32_t v[2] = {0, 0};
    const int32_t *cc = (const int32_t *)(c->arena + c->lay.rm_cnt);
    HIPCHK(c, hipMemcpy(&v[0], cc + k0, sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(&v[1], cc + k1, sizeof(int32_t), hipMemcpyDeviceToHost));
    *begin = v[0];
    *count = v[1] - v[0];
    return TPCCA_OK;
}

tpcca_status tpcca_get_membrane_merges(tpcca_ctx *c, int32_t frame, int32_t sector, int32_t *partner, int64_t cap,
                                       int64_t *n_out) {
    if (!c || !n_out) return TPCCA_ERR_INVALID_ARG;
    if (!c->mem_valid) return fail(c, TPCCA_ERR_STATE, "no membrane merges (call tpcca_merge_membrane)");
    int si;
    SiState st;
    tpcca_status s = locate(c, frame, sector, si, st);
    if (s != TPCCA_OK) return s;
    *n_out = st.n_tracks;
    if (cap < st.n_tracks) return fail(c, TPCCA_ERR_CAPACITY, "buffer too small");
    if (st.n_tracks == 0 || !partner) return TPCCA_OK;
    const int half = c->cfg.n_sectors / 2, side = sector / half;
    int si_o;
    SiState sto;
    s = locate(c, frame, side == 0 ? sector + half : sector - half, si_o, sto);
    if (s != TPCCA_OK) return s;
    HIPCHK(c, hipMemcpy(partner, c->arena + (side == 0 ? c->mem_a_off : c->mem_c_off) +
                                     sizeof(int32_t) * (size_t)st.trk_base,
                        sizeof(int32_t) * (size_t)st.n_tracks, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < st.n_tracks; i++)
        if (partner[i] >= 0) partner[i] -= sto.trk_base;
    return TPCCA_OK;
}

tpcca_status tpcca_get_assignment(tpcca_ctx *c, int32_t frame, int32_t sector, int32_t *out, int64_t n) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    int si;
    SiState st;
    tpcca_status s = locate(c, frame, sector, si, st);
    if (s != TPCCA_OK) return s;
    const SiDesc &d = c->si_host[si];
    if (n != d.n) return fail(c, TPCCA_ERR_INVALID_ARG, "n must equal the sector's cluster count");
    if (n > 0) {
        if (!out) return TPCCA_ERR_INVALID_ARG;
        HIPCHK(c, hipMemcpy(out, c->arena + c->lay.assign + sizeof(int32_t) * (size_t)d.in_base,
                            sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));
    }
    return TPCCA_OK;
}

tpcca_status tpcca_get_links(tpcca_ctx *c, int32_t frame, int32_t sector, int32_t cleaned, int32_t *up,
                             int32_t *dn, int64_t n) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    int si;
    SiState st;
    tpcca_status s = locate(c, frame, sector, si, st);
    if (s != TPCCA_OK) return s;
    const SiDesc &d = c->si_host[si];
    if (n != d.n) return fail(c, TPCCA_ERR_INVALID_ARG, "n must equal the sector's cluster count");
    if (n == 0) return TPCCA_OK;
    if (!up || !dn) return TPCCA_ERR_INVALID_ARG;
    const int nv = st.n_valid;
    std::vector<Rec> rec((size_t)nv);
    std::vector<int2> lk((size_t)nv);
    if (nv > 0) {
        HIPCHK(c, hipMemcpy(rec.data(), c->arena + c->lay.rec + sizeof(Rec) * (size_t)st.sbase,
                            sizeof(Rec) * (size_t)nv, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(lk.data(), c->arena + c->lay.link + sizeof(int2) * (size_t)st.sbase,
                            sizeof(int2) * (size_t)nv, hipMemcpyDeviceToHost));
    }
    for (int64_t i = 0; i < n; i++) up[i] = dn[i] = -1;
    const int base = st.sbase;
    for (int p = 0; p < nv; p++) {
        const int u = lk[p].x, dd = lk[p].y;
        const int id = rec[p].id;
        int uo = -1, doo = -1;
        if (u >= 0 && (!cleaned || lk[u - base].y == p + base)) uo = rec[u - base].id;
        if (dd >= 0 && (!cleaned || lk[dd - base].x == p + base)) doo = rec[dd - base].id;
        up[id] = uo;
        dn[id] = doo;
    }
    return TPCCA_OK;
}

}  // extern "C"

// ------------------------------------------------------------------- MLP
static uint16_t host_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

extern "C" {

tpcca_status tpcca_mlp_state_bytes(size_t *bytes) {
    if (!bytes) return TPCCA_ERR_INVALID_ARG;
    *bytes = MlpState::bytes;
    return TPCCA_OK;
}

tpcca_status tpcca_mlp_attach(tpcca_ctx *c, void *ptr, size_t bytes) {
    if (!c) return TPCCA_ERR_INVALID_ARG;
    if (ptr && ((uintptr_t)ptr & 255)) return fail(c, TPCCA_ERR_INVALID_ARG, "state buffer must be 256-byte aligned");
    if (ptr && bytes < MlpState::bytes) return fail(c, TPCCA_ERR_NOMEM, "network state buffer too small");
    (void)hipStreamSynchronize(c->stream);
    c->mlp = (char *)ptr;
    c->mlp_loaded = false;
    c->graph_valid = false;
    return TPCCA_OK;
}

tpcca_status tpcca_mlp_load(tpcca_ctx *c, const float *params) {
    if (!c || !params) return TPCCA_ERR_INVALID_ARG;
    if (!c->mlp) return fail(c, TPCCA_ERR_STATE, "no network state buffer attached");
    for (int i = 0; i < kMlpNParam; i++)
        if (!std::isfinite(params[i])) return fail(c, TPCCA_ERR_INVALID_ARG, "non-finite network parameter");
    std::vector<uint16_t> w1(kMlpH * kMlpInP), w2(kMlpH * kMlpH), w3(kMlpH);
    std::vector<float> master(params, params + kMlpNParam);
    for (int j = 0; j < kMlpH; j++)
        for (int k = kMlpIn; k < kMlpInP; k++) master[j * kMlpInP + k] = 0.f;  // unused input columns
    for (int i = 0; i < kMlpH * kMlpInP; i++) w1[i] = host_bf16(master[i]);
    for (int i = 0; i < kMlpH * kMlpH; i++) w2[i] = host_bf16(master[1088 + i]);
    for (int i = 0; i < kMlpH; i++) w3[i] = host_bf16(master[5248 + i]);
    std::vector<char> zeros(MlpState::bytes - MlpState::adam_m, 0);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->mlp + MlpState::w1, w1.data(), w1.size() * 2, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->mlp + MlpState::w2, w2.data(), w2.size() * 2, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->mlp + MlpState::w3, w3.data(), w3.size() * 2, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->mlp + MlpState::b1, master.data() + 1024, kMlpH * 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->mlp + MlpState::b2, master.data() + 5184, kMlpH * 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->mlp + MlpState::b3, master.data() + 5312, 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->mlp + MlpState::master, master.data(), kMlpNParam * 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->mlp + MlpState::adam_m, zeros.data(), zeros.size(), hipMemcpyHostToDevice));
    if (!c->mlp_loaded) c->graph_valid = false;  // the run's flow changes (plain -> pruned)
    c->mlp_loaded = true;
    return TPCCA_OK;
}

tpcca_status tpcca_mlp_fetch(tpcca_ctx *c, float *params) {
    if (!c || !params) return TPCCA_ERR_INVALID_ARG;
    if (!c->mlp || !c->mlp_loaded) return fail(c, TPCCA_ERR_STATE, "no network loaded");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(params, c->mlp + MlpState::master, kMlpNParam * 4, hipMemcpyDeviceToHost));
    return TPCCA_OK;
}

static MlpDev mlp_dev(tpcca_ctx *c) {
    MlpDev W;
    W.w1 = (const uint16_t *)(c->mlp + MlpState::w1);
    W.w2 = (const uint16_t *)(c->mlp + MlpState::w2);
    W.w3 = (const uint16_t *)(c->mlp + MlpState::w3);
    W.b1 = (const float *)(c->mlp + MlpState::b1);
    W.b2 = (const float *)(c->mlp + MlpState::b2);
    W.b3 = (const float *)(c->mlp + MlpState::b3);
    return W;
}

tpcca_status tpcca_copy(tpcca_ctx *c, const void *src, void *dst, size_t bytes) {
    if (!c || (bytes && (!src || !dst)) || (bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
        return fail(c, TPCCA_ERR_INVALID_ARG, "copy needs 16-byte aligned buffers and a multiple of 16 bytes");
    launch_copy(src, dst, (int64_t)(bytes / 16), std::max(1, c->n_cu) * 8, c->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "copy launch");
    return TPCCA_OK;
}

tpcca_status tpcca_mlp_infer(tpcca_ctx *c, const uint16_t *x, int64_t n, float *z) {
    if (!c || n < 0 || n > 0x7fff0000 || (n > 0 && (!x || !z))) return TPCCA_ERR_INVALID_ARG;
    if (!c->mlp || !c->mlp_loaded) return fail(c, TPCCA_ERR_STATE, "no network loaded");
    if (n == 0) return TPCCA_OK;
    const int grid = (int)std::min<int64_t>((n + 63) / 64, (int64_t)c->n_cu * 8);
    launch_mlp_infer(mlp_dev(c), x, nullptr, (int32_t)n, z, grid, c->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "mlp infer launch");
    return TPCCA_OK;
}

static tpcca_status mlp_step(tpcca_ctx *c, const uint16_t *x, const float *y, int64_t n, float pos_weight,
                             const tpcca_mlp_hparams *hp, float *grad, float *loss) {
    if (!c || n < 1 || n > kMlpMaxBatch || !x || !y) return fail(c, TPCCA_ERR_INVALID_ARG, "batch of 1..8192 examples");
    if (!c->mlp || !c->mlp_loaded) return fail(c, TPCCA_ERR_STATE, "no network loaded");
    MlpTrainArgs t{};
    char *M = c->mlp;
    t.w1 = (uint16_t *)(M + MlpState::w1);
    t.w2 = (uint16_t *)(M + MlpState::w2);
    t.w3 = (uint16_t *)(M + MlpState::w3);
    t.b1 = (float *)(M + MlpState::b1);
    t.b2 = (float *)(M + MlpState::b2);
    t.b3 = (float *)(M + MlpState::b3);
    t.master = (float *)(M + MlpState::master);
    t.adam_m = (float *)(M + MlpState::adam_m);
    t.adam_v = (float *)(M + MlpState::adam_v);
    t.step = (int32_t *)(M + MlpState::step);
    t.X = x;
    t.Y = y;
    t.n = (int32_t)n;
    t.pos_weight = hp ? hp->pos_weight : pos_weight;
    if (hp) {
        if (!(hp->lr > 0) || !(hp->beta1 >= 0 && hp->beta1 < 1) || !(hp->beta2 >= 0 && hp->beta2 < 1) ||
            !(hp->eps > 0) || !(hp->weight_decay >= 0) || !(hp->pos_weight > 0))
            return fail(c, TPCCA_ERR_INVALID_ARG, "bad optimiser hyper-parameters");
        t.lr = hp->lr;
        t.beta1 = hp->beta1;
        t.beta2 = hp->beta2;
        t.eps = hp->eps;
        t.weight_decay = hp->weight_decay;
        t.update = 1;
    } else {
        if (!grad) return TPCCA_ERR_INVALID_ARG;
        t.update = 0;
        t.grad_out = grad;
    }
    t.loss_out = loss;
    launch_mlp_train(t, c->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "mlp step launch");
    return TPCCA_OK;
}

tpcca_status tpcca_mlp_grad(tpcca_ctx *c, const uint16_t *x, const float *y, int64_t n, float pos_weight, float *grad,
                            float *loss) {
    if (!(pos_weight > 0)) return fail(c, TPCCA_ERR_INVALID_ARG, "pos_weight must be > 0");
    return mlp_step(c, x, y, n, pos_weight, nullptr, grad, loss);
}

tpcca_status tpcca_mlp_train_step(tpcca_ctx *c, const uint16_t *x, const float *y, int64_t n,
                                  const tpcca_mlp_hparams *hp, float *loss) {
    if (!hp) return TPCCA_ERR_INVALID_ARG;
    return mlp_step(c, x, y, n, 0.f, hp, nullptr, loss);
}

tpcca_status tpcca_triplet_samples(tpcca_ctx *c, float keep, uint64_t seed, uint16_t *feat_dev, float *label_dev,
                                   int64_t cap, int64_t *n_out) {
    if (!c || !n_out || !(keep >= 0.f && keep <= 1.f) || cap < 0 || (cap > 0 && (!feat_dev || !label_dev)))
        return fail(c, TPCCA_ERR_INVALID_ARG, "keep in [0, 1], cap >= 0, output buffers for cap > 0");
    if (((uintptr_t)feat_dev & 15)) return fail(c, TPCCA_ERR_INVALID_ARG, "feature buffer must be 16-byte aligned");
    if (!c->have_results || !c->args.keep_pool || !c->arena)
        return fail(c, TPCCA_ERR_STATE, "no pruned run that kept its triplet pool");
    // the counter lives in the run's counters (in the arena): no allocation
    unsigned long long *cnt_dev = (unsigned long long *)(c->arena + c->lay.cnt + offsetof(Counters, n_samples));
    launch_fill_i32((int32_t *)cnt_dev, 2, 0, c->stream);
    launch_samples(c->args, keep, seed, feat_dev, label_dev, cap, cnt_dev, std::max(1, c->n_cu) * 8, c->stream);
    unsigned long long h = 0;
    HIPCHK(c, hipMemcpyAsync(&h, cnt_dev, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *n_out = (int64_t)h;
    return (int64_t)h > cap ? fail(c, TPCCA_ERR_CAPACITY, "sample buffer too small") : TPCCA_OK;
}

tpcca_status tpcca_get_triplets(tpcca_ctx *c, int32_t frame, int32_t sector, int32_t *tri, uint16_t *feat, float *z,
                                int64_t cap, int64_t *n_out) {
    if (!c || !n_out) return TPCCA_ERR_INVALID_ARG;
    int si;
    SiState st;
    tpcca_status s = locate(c, frame, sector, si, st);
    if (s != TPCCA_OK) return s;
    if (!c->args.keep_pool) return fail(c, TPCCA_ERR_STATE, "the last run was not a pruned run that kept its triplet pool");
    const int nv = st.n_valid;
    std::vector<int32_t> hoff(nv), hn1(nv), hn2(nv);
    std::vector<Rec> rec(nv);
    if (nv > 0) {
        const size_t o = (size_t)st.sbase;
        HIPCHK(c, hipMemcpy(hoff.data(), c->arena + c->lay.hoff + 4 * o, 4 * (size_t)nv, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(hn1.data(), c->arena + c->lay.hn1 + 4 * o, 4 * (size_t)nv, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(hn2.data(), c->arena + c->lay.hn2 + 4 * o, 4 * (size_t)nv, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(rec.data(), c->arena + c->lay.rec + sizeof(Rec) * o, sizeof(Rec) * (size_t)nv,
                            hipMemcpyDeviceToHost));
    }
    int64_t total = 0, lo = INT64_MAX, hi = 0;
    std::vector<int> order(nv);
    for (int p = 0; p < nv; p++) {
        order[p] = p;
        const int64_t k = (int64_t)hn1[p] + hn2[p];
        total += k;
        if (k > 0 && hoff[p] >= 0) {
            lo = std::min<int64_t>(lo, hoff[p]);
            hi = std::max<int64_t>(hi, hoff[p] + k);
        }
    }
    *n_out = total;
    if (cap < total) return fail(c, TPCCA_ERR_CAPACITY, "triplet buffer too small");
    if (total == 0) return TPCCA_OK;
    const size_t span = (size_t)(hi - lo);
    std::vector<uint16_t> pf(span * kMlpInP);
    std::vector<int32_t> pd(span), pu(span);
    std::vector<float> pz(span);
    HIPCHK(c, hipMemcpy(pf.data(), c->arena + c->lay.pfeat + 2 * kMlpInP * (size_t)lo, 2 * kMlpInP * span,
                        hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(pd.data(), c->arena + c->lay.pd + 4 * (size_t)lo, 4 * span, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(pu.data(), c->arena + c->lay.pu + 4 * (size_t)lo, 4 * span, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(pz.data(), c->arena + c->lay.pz + 4 * (size_t)lo, 4 * span, hipMemcpyDeviceToHost));
    std::sort(order.begin(), order.end(), [&](int a, int b) { return rec[a].id < rec[b].id; });
    int64_t k = 0;
    const int base = st.sbase;
    std::vector<int64_t> srcs;
    for (int p : order) {
        for (int g = 0; g < 2; g++) {
            // one gap's triplets, by (down id, up id)
            const int j0 = g ? hn1[p] : 0, j1 = g ? hn1[p] + hn2[p] : hn1[p];
            srcs.clear();
            for (int j = j0; j < j1; j++) srcs.push_back((int64_t)hoff[p] + j - lo);
            std::sort(srcs.begin(), srcs.end(), [&](int64_t u, int64_t v) {
                const int du = rec[pd[u] - base].id, dv = rec[pd[v] - base].id;
                return du < dv || (du == dv && rec[pu[u] - base].id < rec[pu[v] - base].id);
            });
            for (int64_t src : srcs) {
                if (tri) {
                    tri[4 * k] = rec[pd[src] - base].id;
                    tri[4 * k + 1] = rec[p].id;
                    tri[4 * k + 2] = rec[pu[src] - base].id;
                    tri[4 * k + 3] = g + 1;
                }
                if (feat) std::memcpy(feat + kMlpInP * k, pf.data() + kMlpInP * src, 2 * kMlpInP);
                if (z) z[k] = pz[src];
                k++;
            }
        }
    }
    return TPCCA_OK;
}

}  // extern "C"
