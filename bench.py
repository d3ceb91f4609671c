"""Throughput of the MI355X TPC track finder: clusters tracked per second.

One step = one pass of the whole hot path (search grid, neighbour links,
cleaning and CA chains, canonical output, iterated Kalman fit) over one whole
synthetic 10 ms Pb-Pb time frame (36 sectors, 500 collisions at 50 kHz,
~1.45e8 clusters), with the frame already resident in HBM. Prints one JSON
line (rank 0) with the throughput, the roofline position of the dominant
kernel (per-stage device times from HIP events recorded on the run's stream
over the timed region) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 vector

# Algorithmic traffic of each stage (what the method must move: each input
# read once, each output written once), bytes per unit; the unit is given by
# the function of the run's counts.
#   grid (hist + setup + scatter + rowsort): row + y + t read (9), sorted
#            SoA y, t, id written (12)                             21 B/cluster
#   links:   own (y, t) read (8; neighbour rows come through LDS), (up, dn)
#            written (8)                                            16 B/cluster
#   seeds:   links read (8), partner links gathered (8), cleaned up link
#            written (4) (cleaning fused with the seed test)        20 B/cluster
#   walk + fit: (y, t, link) per track cluster read (12), assignment
#            written (4), 128-byte track record per track           16 B/track cluster + 128 B/track
# The per-kernel figures below split the same totals over the kernels that
# move them (the grid's kernels each read or write an intermediate record).
STAGE_BYTES = {
    "hist": lambda s: 9 * s["n_clusters"],
    "scatter": lambda s: 25 * s["n_clusters"],
    "rowsort": lambda s: 32 * s["n_clusters"],
    "links": lambda s: 16 * s["n_clusters"],
    "seeds": lambda s: 20 * s["n_clusters"],
    # chain walk and copy: records gathered, copies written
    "walk": lambda s: 32 * s["n_track_clusters"],
    # the fit (the cluster lists and the assignment run beside it)
    "fit": lambda s: 16 * s["n_track_clusters"] + 128 * s["n_tracks"],
}
GRID_BYTES_PER_CLUSTER = 21
CPU_SHARE = 16               # host cores that go with one GPU
# one Kalman filter step per track cluster: helix transport ~25 flops (two
# square roots, one division), covariance transport ~60, 2-D update ~80
FIT_FLOPS_PER_CLUSTER = 170
GRID_STAGES = ("hist", "setup", "scatter", "rowsort")

# the kernel that dominates each stage (the stage's other launches are small)
STAGE_KERNEL = {"hist": "k_hist", "scatter": "k_scatter", "rowsort": "k_rowsort", "links": "k_links",
                "seeds": "k_seeds", "walk": "k_walk", "fit": "k_fit"}

WORKLOADS = {
    "frame_10ms": "whole 10 ms TPC time frame: 36 sectors x 152 rows, 500 Pb-Pb collisions at 50 kHz "
                  "(multiplicity Exp(2000) truncated at 15000, |eta|<0.9, pT=0.1+Exp(0.6) GeV), 0.5 T, "
                  "sigma 0.1 cm, 5% noise, drift time as coordinate",
    "slice_1ms": "1 ms continuous TPC slice: 36 sectors, 50 collisions, same generator",
    "batch64": "time frames of uneven length U(0.5, 10) ms (lengths from seed 4999, frames seeds 4000-4063; the "
               "first --batch-frames of the 64), 50 kHz Pb-Pb, same generator; run in sub-batches of whole frames, "
               "one HIP graph each",
}

BATCH_MAX_CLUSTERS = 1_200_000_000   # clusters per sub-batch (one run, 32-bit positions)
# The full 64-frame batch stalled on the GPU in the first run of its second
# large sub-batch; until the cause is found only these sizes run.
BATCH_SAFE_FRAMES = 16
BATCH_SAFE_LATER = 100_000_000


def batch_bench(args, log):
    """Throughput over 64 uneven frames: the frames are generated and made
    resident on the device one by one, grouped into sub-batches of whole
    frames (one tracker each, all sharing one arena and one stream, each run
    replayed from its captured HIP graph); a step runs every sub-batch."""
    import torch
    from paper_2102_08862_amd import autotune, synth, tpcca
    if args.batch_frames > BATCH_SAFE_FRAMES:
        raise SystemExit("batch64: more than %d frames is disabled: the full 64-frame batch stalled on the GPU in "
                         "the first run of its second large sub-batch and the cause is not found" % BATCH_SAFE_FRAMES)
    lens = np.random.default_rng(4999).uniform(0.5, 10.0, 64)[:args.batch_frames]
    nth = args.threads or min(16, os.cpu_count() or 1)
    stream = torch.cuda.Stream()
    groups, cur, cur_n = [], [], 0
    total = 0
    t0 = time.perf_counter()
    for i, L in enumerate(lens):
        fr = synth.generate("frame_10ms", seed=4000 + i, n_threads=nth, frame_us=1000.0 * L,
                            n_collisions=int(round(50 * L)))
        n = fr.n_clusters
        if cur and cur_n + n > BATCH_MAX_CLUSTERS:
            groups.append(cur)
            cur, cur_n = [], 0
        ns = [len(r) for r in fr.rows]
        dev = [torch.from_numpy(np.concatenate(a)).cuda() for a in (fr.rows, fr.ys, fr.ts)]
        cur.append((dev, ns))
        cur_n += n
        total += n
        del fr
        if i % 8 == 7:
            log("generated %d frames (%d clusters) in %.0f s" % (i + 1, total, time.perf_counter() - t0))
    groups.append(cur)
    sizes = [sum(int(np.sum(ns)) for _, ns in g) for g in groups]
    if any(n > BATCH_SAFE_LATER for n in sizes[1:]):
        raise SystemExit("batch64: a second sub-batch of more than %d clusters is disabled (sizes %s): such a run "
                         "stalled on the GPU and the cause is not found" % (BATCH_SAFE_LATER, sizes))
    torch.cuda.synchronize()
    trks, need = [], 0
    for g in groups:
        trk = tpcca.Tracker()
        for dev, ns in g:
            f = trk.add_frame()
            off = np.concatenate([[0], np.cumsum(ns)])
            for sct in range(len(ns)):
                a, b = int(off[sct]), int(off[sct + 1])
                trk.load_sector(f, sct, dev[0][a:b], dev[1][a:b], dev[2][a:b])
        need = max(need, trk.required_arena())
        trks.append(trk)
    arena = torch.empty(need + 4096, dtype=torch.uint8, device="cuda")
    tuning = {}
    for k, trk in enumerate(trks):
        trk.set_stream(stream)
        trk.use_arena(arena)
        if k == 0 and args.tune:
            tuning, _ = autotune.tune(trk, [0], log=log)
            autotune.save(tuning, total // max(1, len(trks)))
        elif not args.no_tuning:
            tuning = autotune.apply(trk, total // max(1, len(trks))) or tuning
        trk.use_arena(arena)
        trk.set_graph(True)
    log("%d frames, %d clusters in %d sub-batches; arena %.1f GB" % (len(lens), total, len(trks), need / 1e9))
    for w in range(max(1, args.warmup)):
        for k, trk in enumerate(trks):
            tw = time.perf_counter()
            trk.run(sync=True)
            log("warm-up %d, sub-batch %d: %.1f ms" % (w, k, 1e3 * (time.perf_counter() - tw)))
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        for trk in trks:
            trk.run()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    for trk in trks:
        trk.synchronize()
    log("timed %d steps: %.2f ms/step over %d clusters" % (args.steps, ms, total))
    return {
        "metric": "TPC clusters tracked per second (plain CA tracker, 64 uneven frames, batched, graph replay)",
        "value": round(total / (ms / 1e3), 1), "unit": "clusters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch64", "description": WORKLOADS["batch64"], "frames": len(lens),
                   "frame_ms": [round(float(x), 3) for x in lens], "clusters": int(total),
                   "sub_batches": len(trks), "parallelism": "single GPU"},
        "launch": {"graph": True, "tuning": tuning},
    }


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def sample_sectors(n_sectors: int, k: int):
    """k sectors alternating between the A side (0..17) and the C side (18..35)."""
    half = n_sectors // 2
    out = []
    for i in range(k):
        s = (i // 2) + (half if i % 2 else 0)
        if s < n_sectors and s not in out:
            out.append(s)
    return out


def gpu_sector_outputs(trk, f, secs):
    """The plain run's outputs of the listed sectors (for the parity check)."""
    out = {}
    for s in secs:
        up, dn = trk.links(f, s, cleaned=False)
        upc, dnc = trk.links(f, s, cleaned=True)
        out[s] = dict(up=up, dn=dn, upc=upc, dnc=dnc, assign=trk.assignment(f, s),
                      clusters=trk.track_clusters(f, s), tracks=trk.tracks(f, s))
    return out


# parameter parity: |gpu - oracle| <= 1e-4 max(|oracle|, floor) (floors at
# a fraction of each parameter's scale, for q/pT also the oracle's standard
# error of q/pT; dt is t minus the input time of the outermost cluster)
PARAM_FLOORS = {"y": 1.0, "dt": 1.0, "sinphi": 0.1, "tau": 0.1, "qpt": 0.1}


def sector_parity(g, ref):
    """Bit-exact integer outputs and the worst floored relative parameter
    error of one sector (GPU outputs g against the oracle's ref)."""
    exact = all(np.array_equal(g[k], ref[k]) for k in ("up", "dn", "upc", "dnc", "assign", "clusters"))
    tr = g["tracks"]
    exact = exact and len(tr) == len(ref["first"]) and np.array_equal(tr["first"], ref["first"])
    worst, excluded = 0.0, 0
    if exact and len(tr):
        fit = ref["fit"]
        ok = (tr["status"] == 0) & (fit["status"] == 0)
        excluded = int((~ok).sum())
        t_base = tr["t_base"][ok].astype(np.float64)
        pairs = {"y": (tr["y"][ok], fit["y"][ok]), "dt": (tr["dt"][ok], fit["t"][ok] - t_base),
                 "sinphi": (tr["sinphi"][ok], fit["sinphi"][ok]), "tau": (tr["tau"][ok], fit["tau"][ok]),
                 "qpt": (tr["qpt"][ok], fit["qpt"][ok])}
        floors = dict(PARAM_FLOORS)
        floors["qpt"] = np.maximum(PARAM_FLOORS["qpt"], np.sqrt(np.maximum(fit["cov"][ok][:, 14], 0.0)))
        for k, (a, b) in pairs.items():
            if len(a):
                rel = np.abs(a.astype(np.float64) - b) / np.maximum(np.abs(b), floors[k])
                worst = max(worst, float(rel.max()))
    return exact, worst, excluded


def cpu_baseline(fr, gpu_out, n_workers: int, follow_gpu=None):
    """The CPU oracle (whole path: links, cleaning, chains, MAP fit), timed on
    one sector with one thread and on n_workers sectors with one thread per
    sector; every sector it computes is compared with the GPU's outputs. With
    follow_gpu (the following tracker's outputs of the first sampled sector),
    the oracle's path with following is timed on that sector (one thread) and
    compared with them."""
    import oracle
    from paper_2102_08862_amd import synth
    x, _ = synth.geometry()
    cfg = oracle.Config(row_x=x)
    oracle.build()
    secs = sample_sectors(len(fr.rows), max(1, n_workers))
    refs = {}

    def one(s):
        row, y, t = fr.sector(s)
        refs[s] = oracle.run_sector(cfg, row, y, t)

    s0 = secs[0]
    t0 = time.perf_counter()
    one(s0)
    dt1 = time.perf_counter() - t0
    n1 = len(fr.rows[s0])
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=max(1, len(secs))) as ex:
        list(ex.map(one, secs))
    dtn = time.perf_counter() - t0
    nn = sum(len(fr.rows[s]) for s in secs)
    exact, worst, excl = True, 0.0, 0
    for s in secs:
        if s in gpu_out:
            e, w, x_ = sector_parity(gpu_out[s], refs[s])
            exact, worst, excl = exact and e, max(worst, w), excl + x_
    fol = None
    if follow_gpu is not None:
        row, y, t = fr.sector(s0)
        t0 = time.perf_counter()
        ref = oracle.run_sector(cfg, row, y, t, follow_cfg=oracle.FollowConfig())
        dtf = time.perf_counter() - t0
        g = follow_gpu
        ex = (np.array_equal(g["assign"], ref["assign"]) and np.array_equal(g["clusters"], ref["clusters"])
              and len(g["tracks"]) == len(ref["first"]) and np.array_equal(g["tracks"]["first"], ref["first"]))
        fol = {"value_1thread": n1 / dtf, "unit": "clusters/s",
               "sample": "sector %d (%d clusters), links + cleaning + chains + following + MAP fit, one thread, %.1f s"
                         % (s0, n1, dtf),
               "parity": {"assignment_lists_bit_exact": bool(ex)}}
    return {"value": nn / dtn, "unit": "clusters/s", "cores": len(secs), "kind": "oracle", "follow": fol,
            "value_1thread": n1 / dt1, "host_cores": host_cores(), "cpu_model": cpu_model(),
            "sample": "sectors %s of the same frame (%d clusters), links + cleaning + chains + MAP fit, one thread "
                      "per sector, %.1f s; 1-thread figure: sector %d (%d clusters, %.1f s)"
                      % (secs, nn, dtn, s0, n1, dt1),
            "parity": {"sectors": secs, "links_assignment_lists_bit_exact": bool(exact),
                       "params_worst_floored_rel": worst, "params_tol": 1e-4, "params_ok": bool(worst <= 1e-4),
                       "fit_excluded": excl}}


def fit_pass_summary(st):
    """Tracks by the number of Kalman passes their fit took (k = 1..14, the
    last bin 15 or more), the mean, and the fits restarted about the
    three-point helix."""
    h = st["fit_passes"]
    n = sum(h[1:])
    mean = sum(k * v for k, v in enumerate(h)) / max(1, n)
    return {"hist": {str(k): int(v) for k, v in enumerate(h) if k and v}, "mean": round(mean, 4),
            "restarts": int(st["n_fit_restarts"])}


def frame_quality(trk, fr, f):
    from paper_2102_08862_amd import metrics
    return metrics.frame_quality(fr, lambda s: trk.track_clusters(f, s), lambda s: trk.tracks(f, s)["n_clusters"])


def pruned_leg(trk, fr, f, args, log, q_plain):
    """The MLP-pruned tracker on the same frame, at the trained network's
    threshold, timed like the plain one; with the efficiency of both against
    the generator's truth."""
    import torch
    from paper_2102_08862_amd import prune_train
    params, meta = prune_train.load_weights()
    if params is None or "theta" not in meta:
        log("pruned leg skipped: no trained weights")
        return {"skipped": "no trained weights"}
    theta = float(meta["theta"])
    trk.set_graph(False)
    trk.mlp_load(params)
    trk.set_pruning(True, theta)
    trk.ensure_arena()
    for _ in range(max(1, args.warmup)):
        trk.run()
    trk.synchronize()
    trk.set_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(trk.stream)
    for _ in range(args.steps):
        trk.run()
    e1.record(trk.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    st = trk.stats()
    runs = max(1, st["n_timed_runs"])
    out = {"value": round(fr.n_clusters / (ms / 1e3), 1), "unit": "clusters/s", "ms_per_step": round(ms, 4),
           "theta": theta, "triplets_scored": int(st["n_triplets"]), "pruned": int(st["n_pruned"]),
           "pruned_fraction_of_scored": round(st["n_pruned"] / max(1, st["n_triplets"]), 4),
           "pool_overflow": int(st["n_pool_overflow"]),
           "stage_ms": {k: round(v / runs, 4) for k, v in st["stage_ms_total"].items()}}
    log("pruned: %.3f ms/step, %d triplets scored, %.1f%% pruned"
        % (ms, out["triplets_scored"], 100 * out["pruned_fraction_of_scored"]))
    if q_plain is not None:
        q = frame_quality(trk, fr, f)
        out["efficiency_plain"] = round(q_plain["efficiency"], 6)
        out["efficiency_pruned"] = round(q["efficiency"], 6)
        out["efficiency_loss"] = round(q_plain["efficiency"] - q["efficiency"], 6)
        out["fake_rate_plain"] = round(q_plain["fake_rate"], 6)
        out["fake_rate_pruned"] = round(q["fake_rate"], 6)
        log("efficiency plain %.5f pruned %.5f (loss %.5f); fake %.5f -> %.5f"
            % (q_plain["efficiency"], q["efficiency"], out["efficiency_loss"], q_plain["fake_rate"], q["fake_rate"]))
    trk.set_pruning(False)
    return out


def remove_leg(trk, fr, f, log, quality=True, pt_min=0.15):
    """Removal of the clusters of fitted tracks below pt_min after the plain
    run: the time of remove_clusters (wall clock; it synchronises, two
    passes over the assignment) and the share of the frame removed; against
    the generator's truth, the share of the removed clusters that belong to
    particles above pt_min. Then the entropy reduction: the time of the
    symbol histograms and the order-0 bits per track cluster of (row, y, t)
    coded as first differences and as track-model residuals; and the rANS
    bytes of every sector (wall clock of the 36 calls, host round trips
    included)."""
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        kept = trk.remove_clusters(pt_min)
        ts.append(time.perf_counter() - t0)
    n = fr.n_clusters
    out = {"pt_min_gev": pt_min, "ms": round(1e3 * float(np.median(ts)), 4), "kept": int(kept.numel()),
           "removed_share": round(1.0 - kept.numel() / max(n, 1), 5)}
    if quality:
        k = kept.cpu().numpy()
        pt = fr.tracks[:, 1]
        removed = high = 0
        for s in range(len(fr.rows)):
            b, c = trk.removal_range(f, s)
            keep = np.zeros(len(fr.rows[s]), bool)
            keep[k[b:b + c]] = True
            lab = fr.labels[s]
            removed += int((~keep).sum())
            high += int((~keep & (lab >= 0) & (pt[np.maximum(lab, 0)] >= pt_min)).sum())
        out["removed_above_pt_min"] = round(high / max(removed, 1), 5)
    # entropy reduction of the track clusters' properties (order-0 entropy of
    # the symbol histograms, an escape costing 32 bits more)
    te = []
    for _ in range(5):
        t0 = time.perf_counter()
        h = trk.entropy_histograms()
        te.append(time.perf_counter() - t0)
    n_sym = max(int(h[0].sum()), 1)
    bits = []
    for k in range(h.shape[0]):
        c = h[k][h[k] > 0].astype(np.float64)
        bits.append(float(-(c * np.log2(c / c.sum())).sum() + 32.0 * h[k][-1]) / n_sym)
    out["entropy_ms"] = round(1e3 * float(np.median(te)), 4)
    out["bits_per_cluster_first_diff"] = round(bits[0] + bits[1] + bits[2], 4)
    out["bits_per_cluster_track_model"] = round(bits[0] + bits[3] + bits[4], 4)
    # rANS coding of every sector's track clusters (per-sector models)
    t0 = time.perf_counter()
    n_bytes = 0
    for s in range(len(fr.rows)):
        data, _ = trk.ans_encode(f, s)
        n_bytes += int(data.numel())
    out["ans_ms_all_sectors"] = round(1e3 * (time.perf_counter() - t0), 3)
    out["ans_bits_per_track_cluster"] = round(8.0 * n_bytes / max(int(h[0].sum()) + len(fr.rows), 1), 4)
    log("remove: %.2f%% of the clusters removed in %.3f ms; %s" % (
        100.0 * out["removed_share"], out["ms"], {k_: out[k_] for k_ in ("removed_above_pt_min", "entropy_ms",
                                                                        "bits_per_cluster_first_diff",
                                                                        "bits_per_cluster_track_model",
                                                                        "ans_ms_all_sectors",
                                                                        "ans_bits_per_track_cluster") if k_ in out}))
    return out


def collisions_leg(trk, fr, f, log, quality=True):
    """Collision candidates after the plain run: the time of
    find_collisions (wall clock; it synchronises, with two host round trips)
    and, against the generator's truth, the candidates' quality per side."""
    from paper_2102_08862_amd import metrics
    gap, min_len, window = 0.5, 60, 5.0
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        n_groups = trk.find_collisions(gap, min_len, window)
        ts.append(time.perf_counter() - t0)
    out = {"gap_cm": gap, "min_clusters": min_len, "window_cm": window, "groups": int(n_groups),
           "ms": round(1e3 * float(np.median(ts)), 4)}
    if quality:
        half = len(fr.rows) // 2
        tc = fr.tracks[:, 5]
        for side, name in ((0, "A"), (1, "C")):
            cols = [[], [], [], []]
            for s in (range(half) if side == 0 else range(half, len(fr.rows))):
                t0, g = trk.track_times(f, s)
                tr = trk.tracks(f, s)
                pm = metrics.track_majority(fr.labels[s], trk.track_clusters(f, s), tr["n_clusters"])
                for c, v in zip(cols, (np.where(pm >= 0, tc[np.maximum(pm, 0)], -1.0), g, tr["n_clusters"],
                                       np.isfinite(t0))):
                    c.append(v)
            q = metrics.collision_quality(*(np.concatenate(c) for c in cols), min_len)
            out[name] = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in q.items()}
    log("collisions: %d groups in %.3f ms; %s" % (out["groups"], out["ms"],
                                                 {k: out[k] for k in ("A", "C") if k in out}))
    return out


def merge_leg(trk, fr, f, log, quality=True):
    """Sector merging after the plain run: the time of merge_sectors and of
    the global refit of the merged pairs (wall clock; both synchronise) and,
    against the generator's truth, the share of merged pairs that join one
    particle's segments (purity), of the particles with long segments in two
    adjacent sectors that are joined (efficiency), and the median q/pT error
    of the first piece alone and of the refit; then the membrane merging
    (sector k with k + 18), timed and scored the same way."""
    from paper_2102_08862_amd import metrics
    min_len, window, cut = 30, 8.0, 25.0
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        n_pairs = trk.merge_sectors(min_len, window, cut)
        ts.append(time.perf_counter() - t0)
    out = {"min_clusters": min_len, "window_cm": window, "d2_cut": cut, "pairs": int(n_pairs),
           "ms": round(1e3 * float(np.median(ts)), 4)}
    # the global refit of the merged pairs (wall clock; it synchronises)
    tr_ = []
    for _ in range(5):
        t0 = time.perf_counter()
        n_ref = trk.refit_merged()
        tr_.append(time.perf_counter() - t0)
    out["refit_ms"] = round(1e3 * float(np.median(tr_)), 4)
    out["refits"] = int(n_ref)
    # membrane merging (sector k with k + 18; wall clock, it synchronises)
    tm_ = []
    for _ in range(5):
        t0 = time.perf_counter()
        n_mem = trk.merge_membrane(min_len, 30.0, cut)
        tm_.append(time.perf_counter() - t0)
    out["membrane_ms"] = round(1e3 * float(np.median(tm_)), 4)
    out["membrane_pairs"] = int(n_mem)
    trk.refit_merged()   # the refit placed after the membrane merges, so both hold
    if quality:
        ns = len(fr.rows)
        half = ns // 2
        P = {}
        for s in range(ns):
            tr = trk.tracks(f, s)
            P[s] = (metrics.track_majority(fr.labels[s], trk.track_clusters(f, s), tr["n_clusters"]), tr)
        good = bad = opp = 0
        dq_piece, dq_refit = [], []
        for s in range(ns):
            side, k = divmod(s, half)
            n = side * half + (k + 1) % half
            (pa, ta), (pb, tb) = P[s], P[n]
            nxt, _ = trk.merges(f, s)
            rf, rfi, _ = trk.refits(f, s)
            for k_, i in enumerate(rfi):
                if pa[i] >= 0 and ta["status"][i] == 0 and rf["status"][k_] == 0:
                    q = fr.tracks[pa[i]][0] / fr.tracks[pa[i]][1]
                    dq_piece.append(abs(float(ta["qpt"][i]) - q))
                    dq_refit.append(abs(float(rf["qpt"][k_]) - q))
            for i, j in enumerate(nxt):
                if j >= 0:
                    good += int(pa[i] >= 0 and pa[i] == pb[j])
                    bad += int(not (pa[i] >= 0 and pa[i] == pb[j]))
            ea = (ta["status"] == 0) & (ta["n_clusters"] >= min_len)
            eb = (tb["status"] == 0) & (tb["n_clusters"] >= min_len)
            opp += len(set(pa[ea][pa[ea] >= 0]) & set(pb[eb][pb[eb] >= 0]))
        out["purity"] = round(good / max(good + bad, 1), 5)
        out["efficiency"] = round(good / max(opp, 1), 5)
        mg = mb = mo = 0
        for k in range(half):
            (pa, ta), (pb, tb) = P[k], P[k + half]
            for i, j in enumerate(trk.membrane_merges(f, k)):
                if j >= 0:
                    ok = pa[i] >= 0 and pa[i] == pb[j]
                    mg += int(ok)
                    mb += int(not ok)
            ea = (ta["status"] == 0) & (ta["n_clusters"] >= min_len)
            eb = (tb["status"] == 0) & (tb["n_clusters"] >= min_len)
            mo += len(set(pa[ea][pa[ea] >= 0]) & set(pb[eb][pb[eb] >= 0]))
        out["membrane_purity"] = round(mg / max(mg + mb, 1), 5)
        out["membrane_efficiency"] = round(mg / max(mo, 1), 5)
        # q/pT resolution against truth: first piece alone vs the refit
        if dq_refit:
            out["median_dqpt_piece"] = round(float(np.median(dq_piece)), 5)
            out["median_dqpt_refit"] = round(float(np.median(dq_refit)), 5)
    log("merge: %d pairs in %.3f ms, refit %.3f ms, membrane %d pairs in %.3f ms; %s" % (
        out["pairs"], out["ms"], out["refit_ms"], out["membrane_pairs"], out["membrane_ms"],
        {k: out[k] for k in ("purity", "efficiency", "median_dqpt_piece", "median_dqpt_refit", "membrane_purity",
                             "membrane_efficiency") if k in out}))
    return out


def follow_leg(fr, args, log, q_plain, tuning_on, sector):
    """The tracker with track following (chain extension and shared-cluster
    selection before the fit) on the same frame, timed like the plain one;
    with its quality against the generator's truth beside the plain
    tracker's, and one sector's outputs for the oracle comparison."""
    import torch
    from paper_2102_08862_amd import autotune, tpcca
    trk = tpcca.Tracker(follow=1)
    f = trk.load_frame_packed(fr)
    need = trk.ensure_arena()
    if tuning_on:
        autotune.apply(trk, fr.n_clusters)
        need = trk.ensure_arena()
    for _ in range(max(1, args.warmup)):
        trk.run()
    trk.synchronize()
    trk.set_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(trk.stream)
    for _ in range(args.steps):
        trk.run()
    e1.record(trk.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    st = trk.stats()
    runs = max(1, st["n_timed_runs"])
    out = {"value": round(fr.n_clusters / (ms / 1e3), 1), "unit": "clusters/s", "ms_per_step": round(ms, 4),
           "chains": int(st["n_chains"]), "tracks": int(st["n_tracks"]),
           "track_clusters": int(st["n_track_clusters"]), "clusters_added": int(st["n_follow_added"]),
           "chains_dropped": int(st["n_follow_dropped"]), "arena_GB": round(need / 1e9, 3),
           "stage_ms": {k: round(v / runs, 4) for k, v in st["stage_ms_total"].items()}}
    log("follow: %.3f ms/step (follow stage %.3f ms), %d chains -> %d tracks, %d clusters added"
        % (ms, out["stage_ms"].get("follow", 0.0), out["chains"], out["tracks"], out["clusters_added"]))
    if q_plain is not None:
        q = frame_quality(trk, fr, f)
        out["quality"] = {k: {"plain": round(q_plain[k], 6), "follow": round(q[k], 6)}
                          for k in ("efficiency", "fake_rate", "clone_rate", "hit_efficiency")}
        log("quality plain -> follow: %s" % out["quality"])
    g = None
    if sector is not None:
        g = dict(assign=trk.assignment(f, sector), clusters=trk.track_clusters(f, sector),
                 tracks=trk.tracks(f, sector))
    del trk
    torch.cuda.empty_cache()
    return out, g


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="frame_10ms", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=3000)
    ap.add_argument("--cpu-sectors", type=int, default=-1,
                    help="oracle sample: sectors timed in parallel, one thread each (-1: host cores, 0: skip)")
    ap.add_argument("--threads", type=int, default=0, help="generator threads (0: auto)")
    ap.add_argument("--tune", action="store_true", help="autotune launch shapes on this frame first (and cache)")
    ap.add_argument("--no-tuning", action="store_true", help="ignore the cached launch shapes")
    ap.add_argument("--graph", action="store_true", help="replay each step from a captured HIP graph")
    ap.add_argument("--no-pruned", action="store_true", help="skip the MLP-pruned tracker leg")
    ap.add_argument("--no-quality", action="store_true", help="skip the truth-based efficiency of both trackers")
    ap.add_argument("--no-follow", action="store_true", help="skip the track-following tracker leg")
    # the full 64-frame batch stalled in its second sub-batch on the GPU (cause
    # not found; see the design notes): the default runs the first 16 frames
    ap.add_argument("--batch-frames", type=int, default=16, help="batch64: use only the first N frames")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(frames and sectors are independent; see the sharding notes). Use --gpus 1.")
        sys.exit(2)

    import torch
    from paper_2102_08862_amd import synth, tpcca

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "batch64":
        print(json.dumps(batch_bench(args, log)), flush=True)
        return
    t0 = time.perf_counter()
    nth = args.threads or min(16, os.cpu_count() or 1)
    fr = synth.generate(args.workload, seed=args.seed, n_threads=nth)
    log("generated %s seed %d: %d clusters, %d particles in %.1f s"
        % (args.workload, args.seed, fr.n_clusters, len(fr.tracks), time.perf_counter() - t0))

    from paper_2102_08862_amd import autotune
    trk = tpcca.Tracker()
    th = time.perf_counter()
    f = trk.load_frame_packed(fr)
    h2d_s = time.perf_counter() - th
    need = trk.ensure_arena()
    log("inputs resident in HBM (%.2f GB H2D in %.2f s); arena %.2f GB"
        % (fr.n_clusters * 9 / 1e9, h2d_s, need / 1e9))
    tuning = {}
    if args.tune:
        log("autotuning launch shapes ...")
        tuning, _ = autotune.tune(trk, [f], log=log)
        autotune.save(tuning, fr.n_clusters)
        log("tuned: %s" % tuning)
    elif not args.no_tuning:
        tuning = autotune.apply(trk, fr.n_clusters)
        if tuning:
            log("cached launch shapes: %s" % tuning)
    trk.ensure_arena()
    if args.graph:
        trk.set_graph(True)

    for _ in range(args.warmup):
        trk.run()
    trk.synchronize()
    log("warmup done (%d steps)" % args.warmup)
    trk.set_timing(True)
    stream = trk.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        trk.run()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = ev[0].elapsed_time(ev[-1]) / args.steps
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    st = trk.stats()
    log("timed %d steps: %.3f ms/step (median %.3f, min %.3f, max %.3f; wall %.3f ms/step)"
        % (args.steps, ms, np.median(step_ms), step_ms.min(), step_ms.max(), 1e3 * wall / args.steps))

    n = fr.n_clusters
    runs = max(1, st["n_timed_runs"])
    stage = {k: v / runs for k, v in st["stage_ms_total"].items()}
    if args.graph:
        # graph replays record no per-stage events: time the stages in eager runs
        trk.set_graph(False)
        trk.set_timing(True)
        for _ in range(min(args.steps, 5)):
            trk.run()
        trk.synchronize()
        st2 = trk.stats()
        stage = {k: v / max(1, st2["n_timed_runs"]) for k, v in st2["stage_ms_total"].items()}
    table = {}
    for k, v in stage.items():
        row = {"ms": round(v, 4)}
        if k in STAGE_BYTES and v > 0:
            b = STAGE_BYTES[k](st)
            row["alg_GB"] = round(b / 1e9, 4)
            row["GB_s"] = round(b / 1e9 / (v / 1e3), 1)
        table[k] = row
    grid_ms = sum(stage.get(k, 0.0) for k in GRID_STAGES)
    if grid_ms > 0:
        gb = GRID_BYTES_PER_CLUSTER * st["n_clusters"]
        table["grid_total"] = {"ms": round(grid_ms, 4), "alg_GB": round(gb / 1e9, 4),
                               "GB_s": round(gb / 1e9 / (grid_ms / 1e3), 1)}
    for k, v in table.items():
        log("  %-9s %s" % (k, v))
    dom = max((k for k in stage if k in STAGE_BYTES), key=lambda k: stage[k])
    from paper_2102_08862_amd import traffic as trf
    kname = STAGE_KERNEL.get(dom)
    tb = trf.lookup(os.path.join(ROOT, "profiles", "traffic_%s.txt" % args.workload), kname) if kname else None
    if dom == "fit":
        # the Kalman fit is bound by FP32 vector issue: algorithmic flops per
        # track cluster of one filter pass against the FP32 vector peak
        fl = FIT_FLOPS_PER_CLUSTER * st["n_track_clusters"]
        achieved = fl / 1e12 / (stage[dom] / 1e3)
        roof = {"kernel": kname, "bound": "alu", "achieved": round(achieved, 2), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": round(tb) if tb else None,
                "flops_per_launch": int(fl), "avg_ms": round(stage[dom], 4)}
    else:
        b = STAGE_BYTES[dom](st)
        achieved = b / 1e9 / (stage[dom] / 1e3)
        roof = {"kernel": kname or dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": round(tb) if tb else None,
                "bytes_per_launch": int(b), "avg_ms": round(stage[dom], 4)}

    # the machine's CPU share for one GPU is 16 cores, whatever the host shows
    ncpu = min(host_cores(), CPU_SHARE) if args.cpu_sectors < 0 else min(args.cpu_sectors, 36)
    gpu_out = gpu_sector_outputs(trk, f, sample_sectors(len(fr.rows), max(1, ncpu))) if ncpu > 0 else {}

    q_plain = None if args.no_quality else frame_quality(trk, fr, f)
    collisions = collisions_leg(trk, fr, f, log, quality=not args.no_quality)
    merge = merge_leg(trk, fr, f, log, quality=not args.no_quality)
    remove = remove_leg(trk, fr, f, log, quality=not args.no_quality)
    pruned = None
    if not args.no_pruned:
        pruned = pruned_leg(trk, fr, f, args, log, q_plain)
    follow, follow_gpu = None, None
    if not args.no_follow:
        follow, follow_gpu = follow_leg(fr, args, log, q_plain, not args.no_tuning,
                                        sample_sectors(len(fr.rows), 1)[0] if ncpu > 0 else None)

    cpu = None
    if ncpu > 0:
        log("cpu baseline: oracle on 1 sector (1 thread), then %d sectors (%d threads) ..." % (ncpu, ncpu))
        cpu = cpu_baseline(fr, gpu_out, ncpu, follow_gpu)
        log("cpu baseline: %.3g clusters/s (%d threads), %.3g clusters/s (1 thread); parity %s"
            % (cpu["value"], cpu["cores"], cpu["value_1thread"], cpu["parity"]))

    out = {
        "metric": "TPC clusters tracked per second (plain CA tracker, whole 10 ms frame resident in HBM)",
        "value": round(n / (ms / 1e3), 1),
        "unit": "clusters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "seed": args.seed,
                   "clusters": n, "tracks": int(st["n_tracks"]), "track_clusters": int(st["n_track_clusters"]),
                   "parallelism": "single GPU"},
        "roofline": roof,
        "pruned": pruned,
        "follow": follow,
        "collisions": collisions,
        "merge": merge,
        "remove": remove,
        "cpu_baseline": cpu,
        "counts": {k: int(st[k]) for k in ("n_links", "n_seeds", "n_tracks", "n_track_clusters", "n_invalid",
                                            "n_overflow_tiles", "n_tiles")},
        "stage_ms": {k: round(v, 4) for k, v in stage.items()},
        "step_ms": {"median": round(float(np.median(step_ms)), 4), "min": round(float(step_ms.min()), 4),
                    "max": round(float(step_ms.max()), 4), "n": int(args.steps)},
        "stage_GB_s": {k: v["GB_s"] for k, v in table.items() if "GB_s" in v},
        "fit_passes": fit_pass_summary(st),
        "h2d_s": round(h2d_s, 3),
        "launch": {"graph": bool(args.graph), "tuning": tuning},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
