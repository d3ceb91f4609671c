"""Launch-shape autotuner for the track finder.

Sweeps, stage by stage, the persistent grid size (workgroups per compute
unit) and, for neighbour finding, the tile budget (clusters a tile may stage
in LDS), timing each stage with the library's HIP events on a real frame. A
candidate is kept only if the run's outputs are bit-identical to the
reference run (the settings must not change any result). The winners are
cached in a JSON file keyed by GPU architecture and workload size bucket.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

STAGES = {            # launch index -> (timed stage, blocks-per-CU candidates, tile-budget candidates)
    1: ("hist", (2, 4, 8, 16), (0,)),
    3: ("scatter", (1, 2, 4), (0,)),
    4: ("rowsort", (1, 2, 3, 4), (0,)),
    5: ("links", (2, 3, 4), (768, 1536, 2304, 3072)),
    6: ("seeds", (2, 4, 8, 16), (0,)),
    7: ("walk", (2, 4, 8, 16), (0,)),
    10: ("fit", (2, 4, 8, 16), (0,)),     # cluster lists, on the side stream beside the fit
    11: ("fit", (2, 4, 8, 16), (0,)),
}

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def size_bucket(n_clusters: int) -> str:
    return "2^%d" % max(0, int(round(math.log2(max(1, n_clusters)))))


def _arch():
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _fingerprint(trk, frame_ids, sectors):
    h = []
    for f in frame_ids:
        for s in sectors:
            tr = trk.tracks(f, s)
            h.append(trk.assignment(f, s).tobytes())
            h.append(trk.track_clusters(f, s).tobytes())
            for k in ("y", "dt", "sinphi", "tau", "qpt", "chi2", "status"):
                h.append(tr[k].tobytes())
    return b"".join(h)


def _stage_ms(trk, reps):
    trk.set_timing(True)
    for _ in range(reps):
        trk.run()
    trk.synchronize()
    st = trk.stats()
    n = max(1, st["n_timed_runs"])
    return {k: v / n for k, v in st["stage_ms_total"].items()}


def tune(trk, frame_ids, sectors=(0, 17, 35), reps=3, log=print):
    """Tune trk in place (frames already loaded, arena attached). Returns the
    chosen settings {stage: [blocks_per_cu, param]} and the stage times."""
    trk.run(sync=True)
    ref = _fingerprint(trk, frame_ids, sectors)
    best = {}
    times = _stage_ms(trk, reps)
    for stage, (name, bpcs, params) in STAGES.items():
        cur = times[name]
        choice = None
        for bpc in bpcs:
            for prm in params:
                trk.set_launch(stage, bpc, prm)
                trk.ensure_arena()
                trk.run(sync=True)
                if _fingerprint(trk, frame_ids, sectors) != ref:
                    raise RuntimeError("launch setting %s %d/%d changed the results" % (name, bpc, prm))
                ms = _stage_ms(trk, reps)[name]
                log("  %-9s blocks/CU %2d param %4d: %.4f ms" % (name, bpc, prm, ms))
                if ms < cur * 0.98:
                    cur, choice = ms, (bpc, prm)
        if choice is not None:
            best[stage] = list(choice)
        # leave the stage at its best setting before tuning the next one
        b = best.get(stage)
        trk.set_launch(stage, *(b if b else _default(stage)))
        trk.ensure_arena()
        times = _stage_ms(trk, reps)
    return best, times


def _default(stage):
    # the library's built-in shapes
    return {1: (8, 0), 3: (1, 0), 4: (4, 0), 5: (4, 3072), 6: (8, 0), 7: (8, 0), 10: (8, 0), 11: (8, 0)}[stage]


def save(settings, n_clusters, path=DEFAULT_CACHE):
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data.setdefault(_arch(), {})[size_bucket(n_clusters)] = {str(k): v for k, v in settings.items()}
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def apply(trk, n_clusters, path=DEFAULT_CACHE):
    """Apply cached settings for this GPU and size bucket (nearest bucket of
    the same architecture). Returns the settings applied ({} if none)."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    per_arch = data.get(_arch(), {})
    if not per_arch:
        return {}
    want = int(size_bucket(n_clusters)[2:])
    key = min(per_arch, key=lambda b: abs(int(b[2:]) - want))
    settings = per_arch[key]
    for k, (bpc, prm) in settings.items():
        trk.set_launch(int(k), bpc, prm)
    return settings
