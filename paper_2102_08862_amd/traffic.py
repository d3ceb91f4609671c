"""HBM traffic of the tracker's kernels from hardware counters.

The counters FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are collected in
two separate rocprofv3 passes over the same workload, which ends with a plain
copy kernel (tpcca_copy) of a known size; each counter is scaled by what it
reads for that copy (bytes copied / counter value), so the figures are in
HBM bytes. The summary records a fingerprint of the kernel sources: a figure
is only valid for the kernels it was taken on.

  W="python -m paper_2102_08862_amd.traffic run"   (add --follow for the follower's kernels)
  rocprofv3 --pmc FETCH_SIZE --kernel-include-regex \\
      'k_links|k_rowsort|k_scatter|k_hist|k_lists|k_asg_fill|k_fit|k_seeds|k_walk|k_follow|k_ford|k_copy' \\
      -d OUT/fetch -o f --output-format csv -- $W
  rocprofv3 --pmc WRITE_SIZE (same options) -d OUT/write -o w --output-format csv -- $W
  python -m paper_2102_08862_amd.traffic summarize OUT/fetch OUT/write --out profiles/traffic_frame_10ms.txt
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
COPY_BYTES = 1 << 30

# kernel -> source file holding it
SOURCES = {
    "k_hist": "k_grid.hip", "k_scatter": "k_grid.hip", "k_rowsort": "k_grid.hip", "k_copy": "k_grid.hip",
    "k_tiles": "k_links.hip", "k_links": "k_links.hip", "k_select": "k_links.hip",
    "k_seeds": "k_chain.hip", "k_walk": "k_chain.hip", "k_lists": "k_chain.hip",
    "k_asg_fill": "k_chain.hip", "k_tile_list": "k_links.hip",
    "k_fit": "k_fit.hip", "k_mlp_infer": "k_mlp.hip",
    "k_follow": "k_follow.hip", "k_follow_keep": "k_follow.hip", "k_ford_hist": "k_follow.hip",
    "k_ford_scatter": "k_follow.hip", "k_follow_slots": "k_follow.hip",
}


def fingerprint(kernel: str) -> str:
    h = hashlib.sha256()
    for f in (SOURCES[kernel], "tpcca_internal.h"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(full: str) -> str:
    """Kernel name without namespace and arguments; template arguments are
    kept (spaces removed) so that instantiations stay apart."""
    m = re.search(r"(k_[a-z0-9_]+(<[^()]*>)?)", full)
    return m.group(1).replace(" ", "") if m else full


def base_name(kernel: str) -> str:
    return kernel.split("<")[0]


def run(argv):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="frame_10ms")
    ap.add_argument("--seed", type=int, default=3000)
    ap.add_argument("--runs", type=int, default=2)
    ap.add_argument("--follow", action="store_true", help="the tracker with track following")
    a = ap.parse_args(argv)
    import torch
    from . import synth, tpcca
    fr = synth.generate(a.workload, seed=a.seed, n_threads=min(16, os.cpu_count() or 1))
    trk = tpcca.Tracker(follow=1) if a.follow else tpcca.Tracker()
    trk.load_frame_packed(fr)
    trk.ensure_arena()
    trk.run(sync=True)                       # warm-up
    for _ in range(a.runs):
        trk.run()
    trk.synchronize()
    src = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    trk.copy(src, dst)
    torch.cuda.synchronize()
    print("traffic workload: %s seed %d%s, %d clusters, %d timed runs, copy %d bytes"
          % (a.workload, a.seed, " (following)" if a.follow else "", fr.n_clusters, a.runs, COPY_BYTES), flush=True)


def _read(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % d)
    per = {}
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                k = short_name(r["Kernel_Name"])
                per.setdefault(k, []).append(float(r["Counter_Value"]))
    return per


def summarize(argv):
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir")
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", default="")
    a = ap.parse_args(argv)
    fe, wr = _read(a.fetch_dir), _read(a.write_dir)
    if "k_copy" not in fe or "k_copy" not in wr:
        raise SystemExit("the copy kernel is missing from the counters")
    ff = (COPY_BYTES / 1024.0) / fe["k_copy"][-1]
    fw = (COPY_BYTES / 1024.0) / wr["k_copy"][-1]
    lines = ["# HBM traffic per dispatch from FETCH_SIZE / WRITE_SIZE (KiB), scaled by the copy kernel",
             "# copy kernel: %d bytes read and written; FETCH_SIZE %.1f KiB, WRITE_SIZE %.1f KiB"
             % (COPY_BYTES, fe["k_copy"][-1], wr["k_copy"][-1]),
             "# scale: fetch %.4f, write %.4f" % (ff, fw)]
    if a.command:
        lines.append("# command: " + a.command)
    lines.append("kernel dispatches fetch_GB write_GB traffic_GB fingerprint")
    for k in sorted(set(fe) & set(wr)):
        if k == "k_copy":
            continue
        # the first dispatch of each kernel is the warm-up run; average the rest
        f = fe[k][1:] or fe[k]
        w = wr[k][1:] or wr[k]
        fb = sum(f) / len(f) * 1024 * ff
        wb = sum(w) / len(w) * 1024 * fw
        lines.append("%s %d %.4f %.4f %.4f %s" % (k, len(f), fb / 1e9, wb / 1e9, (fb + wb) / 1e9,
                                                  fingerprint(base_name(k)) if base_name(k) in SOURCES else "-"))
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def lookup(path: str, kernel: str):
    """Traffic bytes of one launch of `kernel` (the sum over its template
    instantiations, which one launch of the stage runs once each) from a
    summary, or None if the summary is absent, lacks the kernel or was taken
    on other kernel sources."""
    if not os.path.exists(path) or kernel not in SOURCES:
        return None
    total, found = 0.0, False
    with open(path) as fh:
        for line in fh:
            p = line.split()
            if len(p) == 6 and base_name(p[0]) == kernel:
                if p[5] != fingerprint(kernel):
                    return None
                total += float(p[4]) * 1e9
                found = True
    return total if found else None


if __name__ == "__main__":
    if len(sys.argv) < 2 or sys.argv[1] not in ("run", "summarize"):
        raise SystemExit("usage: traffic.py run|summarize ...")
    (run if sys.argv[1] == "run" else summarize)(sys.argv[2:])
