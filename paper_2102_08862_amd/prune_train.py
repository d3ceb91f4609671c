"""Learned triplet pruning: training data, GPU training, threshold choice and
the gain test.

The paper names machine-learning methods as a direction for reconstruction
(Sec. 1 and Sec. 5) but specifies no network, features or training; the
choices here are this project's:

  - data: candidate triplets (down, cluster, up) of the neighbour finder,
    enumerated by a pruned run with the threshold at -inf (the links are then
    the plain finder's), with their 12 BF16 features computed on the GPU;
  - label: 1 if the plain tracker's cleaned links put `down` directly below
    and `up` directly above `cluster` and `cluster` sits on a track, else 0;
  - sampling: a uniform random share of every training frame's triplets
    (stratified by frame), kept and labelled on the device;
  - loss: binary cross-entropy on the logit, positives weighted by
    N_neg / N_pos; optimiser AdamW (lr 1e-3, betas 0.9/0.999, weight decay
    1e-4), batch 4096, FP32 master weights with BF16 copies, all on the GPU
    through the library's own forward/backward/update kernel;
  - threshold: the largest logit threshold whose efficiency loss against the
    plain tracker on held-out frames is at most 0.004 (absolute), measured
    against the generator's truth;
  - gain test: at that threshold, on 10 ms frames, the pruned tracker against
    the plain tracker, a tighter pair cut that prunes the same share of
    triplets, and an untrained network at the same share.

Run as a module: python -m paper_2102_08862_amd.prune_train --help
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import metrics, synth, tpcca

NPARAM = tpcca.MLP_NPARAM
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "prune_mlp.json")

TRAIN_SEEDS = (2000, 2200)     # 1 ms slices used for training
VAL_SEEDS = (2200, 2220)       # held-out 1 ms slices for the threshold
EVAL_SEEDS = (3000, 3010)      # 10 ms frames for the gain test


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ network
def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, in the library's flat order
    (w1[64][16] with input columns 12..15 zero, b1, w2[64][64], b2, w3, b3)."""
    rng = np.random.default_rng(seed)
    w1 = np.zeros((64, 16))
    w1[:, :12] = rng.normal(0.0, math.sqrt(2.0 / 12), (64, 12))
    w2 = rng.normal(0.0, math.sqrt(2.0 / 64), (64, 64))
    w3 = rng.normal(0.0, math.sqrt(1.0 / 64), 64)
    flat = np.concatenate([w1.ravel(), np.zeros(64), w2.ravel(), np.zeros(64), w3, [0.0]])
    assert flat.size == NPARAM
    return flat.astype(np.float32)


def save_weights(params, meta, path=WEIGHTS):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump({"meta": meta, "params": [float(v) for v in np.asarray(params, np.float32)]}, f)


REPORT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "prune_gain_report.json")


def load_report(path=REPORT):
    """The training and gain-test report written next to the weights."""
    with open(path) as f:
        return json.load(f)


def load_weights(path=WEIGHTS):
    """(params float32[5313], meta dict) or (None, None) if absent or invalid."""
    try:
        with open(path) as f:
            d = json.load(f)
        p = np.asarray(d["params"], np.float32)
        if p.size != NPARAM or not np.all(np.isfinite(p)):
            return None, None
        return p, d.get("meta", {})
    except (OSError, ValueError, KeyError):
        return None, None


# ------------------------------------------------------------------ data
def triplet_labels(tri, up_clean, dn_clean, assign):
    """tri int32[n, 4] = (down, cluster, up, gap) input indices."""
    d, i, u = tri[:, 0], tri[:, 1], tri[:, 2]
    return ((dn_clean[i] == d) & (up_clean[i] == u) & (assign[i] >= 0)).astype(np.float32)


def frame_triplets(trk, f, n_sectors, keep, rng):
    """Features and labels of a share `keep` of the triplets of frame f
    (after a pruned run with the threshold at -inf)."""
    xs, ys, n_all, n_pos = [], [], 0, 0
    for s in range(n_sectors):
        tri, feat, _ = trk.triplets(f, s)
        if len(tri) == 0:
            continue
        up, dn = trk.links(f, s, cleaned=True)
        lab = triplet_labels(tri, up, dn, trk.assignment(f, s))
        n_all += len(lab)
        n_pos += int(lab.sum())
        m = rng.random(len(lab)) < keep
        xs.append(feat[m])
        ys.append(lab[m])
    return np.concatenate(xs), np.concatenate(ys), n_all, n_pos


def prefetch(workload, seeds, n_threads):
    """Generate frames in a background thread, one ahead of use."""
    ex = ThreadPoolExecutor(max_workers=1)
    fut = None
    for k, sd in enumerate(seeds):
        if fut is None:
            fut = ex.submit(synth.generate, workload, sd, n_threads)
        fr = fut.result()
        fut = ex.submit(synth.generate, workload, seeds[k + 1], n_threads) if k + 1 < len(seeds) else None
        yield sd, fr
    ex.shutdown()


def collect(trk, seeds, per_frame, seed, n_threads):
    """Training set from the given 1 ms slice seeds, sampled and labelled on
    the device: returns device tensors (feat int16 [m, 16], label float [m])
    and counts (triplets seen, positives among the kept)."""
    import torch
    X, Y, tot = [], [], 0
    trk.set_pruning(True, -1e30)
    for sd, fr in prefetch("slice_1ms", seeds, n_threads):
        trk.clear_frames()
        trk.load_frame_packed(fr)
        trk.run(sync=True)
        st = trk.stats()
        if st["n_pool_overflow"]:
            raise RuntimeError("triplet pool overflow on seed %d" % sd)
        n_all = max(1, st["n_triplets"])
        keep = min(1.0, per_frame / n_all)
        x, y = trk.triplet_samples(keep, seed * 1000003 + sd, int(per_frame * 1.2) + 4096)
        X.append(x.clone())
        Y.append(y.clone())
        tot += n_all
        log("  seed %d: %d clusters, %d triplets (%.2f per cluster), kept %d (%.1f%% positive)"
            % (sd, fr.n_clusters, n_all, n_all / max(1, fr.n_clusters), len(y), 100.0 * float(y.mean().item())))
    X = torch.cat(X)
    Y = torch.cat(Y)
    return X, Y, tot, int(Y.sum().item())


# ------------------------------------------------------------------ training
def to_device(feat, lab):
    import torch
    x = torch.from_numpy(np.ascontiguousarray(feat).view(np.int16)).cuda()
    y = torch.from_numpy(np.ascontiguousarray(lab, np.float32)).cuda()
    return x, y


def train(trk, x, y, epochs=5, batch=4096, lr=1e-3, weight_decay=1e-4, seed=0, pos_weight=None, every=1000):
    """AdamW epochs over device tensors x (int16 [m, 16] BF16 bits) and
    y (float [m]). Returns the loss history [(step, mean batch loss)]."""
    import torch
    m = x.shape[0]
    if pos_weight is None:
        npos = float(y.sum().item())
        pos_weight = (m - npos) / max(1.0, npos)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    loss = torch.zeros(1, device="cuda")
    acc = torch.zeros(1, device="cuda")
    hist, step, t0 = [], 0, time.perf_counter()
    nb = m // batch
    for ep in range(epochs):
        perm = torch.randperm(m, device="cuda", generator=g)
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            trk.mlp_train_step(x[idx].contiguous(), y[idx].contiguous(), lr=lr, weight_decay=weight_decay,
                               pos_weight=pos_weight, loss_dev=loss)
            acc += loss
            step += 1
            if step % every == 0:
                v = acc.item() / every
                acc.zero_()
                hist.append((step, v))
                log("  epoch %d step %d: loss %.5f (%.1f s)" % (ep, step, v, time.perf_counter() - t0))
    torch.cuda.synchronize()
    return hist, pos_weight


def logits(trk, x, chunk=1 << 22):
    import torch
    out = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
    for a in range(0, x.shape[0], chunk):
        trk.mlp_infer(x[a:a + chunk], out[a:a + chunk])
    return out


def bce(z, y, pos_weight):
    """Mean weighted binary cross-entropy of logits (evaluation only)."""
    import torch
    sp = torch.nn.functional.softplus
    return float((pos_weight * y * sp(-z) + (1 - y) * sp(z)).mean().item())


# ------------------------------------------------------------------ evaluation
class FrameSet:
    """Frames kept in host memory and run one at a time through a tracker;
    quality is measured against the generator's truth."""

    def __init__(self, workload, seeds, n_threads):
        self.frames = [fr for _, fr in prefetch(workload, list(seeds), n_threads)]
        self.n_clusters = sum(fr.n_clusters for fr in self.frames)

    def evaluate(self, trk, timing=False, quality=True):
        counts, trip, pruned, ms, tlen = [], 0, 0, 0.0, []
        for fr in self.frames:
            trk.clear_frames()
            f = trk.load_frame_packed(fr)
            trk.ensure_arena()
            if timing:
                trk.run(sync=True)      # warm-up after a new load
                trk.set_timing(True)
            trk.run(sync=True)
            st = trk.stats()
            if st["n_pool_overflow"]:
                raise RuntimeError("triplet pool overflow")
            trip += st["n_triplets"]
            pruned += st["n_pruned"]
            if timing:
                ms += sum(st["stage_ms_total"].values()) / max(1, st["n_timed_runs"])
            for s in range(len(fr.rows) if quality else 0):
                tr = trk.tracks(f, s)
                tlen.append(tr["n_clusters"])
                counts.append(metrics.sector_counts(fr.labels[s], trk.track_clusters(f, s), tr["n_clusters"]))
        q = metrics.summarize(counts) if counts else {}
        tl = np.concatenate(tlen) if tlen else np.zeros(0)
        q["mean_track_length"] = float(tl.mean()) if len(tl) else 0.0
        q["triplets"] = int(trip)
        q["pruned"] = int(pruned)
        q["pruned_fraction"] = pruned / max(1, trip)
        if timing:
            q["device_ms"] = ms
            q["clusters_per_s"] = self.n_clusters / (ms / 1e3) if ms > 0 else None
        return q


def select_theta(trk, vset, z_sample, max_loss=0.004, log=log):
    """Largest threshold with efficiency loss <= max_loss on the frame set:
    a scan over quantiles of the triplet logits, then bisection."""
    trk.set_pruning(False)
    base = vset.evaluate(trk)
    log("  plain: eff %.5f fake %.5f" % (base["efficiency"], base["fake_rate"]))
    zs = np.sort(z_sample)
    ok_t, ok_q, bad_t = -1e30, None, None
    for frac in (0.05, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7):
        th = float(zs[int(frac * (len(zs) - 1))])
        trk.set_pruning(True, th)
        q = vset.evaluate(trk)
        loss = base["efficiency"] - q["efficiency"]
        log("  theta %.4f (logit quantile %.2f): pruned %.3f eff %.5f (loss %.5f) fake %.5f"
            % (th, frac, q["pruned_fraction"], q["efficiency"], loss, q["fake_rate"]))
        if loss <= max_loss:
            ok_t, ok_q = th, q
        else:
            bad_t = th
            break
    if bad_t is not None and ok_q is not None:
        lo, hi = ok_t, bad_t
        for _ in range(5):
            mid = 0.5 * (lo + hi)
            trk.set_pruning(True, mid)
            q = vset.evaluate(trk)
            loss = base["efficiency"] - q["efficiency"]
            log("  theta %.4f: pruned %.3f eff %.5f (loss %.5f)" % (mid, q["pruned_fraction"], q["efficiency"], loss))
            if loss <= max_loss:
                lo, ok_q = mid, q
            else:
                hi = mid
        ok_t = lo
    return ok_t, base, ok_q


def matched_pair_cut(make_tracker, vset, target_fraction, base_c2=0.2, log=log):
    import torch
    """Tighter pair cut C2' whose accepted triplets are (1 - target_fraction)
    of those at base_c2, by bisection; counts come from pruned runs with the
    threshold at -inf (enumeration only)."""
    def count(c2):
        t = make_tracker(pair_c2=c2)
        t.mlp_load(init_params(0))
        t.set_pruning(True, -1e30)
        n = vset.evaluate(t, quality=False)["triplets"]
        del t
        torch.cuda.empty_cache()
        return n
    n0 = count(base_c2)
    lo, hi = 0.0, base_c2
    for _ in range(7):
        mid = 0.5 * (lo + hi)
        frac = 1.0 - count(mid) / max(1, n0)
        log("  C2 %.5f prunes %.4f" % (mid, frac))
        if frac > target_fraction:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


# ------------------------------------------------------------------ driver
def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train-frames", type=int, default=TRAIN_SEEDS[1] - TRAIN_SEEDS[0])
    ap.add_argument("--val-frames", type=int, default=VAL_SEEDS[1] - VAL_SEEDS[0])
    ap.add_argument("--eval-frames", type=int, default=2)
    ap.add_argument("--samples", type=float, default=2e7, help="training triplets in total")
    ap.add_argument("--epochs", type=int, default=5)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--report", default="")
    ap.add_argument("--skip-train", action="store_true", help="use the saved weights (from --out)")
    ap.add_argument("--skip-gain", action="store_true", help="stop after training and the threshold")
    args = ap.parse_args(argv)
    import torch
    nth = args.threads or min(16, os.cpu_count() or 1)
    x_row, _ = synth.geometry()

    def make_tracker(**kw):
        # training, threshold and gain test count every candidate triplet:
        # pruned runs keep the triplet pool
        kw.setdefault("pool_per_cluster", 12)
        t = tpcca.Tracker(row_x=x_row, **kw)
        t.set_triplet_pool(True)
        return t

    trk = make_tracker()
    report = {"seeds": {}}
    if args.skip_train:
        params, meta = load_weights(args.out)
        if params is None:
            raise SystemExit("no saved weights at %s" % args.out)
        trk.mlp_load(params)
        report.update(meta)
    else:
        tr_seeds = list(range(TRAIN_SEEDS[0], TRAIN_SEEDS[0] + args.train_frames))
        log("collecting triplets from %d training slices ..." % len(tr_seeds))
        trk.mlp_load(init_params(args.seed))
        t0 = time.perf_counter()
        X, Y, tot, pos = collect(trk, tr_seeds, args.samples / len(tr_seeds), args.seed, nth)
        log("  %d of %d triplets sampled (%.1f%% positive) in %.0f s"
            % (len(Y), tot, 100.0 * pos / max(1, len(Y)), time.perf_counter() - t0))
        # 2% held out for a loss check
        g = torch.Generator(device="cuda")
        g.manual_seed(args.seed + 1)
        ho = torch.rand(len(Y), device="cuda", generator=g) < 0.02
        xt, yt = X[~ho].contiguous(), Y[~ho].contiguous()
        xh, yh = X[ho].contiguous(), Y[ho].contiguous()
        del X, Y
        trk.mlp_load(init_params(args.seed))
        z0 = logits(trk, xh)
        t0 = time.perf_counter()
        hist, pw = train(trk, xt, yt, epochs=args.epochs, seed=args.seed)
        train_s = time.perf_counter() - t0
        zh = logits(trk, xh)
        acc = float(((zh > 0).float() == yh).float().mean().item())
        meta = {"train_seeds": [tr_seeds[0], tr_seeds[-1]], "triplets_seen": int(tot), "samples": int(xt.shape[0]),
                "positive_fraction": float(yt.mean().item()), "pos_weight": pw, "epochs": args.epochs, "batch": 4096,
                "lr": 1e-3, "weight_decay": 1e-4, "seed": args.seed, "train_s": round(train_s, 1),
                "heldout_bce_init": bce(z0, yh, pw), "heldout_bce": bce(zh, yh, pw), "heldout_accuracy": acc,
                "loss_history": hist[:: max(1, len(hist) // 50)]}
        log("  trained in %.0f s: held-out BCE %.4f -> %.4f, accuracy %.4f"
            % (train_s, meta["heldout_bce_init"], meta["heldout_bce"], acc))
        params = trk.mlp_fetch()
        report.update(meta)
        zs = zh.cpu().numpy()
        del xt, yt, xh, yh
        torch.cuda.empty_cache()

        va_seeds = range(VAL_SEEDS[0], VAL_SEEDS[0] + args.val_frames)
        log("threshold on %d held-out slices ..." % args.val_frames)
        vset = FrameSet("slice_1ms", va_seeds, nth)
        theta, vbase, vq = select_theta(trk, vset, zs)
        meta.update({"theta": theta, "val_seeds": [VAL_SEEDS[0], VAL_SEEDS[0] + args.val_frames - 1],
                     "val_plain": vbase, "val_pruned": vq})
        save_weights(params, meta, args.out)
        log("saved %s (theta %.4f)" % (args.out, theta))
        report.update(meta)
        del vset
    if args.skip_gain:
        print(json.dumps(report, indent=1, default=float))
        return

    # gain test on 10 ms frames
    theta = report["theta"]
    ev = FrameSet("frame_10ms", range(EVAL_SEEDS[0], EVAL_SEEDS[0] + args.eval_frames), nth)
    log("gain test on %d 10 ms frames (%d clusters) ..." % (args.eval_frames, ev.n_clusters))
    trk.set_pruning(False)
    plain = ev.evaluate(trk, timing=True)
    trk.set_pruning(True, theta)
    learned = ev.evaluate(trk, timing=True)
    frac = learned["pruned_fraction"]
    log("  plain eff %.5f, learned eff %.5f, pruned %.3f" % (plain["efficiency"], learned["efficiency"], frac))
    c2 = matched_pair_cut(make_tracker, ev, frac)
    hand_trk = make_tracker(pair_c2=c2)
    hand = ev.evaluate(hand_trk, timing=True)
    del hand_trk
    torch.cuda.empty_cache()
    rnd = make_tracker()
    rnd.mlp_load(init_params(args.seed + 100))
    rnd.set_pruning(True, -1e30)
    rnd.clear_frames()
    f0 = rnd.load_frame_packed(ev.frames[0])
    rnd.run(sync=True)
    zr = np.concatenate([rnd.triplets(f0, s)[2] for s in range(0, 36, 6)])
    th_r = float(np.quantile(zr, frac))
    rnd.set_pruning(True, th_r)
    random_net = ev.evaluate(rnd, timing=True)
    res = {"theta": theta, "plain": plain, "learned": learned, "hand_cut": dict(hand, pair_c2=c2),
           "random_net": dict(random_net, theta=th_r)}
    for k in ("learned", "hand_cut", "random_net"):
        q = res[k]
        q["efficiency_loss"] = plain["efficiency"] - q["efficiency"]
        q["delta_fake"] = q["fake_rate"] - plain["fake_rate"]
        q["delta_clone"] = q["clone_rate"] - plain["clone_rate"]
        q["delta_mean_length"] = q["mean_track_length"] - plain["mean_track_length"]
        log("  %-10s eff loss %+.5f fake %+.5f clone %+.5f length %+.3f pruned %.3f clusters/s %.3g"
            % (k, q["efficiency_loss"], q["delta_fake"], q["delta_clone"], q["delta_mean_length"],
               q["pruned_fraction"], q.get("clusters_per_s") or 0))
    res["learned_beats_hand_cut"] = bool(res["learned"]["efficiency_loss"] <= 0.005 and
                                         res["learned"]["efficiency"] > res["hand_cut"]["efficiency"])
    res["eval_seeds"] = [EVAL_SEEDS[0], EVAL_SEEDS[0] + args.eval_frames - 1]
    report["gain_test"] = res
    out = json.dumps(report, indent=1, default=float)
    if args.report:
        with open(args.report, "w") as f:
            f.write(out)
    print(out)


if __name__ == "__main__":
    main()
