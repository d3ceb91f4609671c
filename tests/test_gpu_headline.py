"""GPU parity at the benchmark's sizes: the whole 10 ms frame (seed 3000,
1.45e8 clusters) run once in the launch configuration the benchmark times,
with one A-side and one C-side sector compared with the CPU oracle element
by element; a batch of uneven frames in one graph-replayed run with sampled
sectors against the oracle; and the gain of the trained triplet network on
the 10 ms frame against the plain tracker and an equal-share tighter cut."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2102_08862_amd import synth

from _parity import compare_sector, oracle_cfg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    from paper_2102_08862_amd import tpcca
    assert torch.cuda.is_available()
    tpcca.load_library()
    return tpcca


@pytest.fixture(scope="module")
def x():
    return synth.geometry()[0]


@pytest.fixture(scope="module")
def frame10():
    fr = synth.generate("frame_10ms", seed=3000, n_threads=16)
    print("frame_10ms seed 3000: %d clusters" % fr.n_clusters, flush=True)
    return fr


def _oracle_sectors(fr, ocfg, secs):
    def one(s):
        row, y, t = fr.sector(s)
        return s, oracle.run_sector(ocfg, row, y, t)
    with ThreadPoolExecutor(max_workers=len(secs)) as ex:
        return dict(ex.map(one, secs))


def test_frame_10ms_sectors_vs_oracle(tp, x, frame10):
    """Sectors 0 (A side) and 18 (C side) of the 10 ms frame: links, cleaned
    links, assignment, track identities and cluster lists bit-exact,
    parameters within 1e-4 (floors of the parity helpers)."""
    import torch
    from paper_2102_08862_amd import autotune
    fr = frame10
    trk = tp.Tracker()
    f = trk.load_frame_packed(fr)
    trk.ensure_arena()
    autotune.apply(trk, fr.n_clusters)
    trk.ensure_arena()
    trk.run(sync=True)
    st = trk.stats()
    assert st["n_clusters"] == fr.n_clusters and st["n_invalid"] == 0
    print("run: %d links, %d tracks" % (st["n_links"], st["n_tracks"]), flush=True)
    oc = oracle_cfg(x)
    refs = _oracle_sectors(fr, oc, (0, 18))
    for s in (0, 18):
        row, y, t = fr.sector(s)
        res = compare_sector(trk, f, s, row, y, t, oc, ref=refs[s])
        print("sector", s, res, flush=True)
        assert res["tracks"] > 50000
    del trk
    torch.cuda.empty_cache()


def test_batched_uneven_frames_graph_vs_oracle(tp, x):
    """Four frames of uneven length (0.6, 2.3, 1.1 and 0.5 ms) in one run,
    replayed from a captured HIP graph three times in the batched launch
    configuration; one sampled sector of every frame (both sides) against
    the oracle after the last replay."""
    import torch
    from paper_2102_08862_amd import autotune
    lens = [0.6, 2.3, 1.1, 0.5]
    frames = [synth.generate("frame_10ms", seed=4100 + i, n_threads=16, frame_us=1000.0 * L,
                             n_collisions=int(round(50 * L))) for i, L in enumerate(lens)]
    total = sum(fr.n_clusters for fr in frames)
    print("batched: %d frames, %d clusters" % (len(frames), total), flush=True)
    trk = tp.Tracker()
    ids = [trk.load_frame_packed(fr) for fr in frames]
    trk.ensure_arena()
    autotune.apply(trk, total)
    trk.ensure_arena()
    trk.set_graph(True)
    for _ in range(3):
        trk.run(sync=True)
    oc = oracle_cfg(x)
    picks = [(0, 3), (1, 20), (2, 35), (3, 17)]
    for (k, s) in picks:
        fr = frames[k]
        row, y, t = fr.sector(s)
        res = compare_sector(trk, ids[k], s, row, y, t, oc)
        print("frame", k, "sector", s, res, flush=True)
        assert res["tracks"] > 1000
    del trk
    torch.cuda.empty_cache()


def _quality(trk, fr, f):
    from paper_2102_08862_amd import metrics
    counts = [metrics.sector_counts(fr.labels[s], trk.track_clusters(f, s), trk.tracks(f, s)["n_clusters"])
              for s in range(len(fr.rows))]
    return metrics.summarize(counts)


def test_trained_network_gain_on_frame_10ms(tp, frame10):
    """What the trained network gains on the 10 ms frame at its stored
    threshold: it removes more than half of all candidate triplets (counted
    through the triplet pool) at an absolute efficiency loss of at most 0.5%
    and a lower fake rate than the plain tracker, where a tighter pair cut
    that removes the same share of triplets loses most of the efficiency."""
    import torch
    from paper_2102_08862_amd import prune_train
    params, meta = prune_train.load_weights()
    assert params is not None and "theta" in meta, "trained weights missing"
    theta = float(meta["theta"])
    fr = frame10

    def tracker(**kw):
        t = tp.Tracker(**kw)
        return t, t.load_frame_packed(fr)

    trk, f = tracker()
    trk.run(sync=True)
    q_plain = _quality(trk, fr, f)
    trk.mlp_load(params)
    trk.set_triplet_pool(True)
    trk.set_pruning(True, theta)
    trk.run(sync=True)
    st = trk.stats()
    assert st["n_pool_overflow"] == 0
    share = st["n_pruned"] / max(1, st["n_triplets"])
    q_learned = _quality(trk, fr, f)
    n_all = st["n_triplets"]
    del trk
    torch.cuda.empty_cache()
    # the tighter cut: the stored C2' of the gain report, checked to prune the
    # same share of triplets (triplet counts of an enumeration-only run)
    c2 = float(prune_train.load_report()["gain_test"]["hand_cut"]["pair_c2"])
    trk, f = tracker(pair_c2=c2)
    trk.mlp_load(params)
    trk.set_triplet_pool(True)
    trk.set_pruning(True, -1e30)
    trk.run(sync=True)
    share_cut = 1.0 - trk.stats()["n_triplets"] / max(1, n_all)
    trk.set_pruning(False)
    trk.set_triplet_pool(False)
    trk.run(sync=True)
    q_cut = _quality(trk, fr, f)
    del trk
    torch.cuda.empty_cache()
    loss = q_plain["efficiency"] - q_learned["efficiency"]
    print("plain eff %.5f fake %.5f | learned (theta %.4f) eff %.5f fake %.5f, %.1f%% of %d triplets pruned "
          "(loss %.5f) | cut C2'=%.5f eff %.5f, %.1f%% pruned"
          % (q_plain["efficiency"], q_plain["fake_rate"], theta, q_learned["efficiency"], q_learned["fake_rate"],
             100 * share, n_all, loss, c2, q_cut["efficiency"], 100 * share_cut), flush=True)
    assert share > 0.5
    assert abs(share_cut - share) < 0.05, "the hand cut does not prune the same share"
    assert loss <= 0.005
    assert q_learned["fake_rate"] < q_plain["fake_rate"]
    assert q_learned["efficiency"] > q_cut["efficiency"] + 0.1
