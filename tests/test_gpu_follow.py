"""GPU parity of the track following and shared-cluster selection: the HIP
path with follow = 1 against the oracle's following on the same inputs.

Assignment, track identities (chain seeds), lengths and cluster lists must be
bit-exact (the filters run in FP32 with one rounding per operation on both
sides, so every box, chi2 and claim decision is the same); parameters of the
fitted kept tracks agree as in the plain parity tests. Cases: single
sectors, sampled sectors of a 1 ms slice, a line broken by empty rows, empty
and trackless inputs, a graph-replayed batch, and two sectors of the 10 ms
frame with the whole frame's quality against the plain tracker."""
import numpy as np
import pytest

import oracle
from paper_2102_08862_amd import metrics, synth

from _parity import compare_params, oracle_cfg

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


def oracle_follow(ocfg, row, y, t):
    return oracle.run_sector(ocfg, row, y, t, follow_cfg=oracle.FollowConfig())


def compare_follow(trk, frame, sector, row, y, t, ocfg, ref=None, check_params=True):
    if ref is None:
        ref = oracle_follow(ocfg, row, y, t)
    assign = trk.assignment(frame, sector)
    assert np.array_equal(assign, ref["assign"]), "assignment differs at %s" % np.nonzero(assign != ref["assign"])[0][:10]
    cl = trk.track_clusters(frame, sector)
    assert np.array_equal(cl, ref["clusters"]), "cluster lists differ"
    tracks = trk.tracks(frame, sector)
    assert len(tracks) == len(ref["first"])
    assert np.array_equal(tracks["first"], ref["first"])
    assert np.array_equal(tracks["n_clusters"], ref["len"])
    ch = ref["chains"]
    kept = ref["kept"] >= 0
    seeds = ch["clusters"][ch["first"]][kept] if len(ch["first"]) else np.zeros(0, np.int32)
    if len(tracks):
        assert np.array_equal(tracks["seed"], seeds)
        assert (tracks["frame"] == frame).all() and (tracks["sector"] == sector).all()
    out = dict(n=len(row), chains=len(ch["first"]), tracks=len(tracks),
               added=int(ref["ext_in"].sum() + ref["ext_out"].sum()), dropped=int((~kept).sum()),
               worst=0.0, excluded=0)
    if check_params and len(tracks):
        out.update(compare_params(tracks, ref, row, y, t, ocfg))
    return out


def _tracker(tp, **kw):
    return tp.Tracker(follow=1, **kw)


@pytest.mark.parametrize("seed", [1, 2])
def test_single_sector(tp, x, seed):
    fr = synth.generate("sector_300", seed=seed)
    row, y, t = fr.sector(0)
    print("case follow sector_300 seed", seed, flush=True)
    trk = _tracker(tp)
    f = trk.add_frame()
    trk.load_sector(f, 0, row, y, t, device=True)
    trk.run(sync=True)
    res = compare_follow(trk, f, 0, row, y, t, oracle_cfg(x))
    print(res)
    st = trk.stats()
    assert st["n_chains"] == res["chains"] and st["n_tracks"] == res["tracks"]
    assert st["n_follow_added"] == res["added"] and st["n_follow_dropped"] == res["dropped"]
    assert res["tracks"] > 50 and res["added"] > 0


def test_row_sort_two_pass_path(tp, x):
    """Every row-sort bucket sorted by the two-pass path (the fine-bin
    starts the following reads come from it too): the oracle's results."""
    fr = synth.generate("sector_300", seed=3)
    row, y, t = fr.sector(0)
    print("case follow sector_300 seed 3, two-pass row sort", flush=True)
    trk = _tracker(tp)
    trk.set_launch(4, 0, 1)
    f = trk.add_frame()
    trk.load_sector(f, 0, row, y, t, device=True)
    trk.run(sync=True)
    res = compare_follow(trk, f, 0, row, y, t, oracle_cfg(x))
    assert res["tracks"] > 50 and res["added"] > 0


def test_slice_1ms_sampled_sectors(tp, x):
    fr = synth.generate("slice_1ms", seed=2300)
    print("case follow slice_1ms seed 2300: %d clusters" % fr.n_clusters, flush=True)
    trk = _tracker(tp)
    f = trk.load_frame_packed(fr)
    trk.run(sync=True)
    oc = oracle_cfg(x)
    for s in (0, 11, 20, 35):
        row, y, t = fr.sector(s)
        res = compare_follow(trk, f, s, row, y, t, oc)
        print("sector", s, res, flush=True)
        assert res["dropped"] > 100


def test_line_broken_by_empty_rows(tp, x):
    """A straight line on rows 10..40 without rows 24 and 25 (two chains
    without their end clusters) ends as one track of all 29 clusters; with
    rows 24..26 empty the two stay apart."""
    for gap, spans in (((24, 25), [29]), ((24, 25, 26), [14, 18])):
        rows = [r for r in range(10, 41 if len(gap) == 2 else 45) if r not in gap]
        r = np.array(rows, np.uint8)
        perm = np.random.default_rng(len(gap)).permutation(len(r))
        r = r[perm]
        xs = x[r].astype(np.float64) - float(x[10])
        y = (0.2 * xs).astype(np.float32)
        t = (5.0 + 0.3 * xs).astype(np.float32)
        print("case follow line gap", gap, flush=True)
        trk = _tracker(tp)
        f = trk.add_frame()
        trk.load_sector(f, 0, r, y, t, device=False)
        trk.run(sync=True)
        res = compare_follow(trk, f, 0, r, y, t, oracle_cfg(x))
        assert sorted(trk.tracks(f, 0)["n_clusters"].tolist()) == spans, res


def test_empty_and_trackless_inputs(tp, x):
    print("case follow empty + noise-only", flush=True)
    trk = _tracker(tp)
    f = trk.add_frame()
    rng = np.random.default_rng(5)
    n = 3000
    row = rng.integers(0, 152, n).astype(np.uint8)
    y = rng.uniform(-20, 20, n).astype(np.float32)
    t = rng.uniform(0, 250, n).astype(np.float32)
    trk.load_sector(f, 3, row, y, t, device=False)
    trk.load_sector(f, 4, row[:0], y[:0], t[:0], device=False)
    trk.run(sync=True)
    compare_follow(trk, f, 3, row, y, t, oracle_cfg(x))
    assert len(trk.tracks(f, 4)) == 0
    st = trk.stats()
    assert st["n_tracks"] == len(trk.tracks(f, 3))


def test_graph_replays_of_a_batch(tp, x):
    """Two frames in one run, replayed from a captured graph: every replay
    gives the oracle's results on sampled sectors of both frames."""
    frames = [synth.generate("frame_10ms", seed=4200 + i, n_threads=16, frame_us=1000.0 * L,
                             n_collisions=int(round(50 * L))) for i, L in enumerate((0.5, 0.8))]
    print("case follow graph batch: %d clusters" % sum(f.n_clusters for f in frames), flush=True)
    trk = _tracker(tp)
    ids = [trk.load_frame_packed(fr) for fr in frames]
    trk.ensure_arena()
    trk.set_graph(True)
    oc = oracle_cfg(x)
    refs = {}
    for rep in range(3):
        trk.run(sync=True)
        for k, s in ((0, 2), (1, 30)):
            row, y, t = frames[k].sector(s)
            if (k, s) not in refs:
                refs[(k, s)] = oracle_follow(oc, row, y, t)
            res = compare_follow(trk, ids[k], s, row, y, t, oc, ref=refs[(k, s)], check_params=rep == 2)
        print("replay", rep, res, flush=True)


def test_frame_10ms_sectors_and_quality(tp, x):
    """Sectors 0 and 18 of the 10 ms frame against the oracle; over the whole
    frame, following merges the CA's clones and attaches more hits."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    fr = synth.generate("frame_10ms", seed=3000, n_threads=16)
    print("case follow frame_10ms seed 3000: %d clusters" % fr.n_clusters, flush=True)

    def quality(trk, f):
        return metrics.summarize([metrics.sector_counts(fr.labels[s], trk.track_clusters(f, s),
                                                        trk.tracks(f, s)["n_clusters"]) for s in range(len(fr.rows))])

    trk = tp.Tracker()
    f = trk.load_frame_packed(fr)
    trk.run(sync=True)
    q_plain = quality(trk, f)
    del trk
    torch.cuda.empty_cache()
    trk = _tracker(tp)
    f = trk.load_frame_packed(fr)
    trk.run(sync=True)
    st = trk.stats()
    q_fol = quality(trk, f)
    print("plain", q_plain, "\nfollow", q_fol, "\nstats chains %d tracks %d added %d dropped %d"
          % (st["n_chains"], st["n_tracks"], st["n_follow_added"], st["n_follow_dropped"]), flush=True)
    oc = oracle_cfg(x)

    def one(s):
        row, y, t = fr.sector(s)
        return s, oracle_follow(oc, row, y, t)
    with ThreadPoolExecutor(max_workers=2) as ex:
        refs = dict(ex.map(one, (0, 18)))
    for s in (0, 18):
        row, y, t = fr.sector(s)
        res = compare_follow(trk, f, s, row, y, t, oc, ref=refs[s])
        print("sector", s, res, flush=True)
    assert q_fol["clone_rate"] < 0.1 * q_plain["clone_rate"]
    assert q_fol["hit_efficiency"] > q_plain["hit_efficiency"] + 0.03
    assert q_fol["fake_rate"] <= q_plain["fake_rate"]
    assert q_fol["efficiency"] >= q_plain["efficiency"] - 0.005
    del trk
    torch.cuda.empty_cache()
