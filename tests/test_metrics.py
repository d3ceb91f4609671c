"""Truth-matching metrics on hand-built cases (closed-form expectations)."""
import numpy as np

from paper_2102_08862_amd import metrics


def test_counts_hand_built():
    # particle 0: 40 hits, particle 1: 35 hits, particle 2: 10 hits (not findable), 5 noise
    labels = np.array([0] * 40 + [1] * 35 + [2] * 10 + [-1] * 5, np.int32)
    idx0 = np.arange(0, 40); idx1 = np.arange(40, 75); idx2 = np.arange(75, 85); noise = np.arange(85, 90)
    tracks = [
        idx0[:30],                                 # matches 0
        idx0[30:],                                 # clone of 0 (10 hits)
        np.concatenate([idx1[:18], idx0[:2]]),     # 18/20 = 0.9 -> matches 1
        np.concatenate([idx2, noise[:3]]),         # 10/13 < 0.9 -> fake
        noise,                                     # majority noise -> fake
    ]
    cl = np.concatenate(tracks)
    ln = np.array([len(t) for t in tracks])
    c = metrics.sector_counts(labels, cl, ln)
    assert c["findable"] == 2 and c["found"] == 2 and c["tracks"] == 5
    assert c["fakes"] == 2 and c["clones"] == 1 and c["matched_pairs"] == 2
    assert c["find_hits"] == 75
    # good hits: 30 + 10 (particle 0 on its two tracks) + 18 (particle 1)
    assert c["good_hits"] == 58
    s = metrics.summarize([c])
    assert s["efficiency"] == 1.0 and abs(s["fake_rate"] - 0.4) < 1e-12 and abs(s["clone_rate"] - 0.5) < 1e-12
    assert abs(s["hit_efficiency"] - 58 / 75) < 1e-12


def test_no_tracks():
    labels = np.array([0] * 31 + [-1], np.int32)
    c = metrics.sector_counts(labels, np.zeros(0, np.int32), np.zeros(0, np.int64))
    assert c["findable"] == 1 and c["found"] == 0 and c["tracks"] == 0
    assert metrics.summarize([c])["efficiency"] == 0.0
