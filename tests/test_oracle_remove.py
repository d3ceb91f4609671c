"""Pins of the oracle's cluster removal (R33): a hand-built sector whose
kept list is written out by hand, the limits of the threshold, and, on a
noise-free generated sector, that exactly the clusters of the low-pT
particles' tracks go (one track per particle there)."""
import numpy as np

import oracle
from paper_2102_08862_amd import synth


def test_hand_built_sector():
    # tracks: 0 ok, pT 2 GeV; 1 ok, pT 0.1 GeV (q/pT = -10); 2 failed fit, q/pT 20; 3 ok, pT exactly 0.2
    status = np.array([0, 0, 2, 0])
    qpt = np.array([0.5, -10.0, 20.0, 5.0])
    assign = np.array([-1, 0, 1, 1, 2, -1, 3, 0, 1])
    kept = oracle.remove_clusters(9, assign, status, qpt, pt_min=0.2)
    # removed: the clusters of track 1 (inputs 2, 3, 8); track 3 sits on the threshold and stays
    assert kept.tolist() == [0, 1, 4, 5, 6, 7]
    assert oracle.remove_clusters(9, assign, status, qpt, pt_min=0.05).tolist() == list(range(9))
    assert oracle.remove_clusters(9, assign, status, qpt, pt_min=1e9).tolist() == [0, 4, 5]
    assert oracle.remove_clusters(0, np.zeros(0, int), status, qpt, 0.2).tolist() == []


def test_noise_free_sector_removes_the_low_pt_particles(geom, ocfg):
    """Noise-free helices of a single sector: each track is one particle's
    chain; removing at pt_min keeps every cluster of a track whose
    particle has pT >= pt_min (up to fitted pT near the threshold) and
    removes those of the clearly lower ones."""
    fr = synth.generate("sector_300", seed=23, sigma_y=0.0, sigma_t=0.0, quant=0.0, noise_frac=0.0)
    row, y, t = fr.sector(0)
    res = oracle.run_sector(ocfg, row, y, t)
    fit = res["fit"]
    pt_min = 0.3
    kept = oracle.remove_clusters(len(row), res["assign"], fit["status"], fit["qpt"], pt_min)
    keep = np.zeros(len(row), bool)
    keep[kept] = True
    lab = fr.labels[0]
    pt = fr.tracks[:, 1]
    on = res["assign"] >= 0
    tr_pt = pt[lab[on]]
    # far from the threshold the decision follows the particle's pT
    assert keep[on][tr_pt > 1.05 * pt_min].all()
    low = (tr_pt < 0.95 * pt_min) & (fit["status"][res["assign"][on]] == 0)
    assert low.any() and not keep[on][low].any()
    assert keep[~on].all()
