"""Pins of the oracle's track following and selection.

Pinned against cases whose outcome is fixed by the definition alone: a
straight track broken by two empty pad rows (the CA gives two chains without
their end clusters; following must join them into one track of every
cluster, ties between the two equally long extended tracks going to the
smaller seed index), the same track broken by three empty rows (one more
than the allowed misses: the two tracks stay apart), noise-free helices
(every cluster of a particle, rows 0 and 151 included, on one track), the
independence of the extension from the input order, and the effect on a 1 ms
slice sector (clones merged, more hits attached)."""
import numpy as np
import pytest

import oracle
from paper_2102_08862_amd import metrics, synth


def _line(x, rows, perm_seed):
    x10 = float(x[10])
    r = np.array(rows, np.uint8)
    y = (0.2 * (x[r].astype(np.float64) - x10)).astype(np.float32)
    t = (5.0 + 0.3 * (x[r].astype(np.float64) - x10)).astype(np.float32)
    perm = np.random.default_rng(perm_seed).permutation(len(r))
    return r[perm], y[perm], t[perm]


@pytest.mark.parametrize("perm_seed", [0, 1, 2])
def test_two_empty_rows_are_bridged(geom, ocfg, perm_seed):
    x = geom[0]
    rows = [r for r in range(10, 41) if r not in (24, 25)]
    row, y, t = _line(x, rows, perm_seed)
    fc = oracle.FollowConfig()
    res = oracle.run_sector(ocfg, row, y, t, fit=False, follow_cfg=fc)
    ch = res["chains"]
    # the CA: rows 11..22 and 27..39 (end clusters have no pair)
    spans = sorted((int(row[ch["clusters"][f]]), int(row[ch["clusters"][f + l - 1]]))
                   for f, l in zip(ch["first"], ch["len"]))
    assert spans == [(11, 22), (27, 39)]
    # following: one track of all 29 clusters in ascending rows
    assert len(res["first"]) == 1 and res["len"][0] == 29
    assert np.array_equal(row[res["clusters"]], np.array(rows, np.uint8))
    assert (res["assign"] == 0).all()
    # both extended tracks hold 29 clusters: the smaller seed index wins
    seeds = [int(ch["clusters"][f]) for f in ch["first"]]
    kept = res["kept"]
    assert sorted(kept.tolist()) == [-1, 29]
    assert seeds[int(np.argmax(kept))] == min(seeds)
    assert sorted((res["ext_in"] + res["ext_out"] + ch["len"]).tolist()) == [29, 29]


def test_three_empty_rows_are_not_bridged(geom, ocfg):
    x = geom[0]
    rows = [r for r in range(10, 45) if r not in (24, 25, 26)]
    row, y, t = _line(x, rows, 5)
    res = oracle.run_sector(ocfg, row, y, t, fit=False, follow_cfg=oracle.FollowConfig())
    spans = sorted((int(row[res["clusters"][f]]), int(row[res["clusters"][f + l - 1]]))
                   for f, l in zip(res["first"], res["len"]))
    # each chain gets its own end clusters back, nothing across the gap
    assert spans == [(10, 23), (27, 44)]


def test_noise_free_particles_end_on_one_track(geom, ocfg):
    fr = synth.generate("sector_300", seed=31, sigma_y=0.0, sigma_t=0.0, noise_frac=0.0)
    row, y, t = fr.sector(0)
    lab = fr.labels[0]
    res = oracle.run_sector(ocfg, row, y, t, fit=False, follow_cfg=oracle.FollowConfig())
    n_rows = len(geom[0])
    good = ends = ends_kept = 0
    parts = [p for p in np.unique(lab) if p >= 0 and (lab == p).sum() >= 30]
    for p in parts:
        mine = np.nonzero(lab == p)[0]
        tr = res["assign"][mine]
        good += int(tr[0] >= 0 and (tr == tr[0]).all())
        for r in (0, n_rows - 1):
            at = mine[row[mine] == r]
            if len(at):
                ends += 1
                ends_kept += int(res["assign"][at[0]] >= 0)
    assert len(parts) > 100
    assert good >= 0.97 * len(parts)
    assert ends > 20 and ends_kept >= 0.95 * ends


def test_extension_does_not_depend_on_input_order(ocfg):
    # Selection breaks ties of equal extended length by seed input index, so
    # only the extension itself is order-free: per chain (keyed by its
    # clusters), the clusters added inward and outward.
    fr = synth.generate("sector_300", seed=32)
    row, y, t = fr.sector(0)
    fc = oracle.FollowConfig()
    a = oracle.run_sector(ocfg, row, y, t, fit=False, follow_cfg=fc)
    perm = np.random.default_rng(3).permutation(len(row))
    b = oracle.run_sector(ocfg, row[perm], y[perm], t[perm], fit=False, follow_cfg=fc)

    def ext(r, p):
        ch = r["chains"]
        return {tuple(sorted(p[ch["clusters"][f:f + l]])): (int(i), int(o))
                for f, l, i, o in zip(ch["first"], ch["len"], r["ext_in"], r["ext_out"])}

    ea, eb = ext(a, np.arange(len(row))), ext(b, perm)
    assert len(ea) > 100 and ea == eb
    assert sum(i + o for i, o in ea.values()) > 0


def test_following_merges_clones_on_a_slice_sector(ocfg):
    fr = synth.generate("slice_1ms", seed=2300, n_threads=8)
    row, y, t = fr.sector(0)
    lab = fr.labels[0]
    q = {}
    for name, fc in (("chains", None), ("follow", oracle.FollowConfig())):
        r = oracle.run_sector(ocfg, row, y, t, fit=False, follow_cfg=fc)
        cl = r["clusters"]
        q[name] = metrics.summarize([metrics.sector_counts(lab, cl, r["len"])])
    assert q["chains"]["clone_rate"] > 0.5
    assert q["follow"]["clone_rate"] < 0.05
    assert q["follow"]["hit_efficiency"] > q["chains"]["hit_efficiency"] + 0.03
    assert q["follow"]["fake_rate"] < q["chains"]["fake_rate"]
    assert q["follow"]["efficiency"] > q["chains"]["efficiency"] - 0.005


def test_filter_without_process_noise_is_least_squares():
    # q = 0: the filter started at the first point with slope prior
    # N(0, var_slope0) is the weighted least-squares line with that prior, at
    # the last point (value, slope) and with covariance the inverse of the
    # information matrix.
    rng = np.random.default_rng(7)
    x = np.cumsum(rng.uniform(0.7, 1.6, 25)).astype(np.float32)
    m = (0.3 - 0.17 * x + rng.normal(0, 0.05, 25)).astype(np.float32)
    var, vs0 = 0.0025, 4.0
    out = oracle.kf1_run(x, m, var, vs0, 0.0).astype(np.float64)
    xd = x.astype(np.float64) - np.float64(x[-1])
    A = np.stack([np.ones_like(xd), xd], 1)
    H = A.T @ A / var + np.diag([0.0, 1.0 / vs0])
    g = A.T @ m.astype(np.float64) / var
    sol = np.linalg.solve(H, g)
    C = np.linalg.inv(H)
    assert np.allclose(out[:2], sol, rtol=1e-4, atol=1e-5)
    assert np.allclose(out[2:], [C[0, 0], C[0, 1], C[1, 1]], rtol=1e-3, atol=1e-9)


def test_filter_with_unbounded_process_noise_follows_the_last_two_points():
    # q -> infinity forgets the past at every step: the value becomes the
    # last measurement and the slope the difference quotient of the last two.
    x = np.array([0.0, 1.1, 2.3, 3.2, 4.5], np.float32)
    m = np.array([1.0, 0.4, 2.0, -0.5, 0.7], np.float32)
    out = oracle.kf1_run(x, m, 1e-4, 1.0, 1e12)
    assert out[0] == pytest.approx(0.7, abs=1e-4)
    assert out[1] == pytest.approx((0.7 + 0.5) / 1.3, rel=1e-3)
