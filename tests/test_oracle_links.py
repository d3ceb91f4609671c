"""Pins of the oracle's neighbour links, cleaning and chains.

The paper gives no worked example, so the oracle is pinned by: brute-force
enumeration of every (down, up) pair on tiny inputs, with exact ties and
duplicated hits (pure Python, numpy float32 scalars, one rounding per
operation); closed-form scores; exact symmetries (time shift, y and time
mirror); and the structural invariants the chain definition implies."""
import numpy as np
import pytest

import oracle
from paper_2102_08862_amd import synth

F = np.float32


def brute_links(cfg, row, y, t):
    """Every candidate pair enumerated directly from the definition."""
    n = len(row)
    x = cfg.row_x
    up = np.full(n, -1, np.int32); dn = np.full(n, -1, np.int32); gap = np.zeros(n, np.int32)
    for i in range(n):
        r = int(row[i])
        for g in range(1, cfg.max_gap + 1):
            if r - g < 0 or r + g > len(x) - 1:
                continue
            w = F(F(x[r] - x[r - g]) / F(x[r + g] - x[r - g]))
            wy = F(F(g) * F(cfg.win_y)); wt = F(F(g) * F(cfg.win_t))
            D = [d for d in range(n) if row[d] == r - g and abs(F(y[i] - y[d])) <= wy and abs(F(t[i] - t[d])) <= wt]
            U = [u for u in range(n) if row[u] == r + g and abs(F(y[u] - y[i])) <= wy and abs(F(t[u] - t[i])) <= wt]
            best = None
            for d in D:
                for u in U:
                    ady = F(y[i] - y[d]); adt = F(t[i] - t[d])
                    by = F(y[u] - y[d]); bt = F(t[u] - t[d])
                    ry = F(ady - F(w * by)); rt = F(adt - F(w * bt))
                    c = F(F(ry * ry) + F(rt * rt))
                    if c <= F(cfg.pair_c2):
                        key = (c, u, d)
                        if best is None or key < best:
                            best = key
            if best is not None:
                up[i], dn[i], gap[i] = best[1], best[2], g
                break
    return up, dn, gap


def _tiny(seed, n, rows=7, spread=1.0, step=0.25, dup=0.2):
    rng = np.random.default_rng(seed)
    row = rng.integers(0, rows, n).astype(np.uint8)
    y = (np.round(rng.uniform(-spread, spread, n) / step) * step).astype(np.float32)
    t = (np.round(rng.uniform(-spread, spread, n) / step) * step).astype(np.float32)
    k = int(dup * n)
    src = rng.integers(0, n, k); dst = rng.integers(0, n, k)
    row[dst] = row[src]; y[dst] = y[src]; t[dst] = t[src]
    return row, y, t


@pytest.mark.parametrize("seed", range(6))
def test_links_match_brute_force_with_ties(ocfg, seed):
    row, y, t = _tiny(seed, 120 + 30 * seed)
    a = oracle.links(ocfg, row, y, t)
    b = brute_links(ocfg, row, y, t)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    assert (a[0] >= 0).sum() > 10


def test_links_match_brute_force_generated(ocfg):
    """Tiny slice of a generated sector (real geometry, all rows)."""
    fr = synth.generate("sector_300", seed=9)
    row, y, t = fr.sector(0)
    m = (t > -3) & (t < 3)
    row, y, t = row[m], y[m], t[m]
    assert 100 < len(row) < 1500
    a = oracle.links(ocfg, row, y, t)
    b = brute_links(ocfg, row, y, t)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_links_subset_equals_full(ocfg):
    fr = synth.generate("sector_300", seed=4)
    row, y, t = fr.sector(0)
    up, dn, gap = oracle.links(ocfg, row, y, t)
    q = np.arange(0, len(row), 7, dtype=np.int32)
    su, sd, sg = oracle.links_subset(ocfg, row, y, t, q)
    assert np.array_equal(su, up[q]) and np.array_equal(sd, dn[q]) and np.array_equal(sg, gap[q])


def test_closed_form_scores(ocfg):
    """Collinear pair and hit: c = 0 is accepted; an offset d in y only gives
    c = d^2 exactly for dyadic values, accepted iff d^2 <= C2."""
    x = ocfg.row_x
    # rows 10, 11, 12; a straight line in (y, t) along x
    r = 11
    for d, expect in ((0.0, True), (0.25, True), (0.5, False)):
        w = F(F(x[r] - x[r - 1]) / F(x[r + 1] - x[r - 1]))
        row = np.array([r - 1, r, r + 1], np.uint8)
        y = np.array([0.0, d, 0.0], np.float32)
        t = np.array([5.0, 5.0, 5.0], np.float32)
        up, dn, gap = oracle.links(ocfg, row, y, t)
        assert (up[1] == 2 and dn[1] == 0 and gap[1] == 1) == expect
        # the end rows of this tiny input have no opposite neighbours
        assert up[0] == -1 and up[2] == -1
    # edge rows never get links
    row = np.array([0, 1, 2, 149, 150, 151], np.uint8)
    y = np.zeros(6, np.float32); t = np.zeros(6, np.float32)
    up, dn, gap = oracle.links(ocfg, row, y, t)
    assert up[0] == -1 and up[5] == -1 and up[1] == 2 and dn[1] == 0 and up[4] == 5 and dn[4] == 3


def test_gap_two_only_when_gap_one_fails(ocfg):
    # hit on row 20; nothing on rows 19/21; a pair on 18/22
    row = np.array([18, 20, 22, 19], np.uint8)
    y = np.array([0.0, 0.0, 0.0, 5.0], np.float32)
    t = np.zeros(4, np.float32)
    up, dn, gap = oracle.links(ocfg, row, y, t)
    assert up[1] == 2 and dn[1] == 0 and gap[1] == 2
    # now add a valid gap-1 pair: gap 1 wins even with a worse score
    row = np.array([18, 20, 22, 19, 21], np.uint8)
    y = np.array([0.0, 0.0, 0.0, 0.25, 0.25], np.float32)
    t = np.zeros(5, np.float32)
    up, dn, gap = oracle.links(ocfg, row, y, t)
    assert up[1] == 4 and dn[1] == 3 and gap[1] == 1


def _frame_sector(seed=21):
    fr = synth.generate("slice_1ms", seed=seed, n_collisions=3)
    return fr.sector(5)


def test_time_shift_and_mirror_invariance(ocfg):
    """Shifting time by a multiple of 2^-9 keeps every FP32 difference exact,
    and negating y or t negates every difference exactly: links identical."""
    row, y, t = _frame_sector()
    ref = oracle.links(ocfg, row, y, t)
    for yy, tt in ((y, t + np.float32(1234.5)), (-y, t), (y, -t), (-y, np.float32(777.25) - t)):
        assert np.all(np.abs(tt) < 2 ** 15)
        got = oracle.links(ocfg, row, yy, tt)
        for u, v in zip(ref, got):
            assert np.array_equal(u, v)


def test_chain_invariants(ocfg):
    row, y, t = _frame_sector(22)
    x = ocfg.row_x
    up, dn, gap = oracle.links(ocfg, row, y, t)
    # uncleaned links: rows r +- gap, windows respected
    m = up >= 0
    assert np.array_equal(row[up[m]].astype(int) - row[m], gap[m])
    assert np.array_equal(row[m] - row[dn[m]].astype(int), gap[m])
    assert (np.abs(y[up[m]] - y[m]) <= gap[m] * 1.5).all()
    upc, dnc = oracle.clean(up, dn)
    mc = upc >= 0
    # cleaned links are mutual and a subset of the uncleaned ones
    assert np.array_equal(dnc[upc[mc]], np.nonzero(mc)[0])
    assert np.array_equal(upc[mc], up[mc])
    first, ln, cl, assign = oracle.tracks(ocfg, upc, dnc)
    assert (ln >= ocfg.min_track_hits).all()
    # each cluster in at most one track, assignment consistent with lists
    assert len(np.unique(cl)) == len(cl)
    for k in range(len(first)):
        c = cl[first[k]: first[k] + ln[k]]
        assert (assign[c] == k).all()
        rr = row[c].astype(int)
        assert (np.diff(rr) >= 1).all() and (np.diff(rr) <= 2).all()
        assert dnc[c[0]] < 0 and upc[c[-1]] < 0
    assert (assign >= 0).sum() == ln.sum()
    # tracks numbered by ascending seed index
    seeds = cl[first]
    assert (np.diff(seeds) > 0).all()
    # every seed with a long enough chain is a track
    clen = oracle.chain_len(upc, dnc)
    is_seed = (dnc < 0) & (upc >= 0) & (clen >= ocfg.min_track_hits)
    assert np.array_equal(np.nonzero(is_seed)[0], seeds)


def test_noise_free_separated_particles_give_one_chain(ocfg, geom):
    """Well-separated noise-free helices: every particle's clusters on rows
    1..150 form exactly one chain wherever consecutive rows are present."""
    x, hw = geom
    fr = synth.generate("sector_300", seed=31, fixed_mult=12, sigma_y=0.0, sigma_t=0.0, quant=0.0,
                        noise_frac=0.0, pt_min=1.0)
    row, y, t = fr.sector(0)
    lab = fr.labels[0]
    res = oracle.run_sector(ocfg, row, y, t, fit=False)
    for p in np.unique(lab):
        idx = np.nonzero(lab == p)[0]
        idx = idx[np.argsort(row[idx])]
        rr = row[idx].astype(int)
        if len(idx) < 12 or not (np.diff(rr) == 1).all():
            continue
        inner = idx[(rr >= 1) & (rr <= 150)]
        k = res["assign"][inner[0]]
        assert k >= 0
        assert (res["assign"][inner] == k).all()
        assert (res["assign"][idx[(rr == 0) | (rr == 151)]] == -1).all()
        assert res["len"][k] == len(inner)


def brute_triplets(cfg, row, y, t):
    """Every accepted (down, cluster, up, gap) of every gap, with the number
    of clusters in the two boxes of that gap, enumerated directly from the
    definition (pure Python over all cluster pairs)."""
    n = len(row)
    x = cfg.row_x
    out = []
    for i in range(n):
        r = int(row[i])
        for g in range(1, cfg.max_gap + 1):
            if r - g < 0 or r + g > len(x) - 1:
                continue
            w = F(F(x[r] - x[r - g]) / F(x[r + g] - x[r - g]))
            wy = F(F(g) * F(cfg.win_y)); wt = F(F(g) * F(cfg.win_t))
            D = [d for d in range(n) if row[d] == r - g and abs(F(y[i] - y[d])) <= wy and abs(F(t[i] - t[d])) <= wt]
            U = [u for u in range(n) if row[u] == r + g and abs(F(y[u] - y[i])) <= wy and abs(F(t[u] - t[i])) <= wt]
            for d in D:
                for u in U:
                    ry = F(F(y[i] - y[d]) - F(w * F(y[u] - y[d])))
                    rt = F(F(t[i] - t[d]) - F(w * F(t[u] - t[d])))
                    if F(F(ry * ry) + F(rt * rt)) <= F(cfg.pair_c2):
                        out.append((d, i, u, g, len(D) + len(U)))
    return out


@pytest.mark.parametrize("seed", range(4))
def test_triplets_match_brute_force(ocfg, seed):
    """The triplet enumeration of the pruned finder: exactly the accepted
    pairs of every gap (none missing, none extra, gap 2 listed also where
    gap 1 has pairs), and the density feature = (|D| + |U|) / 8 of the
    boxes of that gap, on tie- and duplicate-heavy tiny inputs."""
    row, y, t = _tiny(100 + seed, 140 + 40 * seed, dup=0.3)
    tri, feat = oracle.triplets(ocfg, row, y, t)
    ref = brute_triplets(ocfg, row, y, t)
    assert len(ref) > 30 and any(g == 2 for _, _, _, g, _ in ref)
    got = sorted(zip(map(tuple, tri.tolist()), feat[:, 11].tolist()))
    exp = sorted(((d, i, u, g), float(oracle.bf16(np.array([F(nb) / F(8.0)], np.float32))[0])) for d, i, u, g, nb in ref)
    assert [k for k, _ in got] == [k for k, _ in exp]
    assert [v for _, v in got] == [v for _, v in exp]
    # features 4 (gap) and 5 (radius) of every triplet, from the definition
    x = ocfg.row_x
    assert np.array_equal(feat[:, 4], tri[:, 3].astype(np.float32))
    assert np.array_equal(feat[:, 5], oracle.bf16(np.asarray(x, np.float32)[row[tri[:, 1]]] / np.float32(245.0)))
    # every uncleaned link is one of the listed gap-g triplets
    up, dn, gap = oracle.links(ocfg, row, y, t)
    s = set(map(tuple, tri.tolist()))
    for i in np.nonzero(up >= 0)[0]:
        assert (dn[i], i, up[i], gap[i]) in s
