"""Pins of the oracle's sector merging (R30).

The residuals are pinned by the generator's own helix code (an independent
implementation of the trajectory): a particle's truth states in two
adjacent sectors give zero residuals; by the straight-track limit; and by a
scalar implementation that works from the circle's centre instead of the
closed form. The selection (mutual best under the cut, least index on ties)
is pinned by a pure-Python brute force."""
import numpy as np
import pytest

import oracle
from paper_2102_08862_amd import synth


def _state(tr, sector, x):
    """Truth state at row line x of a sector, if the particle crosses it on
    the sector's own side of the membrane (z > 0 for sectors 0-17)."""
    h = synth.helix_at(tr, sector, float(x), False)
    if h is None:
        return None
    Y, z, sphi, arc, t, dtdl = h
    if z * (1.0 if sector < 18 else -1.0) <= 0:
        return None
    return dict(x=float(x), y=Y, t=t, sinphi=sphi, tau=dtdl, qpt=tr[0] / tr[1], arc=arc)


def test_truth_states_in_adjacent_sectors_match(geom, ocfg):
    x = geom[0]
    fr = synth.generate("slice_1ms", seed=2400, n_threads=8)
    rng = np.random.default_rng(1)
    done = 0
    # pT >= 0.5 GeV: radius above 3 m, so two states of one sector pair lie
    # within half a turn (the nearest point on the circle is defined modulo
    # a turn, and a looper's states can be a turn apart)
    for pid in rng.permutation(len(fr.tracks))[:8000]:
        tr = fr.tracks[pid]
        if tr[1] < 0.5:
            continue
        for s in range(36):
            side, k = divmod(s, 18)
            n = 18 * side + (k + 1) % 18
            a = b = None
            for r in range(151, -1, -10):
                a = a or _state(tr, s, x[r])
            for r in range(0, 152, 10):
                b = b or _state(tr, n, x[r])
            if a is None or b is None:
                continue
            A = {k_: np.array([v]) for k_, v in a.items()}
            B = {k_: np.array([v]) for k_, v in b.items()}
            dr, dphi, dt, dtau = (v[0, 0] for v in oracle.merge_residuals(ocfg, A, B, np.deg2rad(20.0)))
            assert abs(dr) < 1e-6 and abs(dphi) < 1e-9 and abs(dt) < 1e-6 and dtau == 0.0, (pid, s, dr, dphi, dt)
            done += 1
            break
        if done >= 200:
            break
    assert done >= 100


def test_straight_track_limit(ocfg):
    A = dict(x=np.array([100.0]), y=np.array([3.0]), t=np.array([50.0]), sinphi=np.array([0.3]),
             tau=np.array([0.4]), qpt=np.array([0.0]))
    B = dict(x=np.array([140.0]), y=np.array([-20.0]), t=np.array([61.0]), sinphi=np.array([0.1]),
             tau=np.array([0.45]), qpt=np.array([1.0]))
    dal = np.deg2rad(20.0)
    dr, dphi, dt, dtau = (v[0, 0] for v in oracle.merge_residuals(ocfg, A, B, dal))
    bx = 140.0 * np.cos(dal) + 20.0 * np.sin(dal)
    by = 140.0 * np.sin(dal) - 20.0 * np.cos(dal)
    c, s_ = np.sqrt(1 - 0.09), 0.3
    along = (bx - 100.0) * c + (by - 3.0) * s_
    across = -(bx - 100.0) * s_ + (by - 3.0) * c
    assert abs(dr - across) < 1e-9
    assert abs(dt - (50.0 + 0.4 * along - 61.0)) < 1e-9
    assert abs(dphi - (np.arcsin(0.1) + dal - np.arcsin(0.3))) < 1e-12
    assert abs(dtau - (-0.05)) < 1e-12


def _residual_scalar(cfg, a, b, dal):
    """From the circle's centre: the centre lies 1/kappa along A's left
    normal; B's point, seen from the centre, sits at an angle from A's; the
    arc is that angle over kappa, the miss the radius minus the distance."""
    k = -2.99792458e-3 * cfg.bz * a["qpt"]
    phi = np.arcsin(a["sinphi"])
    bx = b["x"] * np.cos(dal) - b["y"] * np.sin(dal)
    by = b["x"] * np.sin(dal) + b["y"] * np.cos(dal)
    if k == 0.0:
        along = (bx - a["x"]) * np.cos(phi) + (by - a["y"]) * np.sin(phi)
        across = -(bx - a["x"]) * np.sin(phi) + (by - a["y"]) * np.cos(phi)
        th, arc, miss = 0.0, along, across
    else:
        cx, cy = a["x"] - np.sin(phi) / k, a["y"] + np.cos(phi) / k
        ang0 = np.arctan2(a["y"] - cy, a["x"] - cx)
        ang1 = np.arctan2(by - cy, bx - cx)
        th = np.arctan2(np.sin(ang1 - ang0), np.cos(ang1 - ang0))
        arc = th / k
        miss = np.sign(k) * (1.0 / abs(k) - np.hypot(bx - cx, by - cy))
    dphi = np.arcsin(b["sinphi"]) + dal - (phi + th)
    return (miss, np.arctan2(np.sin(dphi), np.cos(dphi)), a["t"] + a["tau"] * arc - b["t"], a["tau"] - b["tau"])


@pytest.mark.parametrize("seed", range(4))
def test_merging_by_brute_force(ocfg, seed):
    rng = np.random.default_rng(70 + seed)
    tracks = []
    for s in range(36):
        m = int(rng.integers(0, 7))
        tracks.append(dict(x=rng.uniform(90, 240, m), y=rng.uniform(-30, 30, m), t=rng.uniform(0, 60, m),
                           sinphi=rng.uniform(-0.5, 0.5, m), tau=rng.uniform(-0.5, 0.5, m),
                           qpt=rng.choice([0.0, 0.4, -0.7, 2.0], m), status=rng.choice([0, 0, 0, 2], m),
                           n=rng.integers(20, 80, m), t0=np.round(rng.uniform(0, 30, m))))
    cut = 1e9   # every pair in the window is a candidate: the selection decides
    nxt, prv, _ = oracle.merge_sectors(ocfg, tracks, min_clusters=30, window=8.0, d2_cut=cut)
    sig = oracle.MERGE_SIGMA
    dal = np.deg2rad(20.0)
    for s in range(36):
        side, k = divmod(s, 18)
        n = 18 * side + (k + 1) % 18
        A, B = tracks[s], tracks[n]
        el = lambda T, i: T["status"][i] == 0 and T["n"][i] >= 30
        d2 = {}
        for i in range(len(A["x"])):
            for j in range(len(B["x"])):
                if el(A, i) and el(B, j) and abs(A["t0"][i] - B["t0"][j]) <= 8.0:
                    r = _residual_scalar(ocfg, {k_: A[k_][i] for k_ in A}, {k_: B[k_][j] for k_ in B}, dal)
                    d2[(i, j)] = sum((ri / si) ** 2 for ri, si in zip(r, sig))
        want = [-1] * len(A["x"])
        for (i, j), v in d2.items():
            bi = min((vv, jj) for (ii, jj), vv in d2.items() if ii == i)
            bj = min((vv, ii) for (ii, jj), vv in d2.items() if jj == j)
            if bi[1] == j and bj[1] == i:
                want[i] = j
        assert nxt[s].tolist() == want, (s, nxt[s], want)
        for i, j in enumerate(want):
            if j >= 0:
                assert prv[n][j] == i
    # the residuals themselves against the scalar form
    a = {k_: tracks[0][k_][:3] for k_ in ("x", "y", "t", "sinphi", "tau", "qpt")}
    b = {k_: tracks[1][k_][:3] for k_ in ("x", "y", "t", "sinphi", "tau", "qpt")}
    R = oracle.merge_residuals(ocfg, a, b, dal)
    for i in range(len(a["x"])):
        for j in range(len(b["x"])):
            r = _residual_scalar(ocfg, {k_: a[k_][i] for k_ in a}, {k_: b[k_][j] for k_ in b}, dal)
            assert np.allclose([R[q][i, j] for q in range(4)], r, rtol=0, atol=1e-9)


def test_refit_of_noise_free_pieces_is_truth(geom, ocfg):
    """Exact helix points of one particle in two adjacent sectors: the refit
    of the merged pair, in the first sector's frame, is the truth state at
    its outermost point (the same argument as for one sector's track: the
    three-point estimate is exact, so is the MAP)."""
    x = geom[0]
    fr = synth.generate("slice_1ms", seed=2402, n_threads=8)
    rng = np.random.default_rng(3)
    dal = np.deg2rad(20.0)
    done = 0
    for pid in rng.permutation(len(fr.tracks))[:20000]:
        tr = fr.tracks[pid]
        if tr[1] < 0.5:
            continue
        for s in range(36):
            side, k = divmod(s, 18)
            n = 18 * side + (k + 1) % 18
            pa = [(float(x[r]), _state(tr, s, x[r])) for r in range(152)]
            pb = [(float(x[r]), _state(tr, n, x[r])) for r in range(152)]
            # the crossings inside each sector's azimuthal acceptance (20 degrees)
            pa = [(xx, h) for xx, h in pa if h is not None and abs(h["y"]) <= xx * np.tan(dal / 2)]
            pb = [(xx, h) for xx, h in pb if h is not None and abs(h["y"]) <= xx * np.tan(dal / 2)]
            if len(pa) < 8 or len(pb) < 8:
                continue
            xa = np.array([v[0] for v in pa]); ya = np.array([v[1]["y"] for v in pa])
            ta = np.array([v[1]["t"] for v in pa])
            xb = np.array([v[0] for v in pb]); yb = np.array([v[1]["y"] for v in pb])
            tb = np.array([v[1]["t"] for v in pb])
            f = oracle.refit_merged(ocfg, xa, ya, ta, xb, yb, tb, dal)
            xr = max(xa.max(), (xb * np.cos(dal) - yb * np.sin(dal)).max())
            assert f["status"] == 0 and abs(f["x_ref"] - xr) < 1e-12
            tru = _state(tr, s, xr)
            if tru is None or abs(tru["sinphi"]) > 0.95:
                continue
            got = np.array([f["y"], f["t"], f["sinphi"], f["tau"], f["qpt"]])
            want = np.array([tru["y"], tru["t"], tru["sinphi"], tru["tau"], tru["qpt"]])
            assert np.allclose(got, want, rtol=1e-8, atol=1e-8), (pid, s, got, want)
            assert f["chi2"] < 1e-10
            done += 1
            break
        if done >= 40:
            break
    assert done >= 20


def _side_state(tr, sector, x):
    """Truth state (with the collision time of its own side's track) at row
    line x of a sector, inside the sector's azimuthal acceptance, on the
    sector's own side of the membrane."""
    h = _state(tr, sector, x)
    if h is None or abs(h["y"]) > x * np.tan(np.deg2rad(10.0)):
        return None
    return h


def test_truth_pieces_across_the_membrane_match(geom, ocfg):
    """A particle that crosses z = 0 inside the drift volume: its truth
    states on the two sides (the A side's at its innermost row, the C
    side's at its outermost, so that the crossing lies between them,
    whichever side the particle starts on) give zero transverse residuals, opposite tau,
    collision times (track_t0 of each state) that differ by twice the vertex
    z, time lines that meet at the arc where z = 0, and that arc between the
    states' reference arcs."""
    x = geom[0]
    fr = synth.generate("frame_10ms", seed=2403, n_threads=8, frame_us=400.0, n_collisions=20)
    done = 0
    for pid in range(len(fr.tracks)):
        tr = fr.tracks[pid]
        q, pt, phi0, tgl, zv = tr[:5]
        if pt < 0.5 or tgl == 0.0:
            continue
        s_cross = -zv / tgl
        if not (x[10] < s_cross < x[140]):
            continue
        for k in range(18):
            a = b = None
            for r in range(152):
                a = a or _side_state(tr, k, x[r])
                b = b or _side_state(tr, k + 18, x[151 - r])
            if a is None or b is None:
                continue
            A = {k_: np.array([v]) for k_, v in a.items()}
            B = {k_: np.array([v]) for k_, v in b.items()}
            for T in (A, B):
                T["t0"] = oracle.track_t0(ocfg, T["x"], T["y"], T["t"], T["sinphi"], T["tau"], T["qpt"])
            dr, dphi, dtau, meet = (v[0, 0] for v in oracle.membrane_residuals(ocfg, A, B))
            assert abs(dr) < 1e-6 and abs(dphi) < 1e-9 and dtau == 0.0 and meet, (pid, k, dr, dphi, dtau)
            assert abs((B["t0"][0] - A["t0"][0]) - 2.0 * zv) < 1e-6
            s_meet = (B["t0"][0] - A["t0"][0]) / (A["tau"][0] - B["tau"][0])
            assert abs(s_meet - s_cross) < 1e-6 * max(1.0, s_cross), (s_meet, s_cross)
            ra = oracle.ref_arc(ocfg, A["x"], A["y"], A["sinphi"], A["qpt"])[0]
            rb = oracle.ref_arc(ocfg, B["x"], B["y"], B["sinphi"], B["qpt"])[0]
            assert min(ra, rb) <= s_cross <= max(ra, rb), (ra, rb, s_cross)
            # the arc of each state: that of the generator's own helix
            assert abs(ra - a["arc"]) < 1e-6 and abs(rb - b["arc"]) < 1e-6, (ra, a["arc"], rb, b["arc"])
            done += 1
            break
        if done >= 30:
            break
    assert done >= 10


def _ref_arc_scalar(cfg, T):
    """Arc from the beam line's closest approach to the state, from the
    circle's centre: the closest point of the circle to the origin lies on
    the ray from the centre through the origin."""
    k = -2.99792458e-3 * cfg.bz * T["qpt"]
    phi = np.arcsin(T["sinphi"])
    if k == 0.0:
        return T["x"] * np.cos(phi) + T["y"] * np.sin(phi)
    cx, cy = T["x"] - np.sin(phi) / k, T["y"] + np.cos(phi) / k
    d = np.arctan2(T["y"] - cy, T["x"] - cx) - np.arctan2(-cy, -cx)
    return np.arctan2(np.sin(d), np.cos(d)) / k


def _meet_scalar(cfg, A, B):
    """Is there an arc s between the pieces' reference arcs (widened by 5
    cm) where the time lines t0 + tau s of A and B agree within 1 cm?"""
    sa, sb = _ref_arc_scalar(cfg, A), _ref_arc_scalar(cfg, B)
    lo, hi = min(sa, sb) - 5.0, max(sa, sb) + 5.0
    D = A["tau"] - B["tau"]
    dT = B["t0"] - A["t0"]
    s = min(max(dT / D, lo), hi) if D != 0.0 else lo
    return abs(dT - D * s) <= 1.0


@pytest.mark.parametrize("seed", range(4))
def test_membrane_merging_by_brute_force(ocfg, seed):
    rng = np.random.default_rng(90 + seed)
    tracks = []
    for s in range(36):
        m = int(rng.integers(0, 7))
        tracks.append(dict(x=rng.uniform(90, 240, m), y=rng.uniform(-30, 30, m), t=rng.uniform(0, 60, m),
                           sinphi=rng.uniform(-0.5, 0.5, m), tau=rng.choice([-0.1, -0.02, 0.0, 0.03, 0.1], m),
                           qpt=rng.choice([0.0, 0.4, -0.7, 2.0], m), status=rng.choice([0, 0, 0, 2], m),
                           n=rng.integers(20, 80, m), t0=np.round(rng.uniform(0, 40, m))))
    cut = 1e9   # every pair in the window whose time lines meet is a candidate
    part, _ = oracle.merge_membrane(ocfg, tracks, min_clusters=30, window=30.0, d2_cut=cut)
    sig = oracle.MERGE_SIGMA
    for k in range(18):
        A, B = tracks[k], tracks[k + 18]
        el = lambda T, i: T["status"][i] == 0 and T["n"][i] >= 30
        d2 = {}
        for i in range(len(A["x"])):
            for j in range(len(B["x"])):
                if not (el(A, i) and el(B, j) and abs(A["t0"][i] - B["t0"][j]) <= 30.0):
                    continue
                Ai, Bj = {k_: A[k_][i] for k_ in A}, {k_: B[k_][j] for k_ in B}
                if not _meet_scalar(ocfg, Ai, Bj):
                    continue
                r = _residual_scalar(ocfg, Ai, Bj, 0.0)
                d2[(i, j)] = (r[0] / sig[0]) ** 2 + (r[1] / sig[1]) ** 2 + ((A["tau"][i] + B["tau"][j]) / sig[3]) ** 2
        want_a = [-1] * len(A["x"])
        want_b = [-1] * len(B["x"])
        for (i, j), v in d2.items():
            bi = min((vv, jj) for (ii, jj), vv in d2.items() if ii == i)
            bj = min((vv, ii) for (ii, jj), vv in d2.items() if jj == j)
            if bi[1] == j and bj[1] == i:
                want_a[i] = j
                want_b[j] = i
        assert list(part[k]) == want_a, (k, list(part[k]), want_a)
        assert list(part[k + 18]) == want_b
    assert sum(int((p >= 0).sum()) for p in part[:18]) > 0
