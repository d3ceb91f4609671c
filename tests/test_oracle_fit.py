"""Pins of the oracle's FP64 helix fit.

Pinned against things other than itself: the generator's exact helix (whose
geometry is pinned by an RK4 Lorentz-force integration), central finite
differences of the transport, textbook straight-line least squares in the
zero-field case, stationarity of the objective, and the chi2 / pull
statistics of the cluster error model."""
import math

import numpy as np
import pytest

import oracle
from paper_2102_08862_amd import synth

KB = 2.99792458e-3 * 0.5


def _truth_state(track8, sector, x, single):
    h = synth.helix_at(track8, sector, float(x), single)
    if h is None:
        return None
    Y, z, s, arc, t, tau = h
    return np.array([Y, t, s, tau, track8[0] / track8[1]])


@pytest.mark.parametrize("workload,single,sector", [("sector_300", True, 0), ("slice_1ms", False, 4),
                                                    ("slice_1ms", False, 22)])
def test_transport_matches_truth_helix(ocfg, geom, workload, single, sector):
    x, hw = geom
    kw = dict(sigma_y=0.0, sigma_t=0.0, quant=0.0, noise_frac=0.0)
    if not single:
        kw["n_collisions"] = 1
    fr = synth.generate(workload, seed=13, **kw)
    lab = fr.labels[sector]
    row = fr.rows[sector]
    n = 0
    for p in np.unique(lab)[:80]:
        rr = np.sort(row[lab == p])
        if len(rr) < 3:
            continue
        r0, r1 = int(rr[0]), int(rr[-1])
        a = _truth_state(fr.tracks[p], sector, x[r0], single)
        b = _truth_state(fr.tracks[p], sector, x[r1], single)
        if a is None or b is None or abs(b[2]) > 0.99:
            continue
        res = oracle.propagate(ocfg, a, float(x[r1]) - float(x[r0]))
        assert res is not None
        q, F = res
        assert np.allclose(q[:3], b[:3], rtol=0, atol=1e-9), (p, q, b)
        assert abs(q[3] - b[3]) < 1e-12 and abs(q[4] - b[4]) < 1e-12
        # and back again
        back = oracle.propagate(ocfg, q, float(x[r0]) - float(x[r1]))
        assert np.allclose(back[0], a, rtol=0, atol=1e-9)
        n += 1
    assert n > 10


def test_transport_jacobian_matches_finite_differences(ocfg):
    rng = np.random.default_rng(2)
    for _ in range(200):
        q = np.array([rng.uniform(-30, 30), rng.uniform(0, 20000), rng.uniform(-0.6, 0.6),
                      rng.uniform(-1.2, 1.2), rng.uniform(-6, 6)])
        dx = rng.uniform(-120, 120)
        res = oracle.propagate(ocfg, q, dx)
        if res is None:
            continue
        _, F = res
        for a in range(5):
            h = 1e-6 * max(1.0, abs(q[a]))
            qp = q.copy(); qp[a] += h
            qm = q.copy(); qm[a] -= h
            rp = oracle.propagate(ocfg, qp, dx); rm = oracle.propagate(ocfg, qm, dx)
            if rp is None or rm is None:
                continue
            col = (rp[0] - rm[0]) / (2 * h)
            assert np.allclose(F[:, a], col, rtol=1e-5, atol=1e-6 * max(1.0, abs(dx))), (a, F[:, a], col)


def _exact_points(track8, sector, rows, x, single):
    pts = [synth.helix_at(track8, sector, float(x[r]), single) for r in rows]
    if any(p is None for p in pts):
        return None
    return (np.array([float(x[r]) for r in rows]), np.array([p[0] for p in pts]), np.array([p[4] for p in pts]))


def test_map_of_noise_free_helix_is_truth(ocfg, geom):
    """Exact helix points: the three-point estimate is the truth, so the prior
    centres are the truth and the MAP is the truth."""
    x, hw = geom
    fr = synth.generate("sector_300", seed=17, sigma_y=0.0, sigma_t=0.0, quant=0.0, noise_frac=0.0)
    n = 0
    for p in range(len(fr.tracks)):
        rr = np.sort(fr.rows[0][fr.labels[0] == p]).astype(int)
        if len(rr) < 10:
            continue
        rows = rr[: min(len(rr), 80)]
        pts = _exact_points(fr.tracks[p], 0, rows, x, True)
        if pts is None:
            continue
        tru = _truth_state(fr.tracks[p], 0, x[rows[-1]], True)
        if abs(tru[2]) > 0.95:
            continue
        for fit in (oracle.fit_map(ocfg, *pts), oracle.fit_kf(ocfg, *pts, passes=3)):
            assert fit["status"] == 0
            got = np.array([fit["y"], fit["t"], fit["sinphi"], fit["tau"], fit["qpt"]])
            assert np.allclose(got, tru, rtol=1e-9, atol=1e-9), (p, got, tru)
            assert fit["chi2"] < 1e-12
        n += 1
    assert n > 20


def test_zero_field_no_prior_is_straight_line_least_squares(geom):
    """B = 0, priors on the slopes off: the MAP is the pair of ordinary
    least-squares lines y(x), t(x) (numpy.polyfit), re-expressed as
    sin(phi) = m / sqrt(1 + m^2), dt/darc = n / sqrt(1 + m^2)."""
    x, hw = geom
    cfg = oracle.Config(row_x=x, bz=0.0, var_s=None, var_tau=None, var_k=100.0)
    rng = np.random.default_rng(5)
    for trial in range(30):
        r0 = int(rng.integers(0, 100)); L = int(rng.integers(10, 152 - r0))
        rows = np.arange(r0, r0 + L)
        xx = x[rows].astype(np.float64)
        a, m, b, nn = rng.uniform(-20, 20), rng.uniform(-0.8, 0.8), rng.uniform(0, 2e4), rng.uniform(-1, 1)
        y = a + m * xx + rng.normal(0, 0.1, L)
        t = b + nn * xx + rng.normal(0, 0.1, L)
        fit = oracle.fit_map(cfg, xx, y, t)
        assert fit["status"] == 0
        py = np.polyfit(xx, y, 1); pt = np.polyfit(xx, t, 1)
        xl = xx[-1]
        ms = py[0]
        norm = math.sqrt(1 + ms * ms)
        assert abs(fit["y"] - np.polyval(py, xl)) < 1e-9
        assert abs(fit["t"] - np.polyval(pt, xl)) < 1e-7
        assert abs(fit["sinphi"] - ms / norm) < 1e-10
        assert abs(fit["tau"] - pt[0] / norm) < 1e-10
        rss = ((y - np.polyval(py, xx)) ** 2).sum() + ((t - np.polyval(pt, xx)) ** 2).sum()
        assert abs(fit["chi2"] - rss / 0.01) < 1e-6 * max(1, rss / 0.01)


def _sector_tracks(ocfg, seed, **kw):
    fr = synth.generate("sector_300", seed=seed, **kw)
    row, y, t = fr.sector(0)
    res = oracle.run_sector(ocfg, row, y, t)
    return fr, row, y, t, res


def test_map_is_a_stationary_minimum(ocfg, geom):
    x, hw = geom
    fr, row, y, t, res = _sector_tracks(ocfg, 23)
    fit = res["fit"]
    n = 0
    for k in range(0, len(fit), 5):
        if fit[k]["status"] != 0:
            continue
        c = res["clusters"][res["first"][k]: res["first"][k] + res["len"][k]]
        xx = x[row[c]].astype(np.float64); yy = y[c].astype(np.float64); tt = t[c].astype(np.float64)
        qL = np.array([fit[k]["y"], fit[k]["t"], fit[k]["sinphi"], fit[k]["tau"], fit[k]["qpt"]])
        q1 = oracle.propagate(ocfg, qL, xx[0] - xx[-1])[0]
        q0 = np.array(fit[k]["init"])
        c0 = oracle.map_cost(ocfg, xx, yy, tt, q1, q0)
        assert abs(c0 - (fit[k]["chi2"] + sum(((q0[a] - q1[a]) ** 2) * w for a, w in ((2, 1.0), (3, 1.0), (4, 0.01))))) < 1e-6 * c0
        for a in range(5):
            h = 1e-4 * max(1.0, abs(q1[a])) if a != 1 else 1e-4
            for sgn in (1, -1):
                qq = q1.copy(); qq[a] += sgn * h
                assert oracle.map_cost(ocfg, xx, yy, tt, qq, q0) >= c0 - 1e-9 * c0
            qp = q1.copy(); qp[a] += h * 1e-2
            qm = q1.copy(); qm[a] -= h * 1e-2
            grad = (oracle.map_cost(ocfg, xx, yy, tt, qp, q0) - oracle.map_cost(ocfg, xx, yy, tt, qm, q0)) / (2 * h * 1e-2)
            # curvature scale of the objective along this axis
            qp2 = q1.copy(); qp2[a] += h
            curv = 2 * (oracle.map_cost(ocfg, xx, yy, tt, qp2, q0) - c0) / h ** 2
            assert abs(grad) <= 1e-3 * max(curv * h, 1e-6)
        n += 1
    assert n > 10


def test_chi2_and_pulls(ocfg, geom):
    """Fit residual statistics match the cluster error model: chi2/ndf ~ 1
    and pulls of the parameters w.r.t. the generated truth ~ N(0, 1)."""
    x, hw = geom
    chi, pulls = [], {a: [] for a in range(5)}
    for seed in range(40, 46):
        fr, row, y, t, res = _sector_tracks(ocfg, seed)
        lab = fr.labels[0]
        fit = res["fit"]
        for k in range(len(fit)):
            c = res["clusters"][res["first"][k]: res["first"][k] + res["len"][k]]
            labs = lab[c]
            if fit[k]["status"] != 0 or len(c) < 40 or not (labs == labs[0]).all() or labs[0] < 0:
                continue
            tru = _truth_state(fr.tracks[labs[0]], 0, x[row[c[-1]]], True)
            if tru is None:
                continue
            chi.append(fit[k]["chi2"] / fit[k]["ndf"])
            est = np.array([fit[k]["y"], fit[k]["t"], fit[k]["sinphi"], fit[k]["tau"], fit[k]["qpt"]])
            cov = fit[k]["cov"]
            diag = [cov[0], cov[2], cov[5], cov[9], cov[14]]
            for a in range(5):
                pulls[a].append((est[a] - tru[a]) / math.sqrt(diag[a]))
    chi = np.array(chi)
    assert len(chi) > 300
    assert abs(chi.mean() - 1.0) < 0.03
    for a in range(5):
        pa = np.array(pulls[a])
        assert abs(pa.mean()) < 0.15, (a, pa.mean())
        assert 0.85 < pa.std() < 1.15, (a, pa.std())


def test_kalman_diagnostic_converges_to_map(ocfg):
    fr, row, y, t, res = _sector_tracks(ocfg, 29)
    kf = oracle.fit_tracks(ocfg, res["first"], res["len"], res["clusters"], row, y, t, kf_passes=5)
    mp = res["fit"]
    ok = (kf["status"] == 0) & (mp["status"] == 0)
    assert ok.sum() > 100
    tb = t[res["clusters"][res["first"] + res["len"] - 1]].astype(np.float64)
    for key, floor in (("y", 1.0), ("sinphi", 1.0), ("tau", 1.0), ("qpt", 1.0)):
        d = np.abs(kf[key][ok] - mp[key][ok])
        assert (d <= 1e-6 * np.maximum(np.abs(mp[key][ok]), floor)).all(), key
    d = np.abs((kf["t"] - tb)[ok] - (mp["t"] - tb)[ok])
    assert (d <= 1e-6).all()


def test_map_converges_on_short_tracks_of_a_slice(ocfg):
    """Every MAP fit of a sector of a 1 ms slice (many short, poorly curved
    chains) that starts also converges, and its result is a stationary point:
    the objective at the reported helix is not lowered by a small move of
    q/pT, the parameter that the data of short tracks constrain least."""
    fr = synth.generate("slice_1ms", seed=2301, n_threads=8)
    row, y, t = fr.sector(5)
    res = oracle.run_sector(ocfg, row, y, t)
    fit = res["fit"]
    assert len(fit) > 3000
    assert (fit["status"] != 4).all(), np.bincount(fit["status"])
    x = np.asarray(ocfg.row_x, np.float64)
    short = np.nonzero((fit["status"] == 0) & (res["len"] <= 12))[0]
    assert len(short) > 100
    for k in short[:40]:
        c = res["clusters"][res["first"][k]: res["first"][k] + res["len"][k]]
        xx = x[row[c]]; yy = y[c].astype(np.float64); tt = t[c].astype(np.float64)
        qL = np.array([fit[k]["y"], fit[k]["t"], fit[k]["sinphi"], fit[k]["tau"], fit[k]["qpt"]])
        q1 = oracle.propagate(ocfg, qL, xx[0] - xx[-1])[0]
        q0 = np.array(fit[k]["init"])
        c0 = oracle.map_cost(ocfg, xx, yy, tt, q1, q0)
        h = 1e-3 * math.sqrt(fit[k]["cov"][14])
        for sgn in (1, -1):
            qq = q1.copy()
            qq[4] += sgn * h
            assert oracle.map_cost(ocfg, xx, yy, tt, qq, q0) >= c0 - 1e-12 * c0
