"""Input generator checks: the helix geometry against an independent RK4
integration of the Lorentz force, determinism, and workload shapes."""
import math

import numpy as np
import pytest

from paper_2102_08862_amd import synth

KB = 2.99792458e-3


def _rk4_crossing(track, alpha, xrow, bz=0.5, h=0.05):
    """Integrate d(pos)/dl = u, du/dl = a*(u_y, -u_x) (force q v x B with B
    along +z, a = q kB Bz / pT) from the origin; return the local Y and arc
    length at the first rising crossing of X = xrow in the frame rotated by
    alpha, within half a turn."""
    q, pt, phi0 = track[0], track[1], track[2]
    a = q * KB * bz / pt

    def f(s):
        return np.array([s[2], s[3], a * s[3], -a * s[2]])

    s = np.array([0.0, 0.0, math.cos(phi0), math.sin(phi0)])
    ca, sa = math.cos(alpha), math.sin(alpha)

    def X(s):
        return s[0] * ca + s[1] * sa

    def step(s, hh):
        k1 = f(s); k2 = f(s + 0.5 * hh * k1); k3 = f(s + 0.5 * hh * k2); k4 = f(s + hh * k3)
        return s + hh / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)

    lmax = math.pi * pt / (KB * bz)
    l = 0.0
    while l < lmax:
        sn = step(s, h)
        if X(s) < xrow <= X(sn) and (sn[2] * ca + sn[3] * sa) > 0:
            lo, hi = 0.0, h
            for _ in range(60):
                mid = 0.5 * (lo + hi)
                if X(step(s, mid)) < xrow:
                    lo = mid
                else:
                    hi = mid
            se = step(s, 0.5 * (lo + hi))
            return -se[0] * sa + se[1] * ca, l + 0.5 * (lo + hi)
        s, l = sn, l + h
    return None


def test_helix_matches_rk4_lorentz(geom):
    x, hw = geom
    fr = synth.generate("sector_300", seed=11, sigma_y=0.0, sigma_t=0.0, quant=0.0, noise_frac=0.0)
    tr = fr.tracks
    alpha0 = math.radians(10.0)
    checked = 0
    for j in range(0, len(tr), 15):
        for r in (0, 40, 90, 151):
            h = synth.helix_at(tr[j], 0, float(x[r]), True)
            rk = _rk4_crossing(tr[j], alpha0, float(x[r]))
            if h is None:
                assert rk is None or abs(rk[0]) > 1e3  # no crossing on the outgoing half turn
                continue
            assert rk is not None
            assert abs(h[0] - rk[0]) < 1e-7
            assert abs(h[3] - rk[1]) < 1e-7
            assert abs(h[1] - (tr[j][4] + tr[j][3] * rk[1])) < 1e-7
            checked += 1
    assert checked > 20


def test_clusters_lie_on_helix(geom):
    """Noise-free clusters are the helix crossings (y exact up to FP32 storage)."""
    x, hw = geom
    fr = synth.generate("sector_300", seed=3, sigma_y=0.0, sigma_t=0.0, quant=0.0, noise_frac=0.0)
    row, y, t = fr.sector(0)
    lab = fr.labels[0]
    assert (lab >= 0).all()
    for i in range(0, len(row), 97):
        h = synth.helix_at(fr.tracks[lab[i]], 0, float(x[row[i]]), True)
        assert h is not None
        assert abs(np.float32(h[0]) - y[i]) == 0.0
        assert abs(np.float32(h[4]) - t[i]) == 0.0
        assert abs(h[0]) <= hw[row[i]] + 1e-6


def test_deterministic_and_thread_independent():
    a = synth.generate("slice_1ms", seed=77, n_threads=1, n_collisions=4)
    b = synth.generate("slice_1ms", seed=77, n_threads=7, n_collisions=4)
    for s in range(36):
        for fa, fb in ((a.rows, b.rows), (a.ys, b.ys), (a.ts, b.ts), (a.labels, b.labels)):
            assert np.array_equal(fa[s], fb[s])
    c = synth.generate("slice_1ms", seed=78, n_threads=3, n_collisions=4)
    assert c.n_clusters != a.n_clusters or not np.array_equal(c.ys[0], a.ys[0])


def test_workload_shapes(geom):
    x, hw = geom
    fr = synth.generate("slice_1ms", seed=5, n_collisions=6)
    lo, hi = fr.t_range
    assert lo == 0.0 and abs(hi - (2.58 * 1000 + 250)) < 1e-9
    q = 1.0 / 512
    for s in range(36):
        row, y, t = fr.sector(s)
        lab = fr.labels[s]
        assert row.max() < 152
        assert (np.abs(y) <= hw[row] + 0.1 * 7).all()  # smearing beyond the edge
        # quantised to 2^-9 cm
        assert np.array_equal(np.round(y.astype(np.float64) * 512), y.astype(np.float64) * 512)
        assert np.array_equal(np.round(t.astype(np.float64) * 512), t.astype(np.float64) * 512)
        sig = (lab >= 0).sum()
        assert (lab < 0).sum() == math.floor(0.05 * sig + 0.5)  # llround: halves away from 0
    # A side clusters come from z > 0: t = v t_c + (250 - z) <= v t_c + 250
    tr = fr.tracks
    row, y, t = fr.sector(3)
    lab = fr.labels[3]
    m = lab >= 0
    tc = tr[lab[m], 5]
    assert (t[m] <= 2.58 * tc + 250 + 1.0).all()
