"""Helpers shared by the GPU parity tests: run the HIP library on a sector
and compare every output with the CPU oracle on the same inputs."""
import numpy as np

import oracle

# parameter tolerance: |gpu - oracle| <= REL * max(|oracle|, floor)
REL = 1e-4
FLOORS = {"y": 1.0, "dt": 1.0, "sinphi": 1.0, "tau": 1.0, "qpt": 1.0}
CHI2_REL = 1e-3


def oracle_cfg(x, **kw):
    return oracle.Config(row_x=x, **kw)


def compare_sector(trk, frame, sector, row, y, t, ocfg, ref=None, check_params=True):
    """Bit-exact links (uncleaned and cleaned), assignment, track identities
    and cluster lists; parameters within REL. Returns a summary dict."""
    if ref is None:
        ref = oracle.run_sector(ocfg, row, y, t)
    up, dn = trk.links(frame, sector, cleaned=False)
    assert np.array_equal(up, ref["up"]), "up links differ at %s" % np.nonzero(up != ref["up"])[0][:10]
    assert np.array_equal(dn, ref["dn"]), "down links differ at %s" % np.nonzero(dn != ref["dn"])[0][:10]
    upc, dnc = trk.links(frame, sector, cleaned=True)
    assert np.array_equal(upc, ref["upc"]) and np.array_equal(dnc, ref["dnc"])
    assign = trk.assignment(frame, sector)
    assert np.array_equal(assign, ref["assign"]), "assignment differs"
    cl = trk.track_clusters(frame, sector)
    assert np.array_equal(cl, ref["clusters"]), "cluster lists differ"
    tracks = trk.tracks(frame, sector)
    assert len(tracks) == len(ref["first"])
    assert np.array_equal(tracks["first"], ref["first"])
    assert np.array_equal(tracks["n_clusters"], ref["len"])
    if len(tracks):
        assert np.array_equal(tracks["seed"], ref["clusters"][ref["first"]])
        assert (tracks["frame"] == frame).all() and (tracks["sector"] == sector).all()
    out = dict(n=len(row), links=int((up >= 0).sum()), tracks=len(tracks), worst=0.0, excluded=0)
    if check_params and len(tracks):
        out.update(compare_params(tracks, ref, row, y, t, ocfg))
    return out


def compare_params(tracks, ref, row, y, t, ocfg):
    fit = ref["fit"] if "fit" in ref else oracle.fit_tracks(ocfg, ref["first"], ref["len"], ref["clusters"], row, y, t)
    last = ref["clusters"][ref["first"] + ref["len"] - 1]
    x = np.asarray(ocfg.row_x, np.float32)
    assert np.array_equal(tracks["x_ref"], x[row[last]])
    assert np.array_equal(tracks["t_base"], t[last])
    ok = (tracks["status"] == 0) & (fit["status"] == 0)
    excluded = int((~ok).sum())
    # a status disagreement is only allowed at the |sin phi| limit
    worst = 0.0
    if ok.any():
        g = tracks[ok]
        f = fit[ok]
        t_base = g["t_base"].astype(np.float64)
        cols = {"y": (g["y"], f["y"]), "dt": (g["dt"], f["t"] - t_base), "sinphi": (g["sinphi"], f["sinphi"]),
                "tau": (g["tau"], f["tau"]), "qpt": (g["qpt"], f["qpt"])}
        for k, (a, b) in cols.items():
            a = a.astype(np.float64)
            rel = np.abs(a - b) / np.maximum(np.abs(b), FLOORS[k])
            i = int(np.argmax(rel))
            assert rel[i] <= REL, "param %s: gpu %r oracle %r (rel %.3g, track %d)" % (k, a[i], b[i], rel[i], i)
            worst = max(worst, float(rel.max()))
        c = g["chi2"].astype(np.float64)
        relc = np.abs(c - f["chi2"]) / np.maximum(f["chi2"], 1.0)
        assert relc.max() <= CHI2_REL, "chi2 rel %.3g" % relc.max()
        assert np.array_equal(g["ndf"], f["ndf"])
    assert excluded <= max(2, len(tracks) // 100), "%d tracks with a failed fit on one side" % excluded
    return dict(worst=worst, excluded=excluded)
