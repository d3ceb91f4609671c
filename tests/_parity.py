"""Helpers shared by the GPU parity tests: run the HIP library on a sector
and compare every output with the CPU oracle on the same inputs."""
import numpy as np

import oracle

# parameter tolerance: |gpu - oracle| <= REL * max(|oracle|, floor). The
# floors are set at a fraction of each parameter's natural scale:
#   y, dt: 1 cm. dt = t - t_base is a residual-sized number (~0.1 cm) while
#     the fit carries time over a track's drift span of up to ~10^2 cm in
#     FP32 (resolution ~1e-5 cm), and y is mostly 10-40 cm;
#   sin phi, tau: 0.1. Both are O(1) slopes that the FP32 filter carries
#     through one transport per cluster; the GPU's passes stop once a pass
#     moves a slope by at most 1e-5 of max(|value|, 0.1), so below 0.1 the
#     check is absolute at 1e-5 and above it relative;
#   q/pT: 0.1 1/GeV (pT = 10 GeV; |q/pT| of the generated tracks lies in
#     (0, 10] 1/GeV), with the same stopping rule, or the oracle's own
#     standard error of q/pT where that is larger: on a short straight track
#     q/pT is known to +-1 1/GeV or worse, FP32 predictions (rounding ~1e-6 cm)
#     pin the MAP to a few 1e-6 of that error, and 1e-4 of it is the
#     relative agreement that the data can define.
# The pure relative error (no floor) is reported beside it.
REL = 1e-4
FLOORS = {"y": 1.0, "dt": 1.0, "sinphi": 0.1, "tau": 0.1, "qpt": 0.1}
CHI2_REL = 1e-3
S_NEAR = 0.99      # |sin phi| beyond which one side's transport may fail and the other's not


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
    # an exclusion must be explained: both sides failed alike, one side did
    # not converge, or the helix reaches |sin phi| >= S_NEAR on the chain
    # (sin phi is linear in x, so its extremes are at the chain's ends)
    x1 = x[row[ref["clusters"][ref["first"]]]].astype(np.float64)
    why = {"both_failed": 0, "not_converged": 0, "sinphi_limit": 0}
    for k in np.nonzero(~ok)[0]:
        gs, fs = int(tracks["status"][k]), int(fit["status"][k])
        if gs == fs == 2:
            why["both_failed"] += 1
            continue
        if gs == 4 or fs == 4:
            why["not_converged"] += 1
            continue
        near = False
        for sl, q in ((float(fit["sinphi"][k]), float(fit["qpt"][k])), (float(tracks["sinphi"][k]), float(tracks["qpt"][k]))):
            s1 = sl + 2.99792458e-3 * ocfg.bz * q * (float(tracks["x_ref"][k]) - x1[k])
            near = near or max(abs(sl), abs(s1)) >= S_NEAR
        init_s = abs(float(fit["init"][k][2]))
        assert near or init_s >= S_NEAR, "track %d excluded (gpu status %d, oracle %d) far from the sin phi limit" % (
            k, gs, fs)
        why["sinphi_limit"] += 1
    worst = 0.0
    pure = {}
    if ok.any():
        g = tracks[ok]
        f = fit[ok]
        t_base = g["t_base"].astype(np.float64)
        cols = {"y": (g["y"], f["y"]), "dt": (g["dt"], f["t"] - t_base), "sinphi": (g["sinphi"], f["sinphi"]),
                "tau": (g["tau"], f["tau"]), "qpt": (g["qpt"], f["qpt"])}
        floors = dict(FLOORS)
        floors["qpt"] = np.maximum(FLOORS["qpt"], np.sqrt(np.maximum(f["cov"][:, 14], 0.0)))
        for k, (a, b) in cols.items():
            a = a.astype(np.float64)
            d = np.abs(a - b)
            rel = d / np.maximum(np.abs(b), floors[k])
            i = int(np.argmax(rel))
            assert rel[i] <= REL, "param %s: gpu %r oracle %r (rel %.3g, track %d)" % (k, a[i], b[i], rel[i], i)
            worst = max(worst, float(rel.max()))
            nz = np.abs(b) > 0
            pure[k] = float(np.percentile(d[nz] / np.abs(b[nz]), 99.9)) if nz.any() else 0.0
        c = g["chi2"].astype(np.float64)
        relc = np.abs(c - f["chi2"]) / np.maximum(f["chi2"], 1.0)
        assert relc.max() <= CHI2_REL, "chi2 rel %.3g" % relc.max()
        assert np.array_equal(g["ndf"], f["ndf"])
    assert excluded <= max(2, len(tracks) // 100), "%d tracks with a failed fit on one side" % excluded
    return dict(worst=worst, excluded=excluded, excluded_why=why, pure_rel_p999=pure)
