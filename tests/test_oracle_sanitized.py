"""The oracle's C code built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code; leaks checked too) and run over one
small sector through every step it implements (links, cleaning, chains, the
MAP and Kalman fits, following, triplets): no error report, and the same
results as the ordinary build."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2102_08862_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _write_input(path, cfg, fcfg, row, y, t):
    rx = np.ascontiguousarray(cfg.row_x, np.float32)
    inv = lambda v: 0.0 if v is None else 1.0 / v
    with open(path, "wb") as fh:
        fh.write(np.array([len(row)], np.int64).tobytes())
        fh.write(np.array([len(rx)], np.int32).tobytes())
        fh.write(rx.tobytes())
        fh.write(np.array([cfg.win_y, cfg.win_t, cfg.pair_c2], np.float32).tobytes())
        fh.write(np.array([cfg.max_gap, cfg.min_track_hits, cfg.max_iter], np.int32).tobytes())
        fh.write(np.array([cfg.bz, cfg.sigma_y, cfg.sigma_t, inv(cfg.var_s), inv(cfg.var_tau), inv(cfg.var_k),
                           cfg.s_max], np.float64).tobytes())
        fh.write(np.array([fcfg.win_y, fcfg.win_t, fcfg.chi2_max, fcfg.q_slope, fcfg.var_y, fcfg.var_t,
                           fcfg.var_slope0], np.float32).tobytes())
        fh.write(np.array([fcfg.max_miss], np.int32).tobytes())
        fh.write(np.ascontiguousarray(row, np.uint8).tobytes())
        fh.write(np.ascontiguousarray(y, np.float32).tobytes())
        fh.write(np.ascontiguousarray(t, np.float32).tobytes())


def _expected(cfg, fcfg, row, y, t):
    up, dn, _ = oracle.links(cfg, row, y, t)
    upc, dnc = oracle.clean(up, dn)
    out = {"links": [int((up >= 0).sum()), int(up.astype(np.int64).sum() + 2 * dn.astype(np.int64).sum()),
                     int((upc >= 0).sum())]}
    first, ln, cl, asg = oracle.tracks(cfg, upc, dnc)
    out["tracks"] = [len(first), int(ln.sum()), int(asg.astype(np.int64).sum())]
    for kf in (0, 3):
        f = oracle.fit_tracks(cfg, first, ln, cl, row, y, t, kf_passes=kf)
        ok = f["status"] == 0
        out["fit%d" % kf] = [int(f["status"].sum()), float(np.sum(f["qpt"][ok])), float(np.sum(f["chi2"][ok]))]
    fo = oracle.follow(cfg, fcfg, row, y, t, first, ln, cl)
    out["follow"] = [len(fo["first"]), int(fo["len"].sum()),
                     int((fo["ext_in"] + 3 * fo["ext_out"] + 7 * fo["kept"]).astype(np.int64).sum())]
    tri, feat = oracle.triplets(cfg, row, y, t)
    out["triplets"] = [len(tri), int(tri.astype(np.int64).sum()), float(feat.astype(np.float64).sum())]
    return out


def test_oracle_under_address_and_ub_sanitizers(ocfg, tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "asan_oracle")
    cmd = ["gcc", "-g", "-O1", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-mfpmath=sse", "-msse2"] + SAN + \
        ["-I" + os.path.join(ROOT, "oracle"), os.path.join(HERE, "asan_oracle.c"),
         os.path.join(ROOT, "oracle", "tpcmlp.c"), "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    fr = synth.generate("sector_300", seed=41)
    row, y, t = fr.sector(0)
    fcfg = oracle.FollowConfig()
    inp = str(tmp_path / "sector.bin")
    _write_input(inp, ocfg, fcfg, row, y, t)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, inp], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
    got = {}
    for line in r.stdout.splitlines():
        k, *v = line.split()
        got[k] = [float(x) if ("." in x or "e" in x) else int(x) for x in v]
    want = _expected(ocfg, fcfg, row, y, t)
    assert set(got) == set(want)
    for k in want:
        for a, b in zip(got[k], want[k]):
            if isinstance(b, float):
                assert abs(a - b) <= 1e-9 * max(1.0, abs(b)), (k, a, b)
            else:
                assert a == b, (k, a, b)
    assert want["tracks"][0] > 10 and want["triplets"][0] > 100
