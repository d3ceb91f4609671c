"""The worked example in tests/golden/worked_example.json: a hand-built
sector (two straight particles and a noise cluster) whose links, chains,
assignment and helix parameters are known in closed form (derivation in
tests/golden/make_worked_example.py). The oracle must reproduce it on the
CPU; the GPU library must too (marked gpu)."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2102_08862_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ex():
    with open(os.path.join(HERE, "golden", "worked_example.json")) as fh:
        d = json.load(fh)
    d["row_a"] = np.array(d["row"], np.uint8)
    d["y_a"] = np.array(d["y"], np.float32)
    d["t_a"] = np.array(d["t"], np.float32)
    return d


def _check_params(ex, y, dt, sinphi, tau, qpt, chi2, ndf):
    for k, tr in enumerate(ex["tracks"]):
        for name, got in (("y", y[k]), ("dt", dt[k]), ("sinphi", sinphi[k]), ("tau", tau[k]), ("qpt", qpt[k])):
            want = tr[name]
            assert abs(float(got) - want) <= 1e-4 * max(abs(want), 1.0), (tr["particle"], name, got, want)
        assert float(chi2[k]) < 1e-3 and int(ndf[k]) == tr["ndf"]


def test_oracle_reproduces_worked_example(ex):
    x = synth.geometry()[0]
    cfg = oracle.Config(row_x=x)
    res = oracle.run_sector(cfg, ex["row_a"], ex["y_a"], ex["t_a"])
    assert res["up"].tolist() == ex["up"] and res["dn"].tolist() == ex["dn"]
    assert res["assign"].tolist() == ex["assign"]
    first, ln, cl = res["first"], res["len"], res["clusters"]
    assert len(first) == len(ex["tracks"])
    for k, tr in enumerate(ex["tracks"]):
        assert cl[first[k]:first[k] + ln[k]].tolist() == tr["clusters"]
    f = res["fit"]
    assert (f["status"] == 0).all()
    last = [tr["clusters"][-1] for tr in ex["tracks"]]
    t_last = ex["t_a"][last].astype(np.float64)
    _check_params(ex, f["y"], f["t"] - t_last, f["sinphi"], f["tau"], f["qpt"], f["chi2"], f["ndf"])


@pytest.mark.gpu
def test_gpu_reproduces_worked_example(ex):
    import torch
    from paper_2102_08862_amd import tpcca
    assert torch.cuda.is_available()
    tpcca.load_library()
    print("case worked example", flush=True)
    trk = tpcca.Tracker(row_x=synth.geometry()[0])
    f = trk.add_frame()
    trk.load_sector(f, 0, ex["row_a"], ex["y_a"], ex["t_a"])
    trk.run(sync=True)
    up, dn = trk.links(f, 0)
    assert up.tolist() == ex["up"] and dn.tolist() == ex["dn"]
    assert trk.assignment(f, 0).tolist() == ex["assign"]
    cl = trk.track_clusters(f, 0)
    tr = trk.tracks(f, 0)
    assert len(tr) == len(ex["tracks"])
    for k, want in enumerate(ex["tracks"]):
        a = int(tr["first"][k])
        assert cl[a:a + int(tr["n_clusters"][k])].tolist() == want["clusters"]
        assert int(tr["seed"][k]) == want["seed"]
    assert (tr["status"] == 0).all()
    _check_params(ex, tr["y"], tr["dt"], tr["sinphi"], tr["tau"], tr["qpt"], tr["chi2"], tr["ndf"])
