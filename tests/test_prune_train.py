"""Host-side pieces of the pruning pipeline: parameter layout, labels and the
weights file."""
import json

import numpy as np

from paper_2102_08862_amd import prune_train


def test_init_params_layout():
    p = prune_train.init_params(3)
    assert p.dtype == np.float32 and p.size == 5313
    w1 = p[:1024].reshape(64, 16)
    assert np.all(w1[:, 12:] == 0) and np.all(w1[:, :12] != 0)
    assert np.all(p[1024:1088] == 0) and np.all(p[5184:5248] == 0) and p[5312] == 0
    assert abs(w1[:, :12].std() - np.sqrt(2 / 12)) < 0.05
    assert np.array_equal(p, prune_train.init_params(3))


def test_triplet_labels():
    # chain 0 -> 2 -> 5 -> 7 (cleaned links), cluster 3 unassigned with links
    n = 8
    up = np.full(n, -1, np.int32)
    dn = np.full(n, -1, np.int32)
    for a, b in ((0, 2), (2, 5), (5, 7)):
        up[a], dn[b] = b, a
    up[3], dn[3] = 4, 1
    assign = np.full(n, -1, np.int32)
    assign[[0, 2, 5, 7]] = 0
    tri = np.array([[0, 2, 5, 1],     # interior, both links: positive
                    [0, 2, 6, 1],     # wrong up
                    [1, 2, 5, 1],     # wrong down
                    [2, 5, 7, 2],     # interior: positive
                    [1, 3, 4, 1],     # links but not on a track
                    [6, 0, 2, 1],     # chain start has no down link
                    ], np.int32)
    lab = prune_train.triplet_labels(tri, up, dn, assign)
    assert lab.tolist() == [1, 0, 0, 1, 0, 0]


def test_weights_roundtrip(tmp_path):
    p = prune_train.init_params(5)
    path = str(tmp_path / "w.json")
    prune_train.save_weights(p, {"theta": -1.25}, path)
    q, meta = prune_train.load_weights(path)
    assert np.array_equal(p, q) and meta["theta"] == -1.25
    # a damaged file is rejected
    d = json.load(open(path))
    d["params"] = d["params"][:-1]
    json.dump(d, open(path, "w"))
    assert prune_train.load_weights(path) == (None, None)
    assert prune_train.load_weights(str(tmp_path / "missing.json")) == (None, None)
