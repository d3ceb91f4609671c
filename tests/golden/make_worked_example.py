"""Write worked_example.json: a hand-built sector whose tracking result is
known in closed form, for an end-to-end pin of both the oracle and the GPU
library (no tracker code is called here: numpy and the pad-row geometry of
the input generator only).

Two straight particles A and B cross pad rows 0..11, exactly on lines
y = y0 + m (x - x0), t = t0 + n (x - x0) (then rounded to FP32), and a noise
cluster N sits on row 5, 1.2 cm in y beside A. By the pair rule of the
neighbour finder (the middle cluster's offset from the down-up line,
c = ry^2 + rt^2 <= 0.2 cm^2 inside the boxes |dy| <= 1.5 g, |dt| <= 2 g):

* every A (B) cluster on rows 1..10 links down and up to its line
  neighbours (c ~ 0); the noise point is in the boxes of A4 and A6 but every
  pair through it has c ~ (1.2/2)^2 = 0.36 > 0.2; N itself has no pair at
  gap 1 or 2 (c ~ 1.44); rows 0 and 11 have no link (no row below / no
  cluster above);
* cleaning keeps mutual links, so the chains are A1..A10 and B1..B10: two
  tracks of 10 clusters (the minimum), numbered by the input index of their
  first cluster;
* a straight line is a helix of zero curvature: the fit reports at the
  outermost cluster y = its y, dt = 0, sin(phi) = m / sqrt(1 + m^2),
  dt/darc = n / sqrt(1 + m^2), q/pT = 0 and chi2 ~ 0, ndf = 15.

Every expectation is checked here against float64 margins of the rule, so
FP32 rounding of the inputs cannot change it.

  python tests/golden/make_worked_example.py
"""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))
from paper_2102_08862_amd import synth  # noqa: E402  (pad-row geometry only)

WIN_Y, WIN_T, C2 = 1.5, 2.0, 0.2
LINES = {"A": (1.0, 0.02, 100.0, 0.5), "B": (-5.0, -0.01, 300.0, 0.3)}   # y0, m, t0, n
ROWS = list(range(12))
NOISE_DY = 1.2


def main():
    x = synth.geometry()[0].astype(np.float64)
    x0 = x[0]
    cl = []   # (name, row, y, t) in construction order
    for name, (y0, m, t0, n) in LINES.items():
        for r in ROWS:
            cl.append((name + str(r), r, np.float32(y0 + m * (x[r] - x0)), np.float32(t0 + n * (x[r] - x0))))
    ya5 = [c for c in cl if c[0] == "A5"][0]
    cl.append(("N5", 5, np.float32(ya5[2] + NOISE_DY), ya5[3]))
    # a fixed shuffle: the input order is unrelated to rows and particles
    perm = np.random.default_rng(20210217).permutation(len(cl))
    cl = [cl[k] for k in perm]
    idx = {c[0]: k for k, c in enumerate(cl)}
    row = np.array([c[1] for c in cl], np.int64)
    y = np.array([c[2] for c in cl], np.float64)
    t = np.array([c[3] for c in cl], np.float64)

    # float64 margins of the rule for every middle cluster and gap
    def score(i, d, u, g):
        w = (x[row[i]] - x[row[d]]) / (x[row[u]] - x[row[d]])
        ry = (y[i] - y[d]) - w * (y[u] - y[d])
        rt = (t[i] - t[d]) - w * (t[u] - t[d])
        return ry * ry + rt * rt

    def inbox(i, j, g):
        return abs(y[j] - y[i]) <= g * WIN_Y and abs(t[j] - t[i]) <= g * WIN_T

    up = np.full(len(cl), -1, np.int64)
    dn = np.full(len(cl), -1, np.int64)
    for name, k in idx.items():
        r = row[k]
        for g in (1, 2):
            if r - g < 0 or r + g > 151:
                continue
            downs = [j for j in range(len(cl)) if row[j] == r - g and inbox(k, j, g)]
            ups = [j for j in range(len(cl)) if row[j] == r + g and inbox(k, j, g)]
            acc = []
            for d in downs:
                for u in ups:
                    c = score(k, d, u, g)
                    assert c < 0.01 or c > 0.3, (name, g, c)      # far from the cut
                    if c <= C2:
                        acc.append((c, d, u))
            if acc:
                assert len(acc) == 1, (name, acc)
                _, dn[k], up[k] = acc[0]
                break
    for name, k in idx.items():       # the construction, stated directly
        p, r = name[0], int(name[1:])
        if p in "AB" and 1 <= r <= 10:
            assert up[k] == idx[p + str(r + 1)] and dn[k] == idx[p + str(r - 1)], name
        else:
            assert up[k] == -1 and dn[k] == -1, name
    tracks = []
    for p in sorted(LINES, key=lambda q: idx[q + "1"]):
        y0, m, t0, n = LINES[p]
        last = idx[p + "10"]
        norm = math.sqrt(1.0 + m * m)
        tracks.append({"particle": p, "seed": idx[p + "1"],
                       "clusters": [idx[p + str(r)] for r in range(1, 11)],
                       "y": float(y[last]), "dt": 0.0, "sinphi": m / norm, "tau": n / norm, "qpt": 0.0,
                       "ndf": 15})
    assign = [-1] * len(cl)
    for k, tr in enumerate(tracks):
        for c in tr["clusters"]:
            assign[c] = k
    out = {
        "about": "hand-built sector: two straight particles on pad rows 0..11 and a noise cluster; expected "
                 "links, chains, assignment and helix parameters in closed form (see make_worked_example.py)",
        "rule": {"win_y": WIN_Y, "win_t": WIN_T, "pair_c2": C2, "max_gap": 2, "min_track_hits": 10, "bz": 0.5},
        "names": [c[0] for c in cl],
        "row": [int(v) for v in row],
        "y": [float(np.float32(v)) for v in y],
        "t": [float(np.float32(v)) for v in t],
        "up": [int(v) for v in up], "dn": [int(v) for v in dn],
        "tracks": tracks, "assign": assign,
        "param_tol": "|p - expected| <= 1e-4 max(|expected|, 1)",
    }
    with open(os.path.join(HERE, "worked_example.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote worked_example.json: %d clusters, %d tracks" % (len(cl), len(tracks)))


if __name__ == "__main__":
    main()
