"""GPU parity: the HIP library against the CPU oracle, element by element.

Links, cleaned links, assignment, track identities and cluster lists must be
bit-exact; track parameters agree within 1e-4 relative (floors in
tests/_parity.py). Inputs are seeded synthetic frames; sizes span many
tiles, chunks and a ragged tail, plus the degenerate cases."""
import numpy as np
import pytest

import oracle
from paper_2102_08862_amd import synth

from _parity import compare_sector, oracle_cfg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    from paper_2102_08862_amd import tpcca
    assert torch.cuda.is_available()
    tpcca.load_library()
    return tpcca


@pytest.fixture(scope="module")
def x():
    return synth.geometry()[0]


def _one_sector(tp, row, y, t, device=True, **cfg):
    trk = tp.Tracker(**cfg)
    f = trk.add_frame()
    trk.load_sector(f, 0, row, y, t, device=device)
    trk.run(sync=True)
    return trk, f


@pytest.mark.parametrize("seed,device", [(1, False), (1, True), (2, True), (7, False)])
def test_single_sector(tp, x, seed, device):
    fr = synth.generate("sector_300", seed=seed)
    row, y, t = fr.sector(0)
    print("case sector_300 seed", seed, "device", device, flush=True)
    trk, f = _one_sector(tp, row, y, t, device=device)
    res = compare_sector(trk, f, 0, row, y, t, oracle_cfg(x))
    print(res)
    assert res["tracks"] > 50
    # the other sectors of the frame were never loaded: empty results
    assert len(trk.tracks(f, 5)) == 0


def test_slice_1ms_sectors(tp, x):
    fr = synth.generate("slice_1ms", seed=2300)
    print("case slice_1ms seed 2300: %d clusters" % fr.n_clusters, flush=True)
    trk = tp.Tracker()
    f = trk.load_frame_packed(fr)
    trk.run(sync=True)
    st = trk.stats()
    assert st["n_clusters"] == fr.n_clusters and st["n_invalid"] == 0
    oc = oracle_cfg(x)
    tot = 0
    for s in (0, 13, 18, 35):
        row, y, t = fr.sector(s)
        res = compare_sector(trk, f, s, row, y, t, oc)
        print(s, res, flush=True)
        tot += res["tracks"]
    assert tot > 1000


def test_tiny_inputs_with_ties_and_duplicates(tp, x):
    """Coarsely quantised values: many exact ties of the pair score and
    duplicated clusters; the tie-break must follow the input indices."""
    rng = np.random.default_rng(3)
    for case in range(4):
        n = [50, 333, 1000, 2500][case]
        row = rng.integers(0, 12, n).astype(np.uint8)
        y = (np.round(rng.uniform(-2, 2, n) * 4) / 4).astype(np.float32)
        t = (np.round(rng.uniform(-2, 2, n) * 4) / 4).astype(np.float32)
        k = n // 5
        src, dst = rng.integers(0, n, k), rng.integers(0, n, k)
        row[dst], y[dst], t[dst] = row[src], y[src], t[src]
        print("case ties", case, n, flush=True)
        trk, f = _one_sector(tp, row, y, t, min_track_hits=3)
        compare_sector(trk, f, 0, row, y, t, oracle_cfg(x, min_track_hits=3), check_params=False)


def test_degenerate_sectors(tp, x):
    oc = oracle_cfg(x)
    cases = {
        "one": (np.array([40], np.uint8), np.zeros(1, np.float32), np.zeros(1, np.float32)),
        "one_row": (np.full(500, 77, np.uint8), np.linspace(-5, 5, 500).astype(np.float32),
                    np.linspace(0, 100, 500).astype(np.float32)),
        "edge_rows": (np.array([0, 1, 2, 149, 150, 151], np.uint8), np.zeros(6, np.float32), np.zeros(6, np.float32)),
        "same_point": (np.repeat(np.arange(152, dtype=np.uint8), 3), np.zeros(456, np.float32),
                       np.full(456, 3.0, np.float32)),
    }
    for name, (row, y, t) in cases.items():
        print("case", name, flush=True)
        trk, f = _one_sector(tp, row, y, t)
        compare_sector(trk, f, 0, row, y, t, oc)


def test_wide_time_range(tp, x):
    """Tracks near t = 0, a line at t = 1e6 and noise from t = -500 to
    3e7: coarse bins wider than a row-sort time slab, so every row is sorted
    as one bucket; and a range with negative times and the clamped slabs."""
    fr = synth.generate("sector_300", seed=4)
    r0, y0, t0 = fr.sector(0)
    rng = np.random.default_rng(13)
    rl = np.arange(10, 40, dtype=np.uint8)
    yl = (0.25 * (x[rl] - x[10])).astype(np.float32)
    tl = (1.0e6 + 0.5 * (x[rl] - x[10])).astype(np.float32)
    n = 600
    rn = rng.integers(0, 152, n).astype(np.uint8)
    yn = rng.uniform(-30, 30, n).astype(np.float32)
    tn = rng.uniform(-500, 3.0e7, n).astype(np.float32)
    oc = oracle_cfg(x)
    for name, parts in (("wide", ((r0, y0, t0), (rl, yl, tl), (rn, yn, tn))),
                        ("negative", ((r0, y0, (t0 - 3000.0).astype(np.float32)), (rn[:50], yn[:50], tn[:50] * 0 - 400.0)))):
        row = np.concatenate([p[0] for p in parts]).astype(np.uint8)
        y = np.concatenate([p[1] for p in parts]).astype(np.float32)
        t = np.concatenate([p[2] for p in parts]).astype(np.float32)
        print("case", name, len(row), flush=True)
        trk, f = _one_sector(tp, row, y, t)
        res = compare_sector(trk, f, 0, row, y, t, oc)
        print(res, flush=True)


def test_dense_rows_overflow_lds(tp, x):
    """A hot spot with far more clusters per coarse bin than a neighbour tile
    can stage in LDS: those tiles are searched in global memory with the
    same predicates."""
    rng = np.random.default_rng(11)
    n = 12000
    row = rng.integers(20, 26, n).astype(np.uint8)
    y = (np.round(rng.uniform(-20, 20, n) * 64) / 64).astype(np.float32)
    t = (np.round(rng.uniform(0, 40, n) * 64) / 64).astype(np.float32)
    fr = synth.generate("sector_300", seed=3)
    r0, y0, t0 = fr.sector(0)
    row = np.concatenate([row, r0]); y = np.concatenate([y, y0]); t = np.concatenate([t, t0])
    print("case dense", len(row), flush=True)
    trk, f = _one_sector(tp, row, y, t, min_track_hits=3)
    assert trk.stats()["n_overflow_tiles"] > 0
    compare_sector(trk, f, 0, row, y, t, oracle_cfg(x, min_track_hits=3), check_params=False)


def test_empty_frame_and_ragged_sizes(tp, x):
    """Several frames in one run: empty sectors, a single cluster, and sizes
    around the work-chunk boundary; each sector equals its own oracle."""
    oc = oracle_cfg(x)
    fr = synth.generate("sector_300", seed=5, fixed_mult=600)
    row, y, t = fr.sector(0)
    trk = tp.Tracker()
    f0 = trk.add_frame()          # stays empty
    f1 = trk.add_frame()
    sizes = {0: 1, 1: 8191, 2: 8192, 3: 8193, 4: len(row)}
    for s, n in sizes.items():
        n = min(n, len(row))
        trk.load_sector(f1, s, row[:n], y[:n], t[:n])
    trk.run(sync=True)
    assert len(trk.tracks(f0, 0)) == 0
    for s, n in sizes.items():
        n = min(n, len(row))
        print("case ragged", s, n, flush=True)
        compare_sector(trk, f1, s, row[:n], y[:n], t[:n], oc)


def test_batched_frames_equal_single_runs(tp, x):
    frs = [synth.generate("slice_1ms", seed=100 + k, n_collisions=4 + 3 * k) for k in range(3)]
    trk = tp.Tracker()
    ids = [trk.load_frame_packed(fr) for fr in frs]
    trk.run(sync=True)
    for fr, f in zip(frs, ids):
        one = tp.Tracker()
        g = one.load_frame_packed(fr)
        one.run(sync=True)
        for s in (0, 9, 27):
            a = trk.tracks(f, s)
            b = one.tracks(g, s)
            b["frame"] = f
            for k in a.dtype.names:
                assert np.array_equal(a[k], b[k]), k
            assert np.array_equal(trk.assignment(f, s), one.assignment(g, s))


def test_deterministic_and_time_shift_invariant(tp, x):
    fr = synth.generate("slice_1ms", seed=41, n_collisions=10)
    trk = tp.Tracker()
    f = trk.load_frame_packed(fr)
    trk.run(sync=True)
    a = [trk.tracks(f, s) for s in range(36)]
    trk.run(sync=True)
    b = [trk.tracks(f, s) for s in range(36)]
    for u, v in zip(a, b):
        for k in u.dtype.names:
            assert np.array_equal(u[k], v[k]), k
    # shift every time by a multiple of 2^-9 that keeps the values exact
    sh = synth.generate("slice_1ms", seed=41, n_collisions=10)
    for s in range(36):
        sh.ts[s] = sh.ts[s] + np.float32(1536.0)
    trk2 = tp.Tracker()
    g = trk2.load_frame_packed(sh)
    trk2.run(sync=True)
    for s in range(36):
        ta, tb = trk.tracks(f, s), trk2.tracks(g, s)
        assert np.array_equal(trk.assignment(f, s), trk2.assignment(g, s))
        for k in ("y", "dt", "sinphi", "tau", "qpt", "chi2", "status", "n_clusters", "seed"):
            assert np.array_equal(ta[k], tb[k]), k


def test_abort_then_rerun(tp, x):
    fr = synth.generate("sector_300", seed=8)
    row, y, t = fr.sector(0)
    trk = tp.Tracker()
    f = trk.add_frame()
    trk.load_sector(f, 0, row, y, t)
    trk.request_abort()
    trk.run()
    with pytest.raises(tp.TpccaError) as e:
        trk.synchronize()
    assert e.value.status == tp.ERR_ABORTED
    trk.run(sync=True)
    compare_sector(trk, f, 0, row, y, t, oracle_cfg(x))


def test_invalid_inputs(tp, x):
    trk = tp.Tracker()
    f = trk.add_frame()
    bad_row = np.array([3, 152], np.uint8)
    with pytest.raises(tp.TpccaError) as e:
        trk.load_sector(f, 0, bad_row, np.zeros(2, np.float32), np.zeros(2, np.float32), device=False)
    assert e.value.status == tp.ERR_INVALID_ARG
    with pytest.raises(tp.TpccaError):
        trk.load_sector(f, 1, np.array([3], np.uint8), np.array([np.nan], np.float32), np.zeros(1, np.float32),
                        device=False)
    with pytest.raises(tp.TpccaError):
        trk.load_sector(f, 99, np.array([3], np.uint8), np.zeros(1, np.float32), np.zeros(1, np.float32))
    trk.load_sector(f, 2, np.array([3], np.uint8), np.zeros(1, np.float32), np.zeros(1, np.float32))
    with pytest.raises(tp.TpccaError) as e:
        trk.load_sector(f, 2, np.array([3], np.uint8), np.zeros(1, np.float32), np.zeros(1, np.float32))
    assert e.value.status == tp.ERR_STATE
    # device inputs are checked on the device: invalid clusters are left out
    fr = synth.generate("sector_300", seed=12)
    row, y, t = fr.sector(0)
    row = row.copy(); y = y.copy()
    bad = np.arange(0, len(row), 97)
    row[bad[::2]] = 200
    y[bad[1::2]] = np.inf
    trk2 = tp.Tracker()
    g = trk2.add_frame()
    trk2.load_sector(g, 0, row, y, t, device=True)
    trk2.run(sync=True)
    assert trk2.stats()["n_invalid"] == len(bad)
    keep = np.setdiff1d(np.arange(len(row)), bad)
    ref = oracle.run_sector(oracle_cfg(x), row[keep], y[keep], t[keep])
    assign = trk2.assignment(g, 0)
    assert (assign[bad] == -1).all()
    assert np.array_equal(assign[keep], ref["assign"])
    cl = trk2.track_clusters(g, 0)
    assert np.array_equal(cl, keep[ref["clusters"]])


def test_arena_too_small_and_state_errors(tp, x):
    trk = tp.Tracker()
    with pytest.raises(tp.TpccaError) as e:
        trk.lib and trk._check(trk.lib.tpcca_run(trk.h))
    assert e.value.status == tp.ERR_STATE
    f = trk.add_frame()
    trk.load_sector(f, 0, np.array([5, 6, 7], np.uint8), np.zeros(3, np.float32), np.zeros(3, np.float32))
    import ctypes
    import torch
    need = trk.required_arena()
    small = torch.empty(need // 2, dtype=torch.uint8, device="cuda")
    trk._check(trk.lib.tpcca_attach_arena(trk.h, ctypes.c_void_p(small.data_ptr()), need // 2))
    with pytest.raises(tp.TpccaError) as e:
        trk._check(trk.lib.tpcca_run(trk.h))
    assert e.value.status == tp.ERR_NOMEM


def test_more_chains_than_walk_rows(tp, x):
    """Many short tracks: more seeds than the chain walk keeps records for
    (n_clusters / 32 + 64 rows), so some tracks take the walk-again path of
    the output stage; every output still equals the oracle's."""
    rng = np.random.default_rng(41)
    rows, ys, ts = [], [], []
    for k in range(700):
        r0 = int(rng.integers(0, 140))
        rr = np.arange(r0, r0 + 12)
        y0, m = rng.uniform(-12, 12), rng.uniform(-0.1, 0.1)
        t0, n = 30.0 * k, rng.uniform(-0.5, 0.5)
        xx = x[rr].astype(np.float64)
        rows.append(rr)
        ys.append(y0 + m * (xx - xx[0]) + rng.normal(0, 0.02, len(rr)))
        ts.append(t0 + n * (xx - xx[0]) + rng.normal(0, 0.02, len(rr)))
    row = np.concatenate(rows).astype(np.uint8)
    y = np.concatenate(ys).astype(np.float32)
    t = np.concatenate(ts).astype(np.float32)
    perm = rng.permutation(len(row))
    row, y, t = row[perm], y[perm], t[perm]
    print("case short tracks", len(row), flush=True)
    trk, f = _one_sector(tp, row, y, t)
    st = trk.stats()
    assert st["n_seeds"] > len(row) // 32 + 64, st["n_seeds"]
    res = compare_sector(trk, f, 0, row, y, t, oracle_cfg(x))
    print(res, "seeds", st["n_seeds"])
    assert res["tracks"] > 500
