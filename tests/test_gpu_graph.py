"""Graph replay and launch shapes: a run captured once in a HIP graph and
replayed several times (with eager work and synchronisations between the
replays) gives the eager results every time; launch shapes and tile budgets
chosen by the autotuner never change a result."""
import numpy as np
import pytest

from paper_2102_08862_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    from paper_2102_08862_amd import tpcca
    assert torch.cuda.is_available()
    tpcca.load_library()
    return tpcca


def _outputs(trk, f, sectors):
    out = []
    for s in sectors:
        tr = trk.tracks(f, s)
        out.append((trk.assignment(f, s), trk.track_clusters(f, s),
                    {k: tr[k].copy() for k in tr.dtype.names}))
    return out


def _same(a, b):
    for (a1, c1, t1), (a2, c2, t2) in zip(a, b):
        assert np.array_equal(a1, a2) and np.array_equal(c1, c2)
        for k in t1:
            assert np.array_equal(t1[k], t2[k]), k


def test_graph_replays_match_eager(tp):
    import torch
    frs = [synth.generate("slice_1ms", seed=600 + k, n_collisions=6) for k in range(2)]
    sectors = (0, 7, 20, 35)
    eager = tp.Tracker()
    fe = [eager.load_frame_packed(fr) for fr in frs]
    eager.run(sync=True)
    ref = [_outputs(eager, f, sectors) for f in fe]
    g = tp.Tracker()
    g.set_graph(True)
    fg = [g.load_frame_packed(fr) for fr in frs]
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        g.run()
        g.synchronize()
        for f, r in zip(fg, ref):
            _same(_outputs(g, f, sectors), r)
        junk.mul_(1.0001).add_(0.5)  # eager work between replays
        torch.cuda.synchronize()


def test_launch_shapes_do_not_change_results(tp):
    fr = synth.generate("slice_1ms", seed=77, n_collisions=8)
    sectors = (1, 18, 30)
    base = tp.Tracker()
    f = base.load_frame_packed(fr)
    base.run(sync=True)
    ref = _outputs(base, f, sectors)
    # (4, 1, 1) and (4, 2, 500): row-sort buckets take the two-pass path
    for stage, bpc, param in ((5, 1, 256), (5, 2, 1024), (5, 4, 3072), (4, 1, 0), (4, 1, 1), (4, 2, 500), (1, 2, 0),
                              (6, 1, 0), (7, 2, 0), (10, 1, 0), (11, 4, 0), (3, 1, 0), (8, 1, 0)):
        t = tp.Tracker()
        t.set_launch(stage, bpc, param)
        g = t.load_frame_packed(fr)
        t.run(sync=True)
        _same(_outputs(t, g, sectors), ref)


def test_shared_arena_between_trackers(tp):
    """Two contexts with different frames share one arena and one stream,
    each replaying its own graph: after each run the running context's
    outputs equal its results in a private arena."""
    import torch
    frs = [synth.generate("slice_1ms", seed=81, n_collisions=6), synth.generate("slice_1ms", seed=82, n_collisions=9)]
    sectors = (2, 19)
    refs = []
    for fr in frs:
        t = tp.Tracker()
        f = t.load_frame_packed(fr)
        t.run(sync=True)
        refs.append(_outputs(t, f, sectors))
    stream = torch.cuda.Stream()
    trks, fids = [], []
    for fr in frs:
        t = tp.Tracker()
        fids.append(t.load_frame_packed(fr))
        trks.append(t)
    need = max(t.required_arena() for t in trks)
    arena = torch.empty(need + 4096, dtype=torch.uint8, device="cuda")
    for t in trks:
        t.set_stream(stream)
        t.use_arena(arena)
        t.set_graph(True)
    for rep in range(3):
        for k in (0, 1, 0):
            trks[k].run(sync=True)
            _same(_outputs(trks[k], fids[k], sectors), refs[k])
