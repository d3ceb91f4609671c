"""The entry point for callers that cannot allocate (tpcca_run_noalloc, the
run in the library's static device arena) against tpcca_run with a
caller-owned arena: two calls in a row on one context, the second with a
smaller input, each bit-identical to an arena run of the same input; a run
that needs more than the static arena is refused with CAPACITY; and the
context goes back to its own arena with tpcca_run."""
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
        up, dn = trk.links(f, s, cleaned=False)
        tr = trk.tracks(f, s)
        out.append((up, dn, trk.assignment(f, s), trk.track_clusters(f, s),
                    {k: tr[k].copy() for k in tr.dtype.names}))
    return out


def _same(a, b):
    for x, y in zip(a, b):
        for u, v in zip(x[:4], y[:4]):
            assert np.array_equal(u, v)
        for k in x[4]:
            assert np.array_equal(x[4][k], y[4][k]), k


def _load(trk, parts):
    f = trk.add_frame()
    for s, (row, y, t) in parts.items():
        trk.load_sector(f, s, row, y, t)
    return f


def test_noalloc_runs_match_arena_runs(tp):
    fr = synth.generate("sector_300", seed=11)
    row, y, t = fr.sector(0)
    fr2 = synth.generate("sector_300", seed=12)
    r2, y2, t2 = fr2.sector(0)
    m = (len(r2) * 3) // 5
    inputs = [{0: (row, y, t), 5: (r2, y2, t2)},          # first call: two sectors
              {3: (r2[:m], y2[:m], t2[:m])}]              # second call: a smaller input
    na = tp.Tracker()
    for parts in inputs:
        ref = tp.Tracker()
        fa = _load(ref, parts)
        ref.run(sync=True)
        want = _outputs(ref, fa, sorted(parts))
        na.clear_frames()
        fn = _load(na, parts)
        na.required_arena()   # sizes the table block (may allocate); the run itself does not
        na.run_noalloc(sync=True)
        assert na.stats()["n_clusters"] == sum(len(p[0]) for p in parts.values())
        _same(_outputs(na, fn, sorted(parts)), want)
        del ref
    # back to a caller-owned arena on the same context
    na.run(sync=True)
    _same(_outputs(na, fn, sorted(inputs[1])), want)


def test_noalloc_refuses_runs_beyond_the_static_arena(tp):
    fr = synth.generate("slice_1ms", seed=2301, n_threads=8)
    trk = tp.Tracker()
    f = trk.load_frame_packed(fr)
    need = trk.required_arena()
    assert need > (160 << 20)
    with pytest.raises(tp.TpccaError) as e:
        trk.run_noalloc(sync=True)
    assert e.value.status == tp.ERR_CAPACITY
