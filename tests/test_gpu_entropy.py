"""GPU symbol histograms of the entropy reduction against the oracle's.

The symbols are integers computed from the quantised inputs along each
track's cluster list; the lists are bit-exact between the GPU and the
oracle (the sector parity tests), and the quantisation is the same FP32
product rounded to nearest even on both. So the histograms must be equal,
bin for bin: per sector (four sectors of the 1 ms slice, with and without
track following) and for the whole run as the sum of its sectors."""
import numpy as np
import pytest

import oracle
from paper_2102_08862_amd import synth

from _parity import oracle_cfg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    from paper_2102_08862_amd import tpcca
    assert torch.cuda.is_available()
    tpcca.load_library()
    return tpcca


@pytest.mark.parametrize("follow", [0, 1])
def test_histograms_of_a_slice_against_the_oracle(tp, follow):
    x = synth.geometry()[0]
    oc = oracle_cfg(x)
    fr = synth.generate("slice_1ms", seed=2300, n_threads=16)
    print("case entropy slice_1ms seed 2300 follow %d" % follow, flush=True)
    trk = tp.Tracker(follow=follow) if follow else tp.Tracker()
    f = trk.load_frame_packed(fr)
    trk.run(sync=True)
    total = trk.entropy_histograms()
    per = np.zeros_like(total)
    for s in range(36):
        per += trk.entropy_histograms(f, s)
    assert np.array_equal(per, total)
    for s in (0, 9, 22, 35):
        row, y, t = fr.sector(s)
        if follow:
            res = oracle.run_sector(oc, row, y, t, fit=False, follow_cfg=oracle.FollowConfig())
        else:
            res = oracle.run_sector(oc, row, y, t, fit=False)
        want = oracle.entropy_histograms(res["first"], res["len"], res["clusters"], row, y, t)
        got = trk.entropy_histograms(f, s)
        assert np.array_equal(got, want), (s, np.nonzero(got != want))
        bits = oracle.entropy_bits(want) / max(want[0].sum(), 1)
        print("sector %d: %d symbols; bits per cluster: first differences %.2f, track model %.2f" % (
            s, int(want[0].sum()), bits[0] + bits[1] + bits[2], bits[0] + bits[3] + bits[4]), flush=True)
