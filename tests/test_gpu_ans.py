"""GPU rANS coding of a sector's track clusters against the oracle's coder.

The oracle takes its own tracks (bit-exact with the GPU's), its own symbol
histogram of the sector and its own model, and encodes each track (the row step and the track-model residuals; the
first differences follow from them); the GPU's bytes must equal them byte
for byte, track for track, and decode (with the oracle's decoder) to the
track's symbols."""
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


def test_ans_bytes_of_sectors_against_the_oracle(tp):
    x = synth.geometry()[0]
    oc = oracle_cfg(x)
    fr = synth.generate("frame_10ms", seed=2320, n_threads=16, frame_us=300.0, n_collisions=15)
    print("case ans 0.3 ms frame seed 2320", flush=True)
    trk = tp.Tracker()
    f = trk.load_frame_packed(fr)
    trk.run(sync=True)
    for s in (3, 30):
        row, y, t = fr.sector(s)
        res = oracle.run_sector(oc, row, y, t, fit=False)
        first, ln, cl = res["first"], res["len"], res["clusters"]
        h = oracle.entropy_histograms(first, ln, cl, row, y, t)
        models = [oracle.ans_model(h[k]) for k in range(oracle.ENT_STREAMS)]
        data, off = trk.ans_encode(f, s)
        data = data.cpu().numpy().tobytes()
        assert len(off) == len(first) + 1 and off[0] == 0 and off[-1] == len(data)
        total = 0
        for i, (f0, L) in enumerate(zip(first, ln)):
            c = cl[f0:f0 + L]
            sym = oracle.entropy_symbols(row[c], y[c], t[c])
            want = oracle.ans_encode_track(sym, models)
            got = data[off[i]:off[i + 1]]
            assert got == want, (s, i, len(got), len(want))
            if i % 97 == 0:
                coded = list(oracle.ANS_STREAMS)
                assert np.array_equal(oracle.ans_decode_track(got, len(sym), models)[:, coded], sym[:, coded])
            total += len(want)
        bits = oracle.entropy_bits(h)[list(oracle.ANS_STREAMS)].sum()
        print("sector %d: %d tracks, %d bytes, order-0 bound %.0f bytes" % (s, len(first), total, bits / 8), flush=True)
        assert total <= 1.02 * bits / 8 + 4 * len(first)
