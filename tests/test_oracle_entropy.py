"""Pins of the oracle's entropy-reduction symbols (R34): a hand-computed
track, exact straight lines (zero track-model residuals whatever the row
gaps), the residual's relation to the extrapolation miss, and the entropy
of known histograms."""
import numpy as np

import oracle


def test_hand_computed_track():
    row = [3, 4, 6, 7]
    y = [1.0, 1.125, 1.5, 1.6]        # quantised: 16, 18, 24, 25.6 -> 26
    t = [10.0, 10.0625, 10.25, 10.25]  # 160, 161, 164, 164
    s = oracle.entropy_symbols(row, y, t)
    assert s.tolist() == [
        [1, 2, 1, 2, 1],
        # dr 2; residual q2*1 - q1*(1+2) + q0*2
        [2, 6, 3, 24 - 54 + 32, 164 - 483 + 320],
        [1, 2, 0, 26 * 2 - 24 * 3 + 18 * 1, 164 * 2 - 164 * 3 + 161 * 1],
    ]


def test_straight_lines_have_zero_residuals():
    rng = np.random.default_rng(5)
    for _ in range(20):
        n = int(rng.integers(3, 40))
        row = np.cumsum(rng.integers(1, 3, n)) + int(rng.integers(0, 20))
        a, b = rng.integers(-200, 200, 2)
        c, d = rng.integers(0, 5000, 2)
        y = (a + b * row) / 16.0           # exact multiples of 1/16
        t = (c + d * row) / 16.0
        s = oracle.entropy_symbols(row, y, t)
        assert (s[1:, 3] == 0).all() and (s[1:, 4] == 0).all()
        assert (s[:, 0] == np.diff(row)).all()


def test_residual_is_the_extrapolation_miss_times_the_row_step():
    row = np.array([10, 12, 13])
    y = np.array([0.0, 1.0, 3.0])   # q: 0, 16, 48; line through the first two predicts 24 at row 13
    s = oracle.entropy_symbols(row, y, y)
    assert s[1, 3] == (48 - 24) * 2


def test_entropy_of_known_histograms():
    h = np.zeros((2, oracle.ENT_BINS), np.int64)
    h[0, 10] = h[0, 11] = h[0, 12] = h[0, 13] = 5     # uniform over 4 symbols: 2 bits each
    h[1, 0] = 8                                       # one symbol: 0 bits
    h[1, -1] = 0
    e = oracle.entropy_bits(h)
    assert abs(e[0] - 40.0) < 1e-9 and e[1] == 0.0
    h[1, -1] = 8                                      # half escapes: 1 bit each plus 32
    assert abs(oracle.entropy_bits(h)[1] - (16.0 + 8 * 32.0)) < 1e-9


def _models(h):
    return [oracle.ans_model(h[k]) for k in range(oracle.ENT_STREAMS)]


def test_ans_model_sums_and_covers():
    rng = np.random.default_rng(3)
    for _ in range(20):
        h = np.zeros(oracle.ENT_BINS, np.int64)
        nz = rng.choice(oracle.ENT_BINS, int(rng.integers(1, 400)), replace=False)
        h[nz] = rng.integers(1, 10 ** int(rng.integers(1, 7)), len(nz))
        f, c = oracle.ans_model(h)
        assert f.sum() == 1 << oracle.ANS_BITS and (f[h > 0] >= 1).all() and f[-1] >= 1
        assert (f[(h == 0) & (np.arange(len(h)) < len(h) - 1)] == 0).all()
        assert c[0] == 0 and (np.diff(c) == f[:-1]).all()


def test_ans_round_trip_and_size():
    """Random tracks (escapes included) decode to their symbols, and the
    bytes stay within a few percent of the order-0 entropy."""
    rng = np.random.default_rng(4)
    syms = []
    for _ in range(60):
        n = int(rng.integers(1, 60))
        s = np.stack([rng.integers(1, 3, n), rng.normal(0, 6, n).round(), rng.normal(0, 3, n).round(),
                      rng.normal(0, 20, n).round(), rng.integers(-400, 400, n)], axis=1).astype(np.int64)
        s[rng.random(s.shape) < 0.01] = 70000
        syms.append(s)
    h = np.zeros((oracle.ENT_STREAMS, oracle.ENT_BINS), np.int64)
    for s in syms:
        b = np.where(np.abs(s) <= oracle.ENT_H, s + oracle.ENT_H, oracle.ENT_BINS - 1)
        for k in range(oracle.ENT_STREAMS):
            h[k] += np.bincount(b[:, k], minlength=oracle.ENT_BINS)
    models = _models(h)
    total = 0
    for s in syms:
        data = oracle.ans_encode_track(s, models)
        coded = list(oracle.ANS_STREAMS)
        assert np.array_equal(oracle.ans_decode_track(data, len(s), models)[:, coded], s[:, coded])
        total += len(data)
    bound = oracle.entropy_bits(h)[list(oracle.ANS_STREAMS)].sum() / 8.0
    assert bound <= total <= 1.05 * bound + 4 * len(syms)
