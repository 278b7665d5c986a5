"""Pins of the token-drop masks and of the zero-fill rule of Sec. 6.2."""
import numpy as np
import pytest

import synth
from oracle import tokenizer as O


def test_splitmix64_published_sequence():
    """SplitMix64 seeded with 0 yields e220a8397b1dcdaf, 6e789e6aa1b965f4,
    06c45d188009454f (the reference generator's first outputs); state k is
    k * 0x9E3779B97F4A7C15."""
    states = np.array([0, O.GOLDEN, (2 * O.GOLDEN) & (2**64 - 1)], dtype=np.uint64)
    out = O.splitmix64(states)
    assert [int(v) for v in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_threshold():
    assert O.drop_threshold(0.0) == 0
    assert O.drop_threshold(1.0) == 2**24
    assert O.drop_threshold(0.25) == 2**22
    assert O.drop_threshold(-1) == 0 and O.drop_threshold(7) == 2**24


@pytest.mark.parametrize("p", [0.05, 0.3, 0.5])
def test_bernoulli_count_within_binomial_band(p):
    keep = O.keep_mask(O.DROP_BERNOULLI, p, 1234, [0, 1, 2], 5, 40, 60)
    n = keep.size
    dropped = n - int(keep.sum())
    assert abs(dropped - n * p) < 4 * np.sqrt(n * p * (1 - p))


def test_extremes_and_batch_invariance():
    assert O.keep_mask(O.DROP_BERNOULLI, 0.0, 1, [0, 1], 3, 8, 8).all()
    assert not O.keep_mask(O.DROP_BERNOULLI, 1.0, 1, [0, 1], 3, 8, 8).any()
    a = O.keep_mask(O.DROP_BERNOULLI, 0.4, 99, [5, 7, 11], 3, 8, 8)
    b = O.keep_mask(O.DROP_BERNOULLI, 0.4, 99, [11], 3, 8, 8)
    np.testing.assert_array_equal(a[2], b[0])
    c = O.keep_mask(O.DROP_BERNOULLI, 0.4, 100, [11], 3, 8, 8)
    assert not np.array_equal(b, c)


def test_rows_mode_and_iframe_protection():
    keep = O.keep_mask(O.DROP_ROWS, 0.5, 3, [0, 1], 3, 16, 16)
    assert np.all((keep.min(axis=-1) == keep.max(axis=-1)))
    assert 0 < keep.mean() < 1
    kp = O.keep_mask(O.DROP_BERNOULLI, 0.9, 3, [0], 3, 16, 16, protect_iframe=True)
    assert kp[:, 0].all() and not kp[:, 1:].all()


def test_apply_keep_zero_fill_bit_exact():
    codes = synth.randn(0, (2, 3, 8, 8, 6), dtype=np.float64)
    keep = O.keep_mask(O.DROP_BERNOULLI, 0.3, 1, [0, 1], 3, 8, 8)
    out = O.apply_keep(codes, keep)
    np.testing.assert_array_equal(out[keep == 1], codes[keep == 1])
    assert np.all(out[keep == 0] == 0.0)


def test_dropped_token_and_lost_packet_look_identical():
    """Sec. 6.2: one packet per token-matrix row carries a W-bit mask and the
    kept tokens; the receiver zero-fills masked tokens and whole lost rows.
    The reassembled tensor equals zero-filling with (mask AND row received)."""
    T2, H2, W2 = 3, 10, 12
    rng = np.random.default_rng(5)
    q = rng.integers(-4, 4, (T2, H2, W2, 6)) / 4.0
    keep = O.keep_mask(O.DROP_BERNOULLI, 0.25, 8, [0], T2, H2, W2)[0]
    received = rng.random(T2 * H2) > 0.3
    rows, masks, payloads = [], [], []
    for r in range(T2 * H2):
        if not received[r]:
            continue
        t, h = divmod(r, H2)
        m = keep[t, h]
        rows.append(r)
        masks.append(m)
        payloads.append(q[t, h][m == 1])
    got = O.reassemble_rows(rows, masks, payloads, T2, H2, W2)
    eff = keep * received.reshape(T2, H2, 1)
    np.testing.assert_array_equal(got, O.apply_keep(q, eff))
