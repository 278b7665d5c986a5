"""Pins of the oracle's finite scalar quantiser: exhaustive code coverage,
index bijection, idempotence, monotonicity, boundary preimages, saturation."""
import itertools

import numpy as np

from oracle import tokenizer as O

LEVELS = O.FSQ_LEVELS


def _preimage(q):
    """z whose bounded value is q - 0.1 sign(q) (inside the open range
    (-h - o, h - o) even for the extreme codes, and rounding to q):
    z = atanh((q - 0.1 sign q + o)/h) - s."""
    h, o, s, _ = O.fsq_constants()
    return np.arctanh((q - 0.1 * np.sign(q) + o) / h) - s


def test_constants():
    h, o, s, d = O.fsq_constants()
    np.testing.assert_allclose(h, [3.4965] * 3 + [1.998] * 3, rtol=1e-15)
    np.testing.assert_allclose(s[:3], 0.1439870, atol=1e-7)
    np.testing.assert_array_equal(s[3:], 0.0)
    np.testing.assert_array_equal(d, [4, 4, 4, 2, 2, 2])
    np.testing.assert_array_equal(O.fsq_basis(), [1, 8, 64, 512, 2560, 12800])


def test_every_code_reached_and_index_is_bijective():
    """All prod(L) = 64000 integer code vectors: their preimages quantise back
    to themselves, their indices are 0..63999 each exactly once, and
    index -> codes inverts."""
    ranges = [np.arange(-(L // 2), L - L // 2) for L in LEVELS]
    qs = np.array(list(itertools.product(*ranges)), np.float64)
    assert qs.shape == (64000, 6)
    codes, idx, q, b = O.fsq(_preimage(qs))
    np.testing.assert_array_equal(q, qs)
    assert sorted(idx.tolist()) == list(range(64000))
    np.testing.assert_array_equal(O.fsq_indices_to_codes(idx), codes)
    np.testing.assert_array_equal(codes * np.array([4, 4, 4, 2, 2, 2]), qs)


def test_level_sets_and_idempotence():
    z = np.random.default_rng(0).normal(0, 3, (100000, 6))
    codes, idx, q, b = O.fsq(z)
    for c, L in enumerate(LEVELS):
        assert set(np.unique(q[:, c]).tolist()) <= set(range(-(L // 2), L - L // 2))
    assert idx.min() >= 0 and idx.max() < 64000
    # quantising the grid point again changes nothing
    assert np.array_equal(np.rint(q), q)
    codes2, idx2, q2, _ = O.fsq(_preimage(q))
    np.testing.assert_array_equal(idx2, idx)


def test_monotone_zero_and_saturation():
    z = np.linspace(-30, 30, 200001)[:, None] * np.ones((1, 6))
    b = O.fsq_bound(z)
    assert np.all(np.diff(b, axis=0) >= 0)
    np.testing.assert_allclose(O.fsq_bound(np.zeros((1, 6))), 0.0, atol=1e-15)
    codes, idx, q, _ = O.fsq(np.zeros((1, 6)))
    np.testing.assert_array_equal(q, 0.0)
    _, _, qlo, _ = O.fsq(np.full((1, 6), -1e3))
    _, _, qhi, _ = O.fsq(np.full((1, 6), 1e3))
    np.testing.assert_array_equal(qlo[0], [-4, -4, -4, -2, -2, -2])
    np.testing.assert_array_equal(qhi[0], [3, 3, 3, 2, 2, 2])


def test_boundary_preimages_split_adjacent_codes():
    h, o, s, _ = O.fsq_constants()
    for c, L in enumerate(LEVELS):
        lo = -(L // 2)
        hi = L - L // 2 - 1
        for k in range(lo, hi):
            zstar = np.arctanh((k + 0.5 + o[c]) / h[c]) - s[c]
            z = np.zeros((2, 6))
            z[0, c] = zstar - 1e-6
            z[1, c] = zstar + 1e-6
            _, _, q, b = O.fsq(z)
            assert q[0, c] == k and q[1, c] == k + 1
            assert np.all(O.fsq_boundary_distance(b[:, c]) < 1e-5)


def test_round_half_to_even():
    assert np.rint(0.5) == 0.0 and np.rint(1.5) == 2.0 and np.rint(-0.5) == 0.0
