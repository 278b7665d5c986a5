"""Pins of the oracle's similarity-based token selection (Sec. 4.3, Eq. 3):
brute force with float64 cosines, exact ties between different integer
vectors, zero norms, the drop count, the I frame, and degenerate rates."""
import math

import numpy as np
import pytest

import synth
from oracle import tokenizer as O

LEVELS = np.array([8, 8, 8, 5, 5, 5])
HALF = LEVELS // 2


def random_codes(seed, N, T2, H2, W2):
    rng = np.random.default_rng(seed)
    q = np.floor(rng.uniform(size=(N, T2, H2, W2, 6)) * LEVELS).astype(np.int64) - HALF
    return q / HALF


def cosine(a, b):
    na, nb = np.linalg.norm(a), np.linalg.norm(b)
    return 0.0 if na == 0 or nb == 0 else float(np.dot(a, b) / (na * nb))


@pytest.mark.parametrize("seed,rate", [(0, 0.3), (1, 0.5), (2, 0.07), (3, 0.999)])
def test_drops_the_most_similar_p_tokens(seed, rate):
    codes = random_codes(seed, 2, 4, 3, 5)
    keep = O.similarity_keep(codes, rate)
    N, T2, H2, W2, _ = codes.shape
    n_p = (T2 - 1) * H2 * W2
    assert (keep[:, 0] == 1).all()  # the I frame is never dropped
    for n in range(N):
        s = np.array([[[cosine(codes[n, t, h, w], codes[n, 0, h, w]) for w in range(W2)] for h in range(H2)]
                      for t in range(1, T2)])
        k = keep[n, 1:]
        assert int((k == 0).sum()) == math.ceil(np.float32(rate) * n_p)
        if (k == 0).any() and (k == 1).any():
            assert s[k == 0].min() >= s[k == 1].max() - 1e-12  # everything dropped is at least as similar


def test_exact_ties_go_to_the_lower_index():
    # cos(x, y) = 1/sqrt(2) from two different integer pairs: (1,0,..) vs (1,1,..) and (2,2,..) vs (1,0,..)
    codes = np.zeros((1, 3, 1, 2, 6))
    codes[0, 0, 0, 0, :2] = [0.25, 0.25]    # I at w=0: 4c = (1, 1)
    codes[0, 0, 0, 1, :2] = [0.25, 0.0]     # I at w=1: 4c = (1, 0)
    codes[0, 1, 0, 0, :2] = [0.25, 0.0]     # P t=1 w=0: (1,0) vs (1,1): 1/sqrt2
    codes[0, 1, 0, 1, :2] = [0.5, 0.5]      # P t=1 w=1: (2,2) vs (1,0): 1/sqrt2
    codes[0, 2, 0, 0, :2] = [0.25, 0.25]    # P t=2 w=0: identical to I: S = 1
    codes[0, 2, 0, 1, :2] = [-0.25, 0.0]    # P t=2 w=1: S = -1
    assert O.similarity_order_key(np.array([1, 0, 0, 0, 0, 0]), np.array([1, 1, 0, 0, 0, 0])) == \
        O.similarity_order_key(np.array([2, 2, 0, 0, 0, 0]), np.array([1, 0, 0, 0, 0, 0]))
    keep = O.similarity_keep(codes, 0.5)    # 2 of 4: S = 1 first, then the lower-index 1/sqrt2 token
    assert keep[0, 2, 0, 0] == 0 and keep[0, 1, 0, 0] == 0
    assert keep[0, 1, 0, 1] == 1 and keep[0, 2, 0, 1] == 1
    keep = O.similarity_keep(codes, 0.75)
    assert keep[0, 1, 0, 1] == 0 and keep[0, 2, 0, 1] == 1


def test_zero_norm_tokens_score_zero():
    codes = np.zeros((1, 2, 1, 3, 6))
    codes[0, 0, 0, :, 0] = 0.5
    codes[0, 1, 0, 0, 0] = 0.25     # S = 1
    codes[0, 1, 0, 2, 0] = -0.25    # S = -1; token 1 is all zero: S = 0
    keep = O.similarity_keep(codes, 0.6)   # 2 of 3 dropped: S = 1, then S = 0
    assert keep[0, 1].tolist() == [[0, 0, 1]]


def test_degenerate_rates_and_single_latent_frame():
    codes = random_codes(9, 1, 3, 2, 2)
    assert (O.similarity_keep(codes, 0.0) == 1).all()
    k = O.similarity_keep(codes, 1.0)
    assert (k[:, 0] == 1).all() and (k[:, 1:] == 0).all()
    assert (O.similarity_keep(random_codes(9, 2, 1, 2, 2), 0.9) == 1).all()  # no P frames


def test_clips_are_selected_independently():
    codes = random_codes(4, 3, 3, 2, 3)
    both = O.similarity_keep(codes, 0.4)
    for n in range(3):
        np.testing.assert_array_equal(both[n], O.similarity_keep(codes[n:n + 1], 0.4)[0])
