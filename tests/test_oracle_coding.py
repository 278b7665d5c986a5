"""Pins of the oracle's coding steps: row packets and reassembly (Sec. 6.2),
the pixel-residual layer (Sec. 4.3, Eq. 4) and GoP-boundary blending
(Sec. 4.2, Eq. 2).  Expected values come from the paper's definitions worked
by hand, closed forms and identities, not from re-running the oracle's code."""
import numpy as np
import pytest

from oracle import coding as K
from oracle import tokenizer as O


def rand_idx_keep(seed, N, T2, H2, W2, p_keep=0.7):
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, 64000, (N, T2, H2, W2))
    keep = (rng.random((N, T2, H2, W2)) < p_keep).astype(np.uint8)
    return idx, keep


# ---- packets ---------------------------------------------------------------

def test_packet_bytes_by_hand():
    """One row of W2 = 10 with mask 1,0,1,1,0,0,0,0,0,1 carrying indices 7,
    300, 63999 (the largest code) and 1: header 4 bytes, mask 2 bytes padded
    to 4, payload 4 u16 = 8 bytes."""
    idx = np.array([[[[7, 5, 300, 63999, 9, 9, 9, 9, 9, 1]]]])
    keep = np.array([[[[1, 0, 1, 1, 0, 0, 0, 0, 0, 1]]]], np.uint8)
    buf, offs = K.serialize(K.packetize(idx, keep), 10)
    expect = bytes([0, 0, 0, 0,                  # row 0
                    0b00001101, 0b00000010, 0, 0,  # columns 0, 2, 3 | column 9
                    7, 0, 44, 1, 0xFF, 0xF9, 1, 0])  # 7, 300 = 0x012C, 63999 = 0xF9FF, 1
    assert buf == expect
    assert offs == [0, 16]


def test_odd_count_pads_and_rows_are_numbered_across_the_batch():
    idx, keep = rand_idx_keep(1, 2, 3, 4, 9)
    keep[1, 2, 3] = [1, 0, 0, 0, 0, 0, 0, 0, 0]   # last row of the batch: one token
    pk = K.packetize(idx, keep)
    assert [g for g, _, _ in pk] == list(range(2 * 3 * 4))
    buf, offs = K.serialize(pk, 9)
    assert len(offs) == 25 and offs[-1] == len(buf)
    last = buf[offs[-2]:]
    assert len(last) == 4 + 4 + 4 and last[:4] == (23).to_bytes(4, "little")
    assert last[-2:] == b"\x00\x00"                 # the pad of an odd payload
    for k, (g, m, pay) in enumerate(pk):
        assert offs[k + 1] - offs[k] == 4 + 4 * (((9 + 7) // 8 + 3) // 4) + 4 * ((sum(m) + 1) // 2)


@pytest.mark.parametrize("seed,N,T2,H2,W2", [(0, 1, 3, 5, 7), (1, 2, 2, 4, 16), (2, 1, 4, 3, 33)])
def test_every_row_received_gives_zero_filled_codes(seed, N, T2, H2, W2):
    idx, keep = rand_idx_keep(seed, N, T2, H2, W2)
    buf, offs = K.serialize(K.packetize(idx, keep), W2)
    codes, k2 = K.reassemble(buf, offs[:-1], N, T2, H2, W2)
    np.testing.assert_array_equal(k2, keep)
    np.testing.assert_array_equal(codes, O.apply_keep(O.fsq_indices_to_codes(idx), keep))


def test_lost_packet_equals_dropped_row_and_order_does_not_matter():
    """Sec. 6.2: a lost row and a row whose tokens were all dropped reach the
    decoder identically."""
    N, T2, H2, W2 = 2, 3, 6, 11
    idx, keep = rand_idx_keep(4, N, T2, H2, W2)
    buf, offs = K.serialize(K.packetize(idx, keep), W2)
    rng = np.random.default_rng(9)
    lost = rng.random(N * T2 * H2) < 0.3
    recv = [offs[g] for g in range(N * T2 * H2) if not lost[g]]
    rng.shuffle(recv)
    codes, k2 = K.reassemble(buf, recv, N, T2, H2, W2)
    eff = keep * (~lost).reshape(N, T2, H2, 1)
    np.testing.assert_array_equal(k2, eff)
    np.testing.assert_array_equal(codes, O.apply_keep(O.fsq_indices_to_codes(idx), eff))


def test_malformed_packets_are_ignored():
    N, T2, H2, W2 = 1, 2, 2, 8
    idx, keep = rand_idx_keep(5, N, T2, H2, W2, p_keep=1.0)
    buf, offs = K.serialize(K.packetize(idx, keep), W2)
    bad = bytearray(buf)
    bad[offs[1]:offs[1] + 4] = (99).to_bytes(4, "little")    # row out of range
    codes, k2 = K.reassemble(bytes(bad), [offs[1], len(buf) - 2, offs[3]], N, T2, H2, W2)
    assert k2.sum() == W2 and (k2[0, 1, 1] == 1).all()        # only the last row arrived intact


# ---- pixel residuals ---------------------------------------------------------

def clip_and_recon(seed, N, T, H, W, noise=0.05):
    rng = np.random.default_rng(seed)
    u8 = rng.integers(0, 256, (N, T, H, W, 3)).astype(np.uint8)
    xhat = O.pixels_to_input(u8) + rng.normal(0, noise, u8.shape)
    return u8, xhat


def test_residual_of_a_perfect_reconstruction_is_empty():
    u8, _ = clip_and_recon(0, 2, 5, 4, 6)
    r, rs, lists = K.residual_compress(u8, O.pixels_to_input(u8), 1e-3)
    assert not r.any() and not rs.any() and all(len(i) == 0 for i, _ in lists)


def test_residual_constant_in_time_is_recovered_exactly():
    """x_hat_t = x_t - c for every t: the mean is c, and with theta below |c|
    the receiver's x_hat_t + r reproduces x exactly (c a dyadic rational)."""
    u8, _ = clip_and_recon(1, 1, 9, 3, 5)
    x = u8.astype(np.float64) / 127.5 - 1.0
    c = np.random.default_rng(2).integers(-8, 9, (1, 3, 5, 3)) / 64.0
    xhat = x - c[:, None]
    r, rs, lists = K.residual_compress(u8, xhat, 0.01)
    np.testing.assert_array_equal(r, c)
    np.testing.assert_array_equal(rs, c)
    np.testing.assert_allclose(K.residual_apply(xhat, rs), x, rtol=0, atol=1e-15)


def test_residual_mean_and_threshold_by_brute_force():
    N, T, H, W = 2, 5, 3, 4
    u8, xhat = clip_and_recon(3, N, T, H, W, noise=0.2)
    theta = 0.05
    r, rs, lists = K.residual_compress(u8, xhat, theta)
    for n in range(N):
        for h in range(H):
            for w in range(W):
                for c in range(3):
                    s = 0.0
                    for t in range(T):
                        s += (u8[n, t, h, w, c] / 127.5 - 1.0) - xhat[n, t, h, w, c]
                    assert abs(r[n, h, w, c] - s / T) < 1e-14
                    assert rs[n, h, w, c] == (0.0 if abs(r[n, h, w, c]) < theta else r[n, h, w, c])
    for n, (ix, val) in enumerate(lists):
        assert (np.diff(ix) > 0).all() and (val != 0).all()
        back = np.zeros(H * W * 3)
        back[ix] = val
        np.testing.assert_array_equal(back.reshape(H, W, 3), rs[n])


def test_residual_threshold_extremes():
    u8, xhat = clip_and_recon(4, 1, 5, 4, 4)
    r, rs0, l0 = K.residual_compress(u8, xhat, 0.0)
    np.testing.assert_array_equal(rs0, r)                     # theta = 0 keeps everything
    _, rsi, li = K.residual_compress(u8, xhat, np.inf)
    assert not rsi.any() and len(li[0][0]) == 0


# ---- GoP blending --------------------------------------------------------------

def test_blend_weights_as_written():
    assert K.blend_weights(2) == [0.5, 0.0]
    assert K.blend_weights(4) == [0.75, 0.5, 0.25, 0.0]


def test_blend_by_hand_n2():
    prev = np.arange(5, dtype=np.float64).reshape(1, 5, 1, 1, 1) * 10.0       # frames 0, 10, 20, 30, 40
    curr = 100.0 + np.arange(4, dtype=np.float64).reshape(1, 4, 1, 1, 1)     # 100, 101, 102, 103
    out = K.gop_blend(prev, curr, 2)
    # i = 1: alpha 1/2 with prev frame T - 2 + 1 = 4 (1-based) = 30; i = 2: alpha 0
    np.testing.assert_array_equal(out.ravel(), [65.0, 101.0, 102.0, 103.0])


def test_blend_identities():
    rng = np.random.default_rng(6)
    a = rng.normal(size=(2, 9, 3, 4, 3))
    b = rng.normal(size=(2, 9, 3, 4, 3))
    np.testing.assert_array_equal(K.gop_blend(a, b, 1), b)     # alpha_1 = 0 for n = 1
    same = a.copy()
    same[:, 6:] = b[:, :3]          # the previous GoP ends as the current one starts: nothing changes
    np.testing.assert_allclose(K.gop_blend(same, b, 3), b, rtol=0, atol=1e-15)
    out = K.gop_blend(a, b, 3)
    np.testing.assert_array_equal(out[:, 3:], b[:, 3:])
    np.testing.assert_allclose(out[:, 0], (2 * a[:, 6] + b[:, 0]) / 3, rtol=0, atol=1e-14)
    np.testing.assert_allclose(out[:, 1], (a[:, 7] + 2 * b[:, 1]) / 3, rtol=0, atol=1e-14)
