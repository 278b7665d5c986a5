"""Pins of the oracle's causal convolution and upsample against definitions
that do not go through its own code: seven nested loops, torch's conv3d in
float64 on explicitly padded input, the 1x1x1 matrix-product special case,
linearity and shift equivariance."""
import numpy as np
import pytest
import torch

import synth
from oracle import tokenizer as O


def _rand(seed, shape):
    return synth.randn(seed, shape, dtype=np.float64)


@pytest.mark.parametrize("stride", [(1, 1), (2, 2)])
@pytest.mark.parametrize("T", [1, 3, 5])
def test_conv_matches_bruteforce(stride, T):
    if stride[0] == 2 and T == 1:
        T = 1
    x = _rand(1, (1, T, 6, 6, 2))
    w = _rand(2, (3, 2, 3, 3, 3))
    b = _rand(3, (3,))
    y = O.conv3d(x, w, b, stride)
    yb = O.conv3d_bruteforce(x, w, b, stride)
    assert y.shape == yb.shape
    np.testing.assert_allclose(y, yb, rtol=0, atol=1e-13)


def test_conv_matches_torch_conv3d_on_padded_input():
    """torch.nn.functional.conv3d (CPU, float64) on an input padded by hand:
    two replicated copies of frame 0 in front, one zero row/col per side."""
    rng = np.random.default_rng(0)
    for stride in [(1, 1), (2, 2)]:
        x = rng.standard_normal((2, 5, 8, 12, 4))
        w = rng.standard_normal((5, 4, 3, 3, 3))
        b = rng.standard_normal(5)
        xt = torch.from_numpy(x).permute(0, 4, 1, 2, 3)  # N C T H W
        xt = torch.cat([xt[:, :, :1], xt[:, :, :1], xt], dim=2)
        xt = torch.nn.functional.pad(xt, (1, 1, 1, 1))
        yt = torch.nn.functional.conv3d(xt, torch.from_numpy(w), torch.from_numpy(b),
                                        stride=(stride[0], stride[1], stride[1]))
        ref = yt.permute(0, 2, 3, 4, 1).numpy()
        np.testing.assert_allclose(O.conv3d(x, w, b, stride), ref, rtol=0, atol=1e-12)


def test_pointwise_conv_is_matmul():
    x = _rand(4, (2, 3, 4, 5, 128))
    w = _rand(5, (6, 128, 1, 1, 1))
    b = _rand(6, (6,))
    ref = np.einsum("nthwi,oi->nthwo", x, w[:, :, 0, 0, 0]) + b
    np.testing.assert_allclose(O.conv3d(x, w, b), ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(O.conv3d_bruteforce(x[:, :1, :2, :2], w, b),
                               ref[:, :1, :2, :2], rtol=0, atol=1e-12)


def test_conv_linearity():
    x1, x2 = _rand(7, (1, 5, 8, 8, 3)), _rand(8, (1, 5, 8, 8, 3))
    w = _rand(9, (4, 3, 3, 3, 3))
    a, c = 0.7, -1.3
    lhs = O.conv3d(a * x1 + c * x2, w)
    rhs = a * O.conv3d(x1, w) + c * O.conv3d(x2, w)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-12)


def test_conv_spatial_shift_equivariance_interior():
    """Shifting the input by 2 px shifts a stride-2 output by 1, away from the border."""
    x = _rand(10, (1, 3, 16, 16, 2))
    w = _rand(11, (3, 2, 3, 3, 3))
    xs = np.zeros_like(x)
    xs[:, :, 2:, 2:] = x[:, :, :-2, :-2]
    y = O.conv3d(x, w, stride=(2, 2))
    ys = O.conv3d(xs, w, stride=(2, 2))
    np.testing.assert_allclose(ys[:, :, 2:7, 2:7], y[:, :, 1:6, 1:6], rtol=0, atol=1e-12)


def test_conv_causal_first_frame():
    """Output frame 0 of a causal conv sees input frame 0 only: it equals a
    2-D conv of frame 0 with the three temporal taps summed."""
    x = _rand(12, (1, 5, 6, 6, 2))
    w = _rand(13, (3, 2, 3, 3, 3))
    y = O.conv3d(x, w)
    w2 = w.sum(axis=2, keepdims=True)
    x0 = torch.from_numpy(x[:, 0]).permute(0, 3, 1, 2)
    ref = torch.nn.functional.conv2d(x0, torch.from_numpy(w2[:, :, 0]), padding=1)
    np.testing.assert_allclose(y[:, 0], ref.permute(0, 2, 3, 1).numpy(), rtol=0, atol=1e-12)


def test_upsample_index_identities():
    x = _rand(14, (2, 3, 4, 5, 3))
    u = O.upsample(x)
    assert u.shape == (2, 5, 8, 10, 3)
    for m in range(1, 3):
        np.testing.assert_array_equal(u[:, 2 * m - 1], u[:, 2 * m])
        np.testing.assert_array_equal(u[:, 2 * m, ::2, ::2], x[:, m])
    np.testing.assert_array_equal(u[:, 0, 1::2, 1::2], x[:, 0])
    # Against a loop over output indices
    for t in range(5):
        for h in range(8):
            for w in range(10):
                np.testing.assert_array_equal(u[:, t, h, w], x[:, (t + 1) // 2, h // 2, w // 2])
