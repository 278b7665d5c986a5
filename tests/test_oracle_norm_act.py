"""Pins of the oracle's per-frame GroupNorm and SiLU."""
import numpy as np
import torch

import synth
from oracle import tokenizer as O


def test_group_norm_matches_torch():
    x = synth.randn(0, (2, 3, 5, 7, 64), scale=3.0, dtype=np.float64) + 1.5
    g = synth.randn(1, (64,), dtype=np.float64)
    b = synth.randn(2, (64,), dtype=np.float64)
    y = O.group_norm(x, g, b)
    N, T, H, W, C = x.shape
    xt = torch.from_numpy(x).reshape(N * T, H, W, C).permute(0, 3, 1, 2)
    ref = torch.nn.functional.group_norm(xt, 32, torch.from_numpy(g), torch.from_numpy(b), eps=1e-6)
    ref = ref.permute(0, 2, 3, 1).reshape(x.shape).numpy()
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12)


def test_group_norm_invariants():
    x = synth.randn(3, (1, 4, 6, 6, 64), scale=2.0, dtype=np.float64)
    y = O.group_norm(x, np.ones(64), np.zeros(64))
    yg = y.reshape(1, 4, 6, 6, 32, 2)
    xg = x.reshape(1, 4, 6, 6, 32, 2)
    np.testing.assert_allclose(yg.mean(axis=(2, 3, 5)), 0.0, atol=1e-12)
    var = xg.var(axis=(2, 3, 5))
    np.testing.assert_allclose(yg.var(axis=(2, 3, 5)), var / (var + 1e-6), rtol=1e-10)
    # invariance to a per-(frame, group) positive affine change of the input
    a = np.random.default_rng(4).uniform(0.5, 2.0, (1, 4, 1, 1, 32, 1))
    c = np.random.default_rng(5).uniform(-3, 3, (1, 4, 1, 1, 32, 1))
    x2 = (xg * a + c).reshape(x.shape)
    # eps breaks exact invariance; compare with eps rescaled
    y2 = O.group_norm(x2 / 1.0, np.ones(64), np.zeros(64), eps=1e-30)
    y1 = O.group_norm(x, np.ones(64), np.zeros(64), eps=1e-30)
    np.testing.assert_allclose(y1, y2, atol=1e-10)


def test_group_norm_is_per_frame():
    """Changing frame 2 leaves the normalised frames 0, 1 bit-identical."""
    x = synth.randn(6, (1, 4, 6, 6, 64), dtype=np.float64)
    x2 = x.copy()
    x2[:, 2:] *= 5.0
    y, y2 = O.group_norm(x, np.ones(64), np.zeros(64)), O.group_norm(x2, np.ones(64), np.zeros(64))
    np.testing.assert_array_equal(y[:, :2], y2[:, :2])


def test_silu_closed_forms():
    x = np.linspace(-40, 40, 10001)
    s = O.silu(x)
    np.testing.assert_allclose(s - O.silu(-x), x, atol=1e-12)
    np.testing.assert_allclose(s, x / (1.0 + np.exp(-x)), rtol=1e-14, atol=1e-300)
    assert O.silu(np.array([0.0]))[0] == 0.0
    np.testing.assert_allclose(O.silu(np.array([-800.0, 800.0])), [-0.0, 800.0])
