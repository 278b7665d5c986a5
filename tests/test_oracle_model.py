"""Whole-model pins of the oracle: shapes, causality (Sec. 4.3: the first
frame of a GoP is coded on its own), prefix consistency, torch cross-check of
the composed encoder/decoder, and a frozen regression fixture."""
import json
import os

import numpy as np
import pytest
import torch

import synth
from oracle import tokenizer as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_config0.json")


@pytest.fixture(scope="module")
def params():
    return {k: v.astype(np.float64) for k, v in synth.make_weights(1, random_affine=True).items()}


@pytest.fixture(scope="module")
def small_clip():
    return synth.make_batch([0], 9, 16, 24)


def test_param_count():
    assert synth.param_count() == 2225929
    conv = sum(int(np.prod(s)) for _, k, s in synth.param_spec() if k == "conv")
    assert conv == 2223744


def test_shapes(params, small_clip):
    z = O.encode(small_clip, params)
    assert z.shape == (1, 3, 4, 6, 6)
    assert O.latent_shape(17, 720, 1280) == (5, 180, 320)
    assert O.latent_shape(33, 1080, 1920) == (9, 270, 480)
    xh = O.decode(O.fsq(z)[0], params)
    assert xh.shape == (1, 9, 16, 24, 3)


def test_encoder_causality(params, small_clip):
    """Perturbing input frame s leaves latent frames k with 4k < s bit-identical."""
    z = O.encode(small_clip, params)
    for s in (1, 5, 8):
        u = small_clip.copy()
        u[:, s] = 255 - u[:, s]
        z2 = O.encode(u, params)
        for k in range(z.shape[1]):
            if 4 * k < s:
                np.testing.assert_array_equal(z2[:, k], z[:, k])
            else:
                assert not np.array_equal(z2[:, k], z[:, k])


def test_decoder_causality(params):
    c = np.random.default_rng(0).integers(-2, 2, (1, 3, 4, 6, 6)) / 2.0
    x = O.decode(c, params)
    for k in (1, 2):
        c2 = c.copy()
        c2[:, k] = -c2[:, k] + 0.5
        x2 = O.decode(c2, params)
        for t in range(x.shape[1]):
            if t <= 4 * k - 4:
                np.testing.assert_array_equal(x2[:, t], x[:, t])
            else:
                assert not np.array_equal(x2[:, t], x[:, t])


def test_prefix_equals_whole_clip(params, small_clip):
    """Encoding the first 4k+1 frames gives the first k+1 latent frames of the
    whole clip; decoding a latent prefix gives the output prefix."""
    z = O.encode(small_clip, params)
    zp = O.encode(small_clip[:, :5], params)
    np.testing.assert_allclose(zp, z[:, :2], rtol=0, atol=1e-12)
    c = O.fsq(z)[0]
    x = O.decode(c, params)
    xp = O.decode(c[:, :2], params)
    np.testing.assert_allclose(xp, x[:, :5], rtol=0, atol=1e-12)


def _torch_causal_conv(x, w, b, stride=1):
    """Library route: pad by hand (frame 0 twice in front, zeros in space), conv3d."""
    if w.shape[2] == 1:
        return torch.nn.functional.conv3d(x, w, b)
    x = torch.cat([x[:, :, :1], x[:, :, :1], x], dim=2)
    x = torch.nn.functional.pad(x, (1, 1, 1, 1))
    return torch.nn.functional.conv3d(x, w, b, stride=stride)


def _torch_up(x):
    T = x.shape[2]
    idx = torch.tensor([(t + 1) // 2 for t in range(2 * T - 1)])
    x = x[:, :, idx]
    return x.repeat_interleave(2, dim=3).repeat_interleave(2, dim=4)


def _torch_gn(x, g, b):
    N, C, T, H, W = x.shape
    y = x.permute(0, 2, 1, 3, 4).reshape(N * T, C, H, W)
    y = torch.nn.functional.group_norm(y, 32, g, b, eps=1e-6)
    return y.reshape(N, T, C, H, W).permute(0, 2, 1, 3, 4)


def torch_encode_decode(u8, p, codes=None):
    """The stand-in composed from torch library routines (float64, NCTHW)."""
    P = {k: torch.from_numpy(np.asarray(v, np.float64)) for k, v in p.items()}
    silu = torch.nn.functional.silu

    def rb(x, n):
        h = _torch_causal_conv(silu(_torch_gn(x, P[n + ".gn_a.gamma"], P[n + ".gn_a.beta"])),
                               P[n + ".a.w"], P[n + ".a.b"])
        h = _torch_causal_conv(silu(_torch_gn(h, P[n + ".gn_b.gamma"], P[n + ".gn_b.beta"])),
                               P[n + ".b.w"], P[n + ".b.b"])
        return x + h

    x = torch.from_numpy(np.asarray(u8, np.float64)).permute(0, 4, 1, 2, 3) / 127.5 - 1.0
    h = _torch_causal_conv(x, P["enc.conv_in.w"], P["enc.conv_in.b"])
    h = rb(rb(h, "enc.rb1"), "enc.rb2")
    h = _torch_causal_conv(h, P["enc.down1.w"], P["enc.down1.b"], 2)
    h = _torch_causal_conv(h, P["enc.down2.w"], P["enc.down2.b"], 2)
    z = _torch_causal_conv(h, P["enc.proj.w"], P["enc.proj.b"])
    c = torch.from_numpy(codes).permute(0, 4, 1, 2, 3)
    g = _torch_causal_conv(c, P["dec.proj_in.w"], P["dec.proj_in.b"])
    g = _torch_causal_conv(_torch_up(g), P["dec.up2.w"], P["dec.up2.b"])
    g = _torch_causal_conv(_torch_up(g), P["dec.up1.w"], P["dec.up1.b"])
    g = rb(rb(g, "dec.rb1"), "dec.rb2")
    xh = _torch_causal_conv(g, P["dec.conv_out.w"], P["dec.conv_out.b"])
    return z.permute(0, 2, 3, 4, 1).numpy(), xh.permute(0, 2, 3, 4, 1).numpy()


def test_model_matches_torch_composition(params, small_clip):
    z = O.encode(small_clip, params)
    c = O.fsq(z)[0]
    zt, xt = torch_encode_decode(small_clip, params, c)
    np.testing.assert_allclose(z, zt, rtol=0, atol=1e-10)
    np.testing.assert_allclose(O.decode(c, params), xt, rtol=0, atol=1e-10)


def test_config0_regression_fixture():
    """Frozen oracle output on the 1x9x64x64 clip (seed 0, weights seed 1),
    written by tests/golden/make_oracle_golden.py from the oracle alone."""
    with open(GOLDEN) as f:
        g = json.load(f)
    u8 = synth.make_batch([0], 9, 64, 64)
    assert synth.sha256(u8) == g["clip_sha256"]
    w = synth.make_weights(1)
    assert synth.sha256(synth.flatten_weights(w)) == g["weights_sha256"]
    r = O.roundtrip(u8, {k: v.astype(np.float64) for k, v in w.items()})
    band = O.fsq_boundary_distance(r["b"]).min(axis=-1) < 1e-3
    ok = ~band.reshape(-1)
    np.testing.assert_array_equal(r["idx"].reshape(-1)[ok], np.array(g["idx"])[ok])
    np.testing.assert_allclose(r["xhat"].reshape(-1)[:: 97], g["xhat_every_97th"], rtol=0, atol=1e-9)
    assert abs(float(r["xhat"].std()) - g["xhat_std"]) < 1e-9
