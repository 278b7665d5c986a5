"""Pins of the oracle's hand-written backward: dot-product (adjoint) tests per
operation, torch float64 autograd of the same composition, and central finite
differences (h = 1e-6) of the frozen-rounding surrogate, whose exact gradient
is the straight-through gradient."""
import numpy as np
import pytest
import torch

import synth
from oracle import backward as B
from oracle import tokenizer as O


def _r(seed, shape):
    return synth.randn(seed, shape, dtype=np.float64)


@pytest.mark.parametrize("stride,k", [((1, 1), 3), ((2, 2), 3), ((1, 1), 1)])
def test_conv_adjoint_dot_product(stride, k):
    x = _r(0, (2, 5, 8, 8, 3))
    w = _r(1, (4, 3, k, k, k))
    y = O.conv3d(x, w, None, stride)
    gy = _r(2, y.shape)
    gx = B.conv3d_dgrad(gy, w, x.shape, stride)
    lhs, rhs = np.vdot(y, gy), np.vdot(x, gx)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
    # wgrad: <conv(x; v), gy> = <v, dW>
    v = _r(3, w.shape)
    gw, gb = B.conv3d_wgrad(x, gy, w.shape, stride)
    lhs = np.vdot(O.conv3d(x, v, None, stride), gy)
    assert abs(lhs - np.vdot(v, gw)) <= 1e-12 * max(abs(lhs), 1.0)
    np.testing.assert_allclose(gb, gy.reshape(-1, 4).sum(0), rtol=1e-13)


def test_upsample_adjoint_dot_product():
    x = _r(4, (1, 3, 4, 6, 5))
    u = O.upsample(x)
    g = _r(5, u.shape)
    assert abs(np.vdot(u, g) - np.vdot(x, B.upsample_adjoint(g))) < 1e-11


def test_group_norm_backward_matches_torch_autograd():
    x = _r(6, (2, 3, 5, 4, 64)) * 2 + 0.3
    gam, bet = _r(7, (64,)), _r(8, (64,))
    gy = _r(9, x.shape)
    dx, dg, db = B.group_norm_backward(x, gam, gy)
    xt = torch.from_numpy(x).requires_grad_()
    gt = torch.from_numpy(gam).requires_grad_()
    bt = torch.from_numpy(bet).requires_grad_()
    N, T, H, W, C = x.shape
    y = torch.nn.functional.group_norm(xt.reshape(N * T, H, W, C).permute(0, 3, 1, 2), 32, gt, bt, 1e-6)
    y = y.permute(0, 2, 3, 1).reshape(x.shape)
    y.backward(torch.from_numpy(gy))
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=0, atol=1e-11)
    np.testing.assert_allclose(dg, gt.grad.numpy(), rtol=0, atol=1e-11)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=0, atol=1e-11)


def test_silu_backward_finite_difference():
    a = np.linspace(-8, 8, 101)
    h = 1e-6
    fd = (O.silu(a + h) - O.silu(a - h)) / (2 * h)
    np.testing.assert_allclose(B.silu_backward(a, np.ones_like(a)), fd, rtol=1e-8, atol=1e-10)


@pytest.fixture(scope="module")
def tiny():
    """Tiny clip 1x5x16x16 with non-trivial biases / affine, and a token mask."""
    u8 = synth.make_batch([0], 5, 16, 16)
    p = {k: v.astype(np.float64) for k, v in synth.make_weights(1, random_affine=True).items()}
    keep = O.keep_mask(O.DROP_BERNOULLI, 0.25, 7, [0], 2, 4, 4)
    return u8, p, keep


def _torch_loss(u8, p, keep):
    """Same objective from torch library routines with autograd; the STE is
    c = z~ + (rint(b)/d - z~).detach()."""
    from tests.test_oracle_model import _torch_causal_conv, _torch_gn, _torch_up
    P = {k: torch.from_numpy(np.asarray(v, np.float64).copy()).requires_grad_() for k, v in p.items()}
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
    L = torch.tensor([8., 8, 8, 5, 5, 5], dtype=torch.float64).reshape(1, 6, 1, 1, 1)
    hh = (L - 1) * (1 - 1e-3) / 2
    o = torch.where(L % 2 == 0, 0.5, 0.0)
    s = torch.atanh(o / hh)
    d = torch.floor(L / 2)
    b = torch.tanh(z + s) * hh - o
    zt = b / d
    c = zt + (torch.round(b) / d - zt).detach()
    kt = torch.from_numpy(np.asarray(keep, np.float64)).unsqueeze(1)
    g = _torch_causal_conv(c * kt, P["dec.proj_in.w"], P["dec.proj_in.b"])
    g = _torch_causal_conv(_torch_up(g), P["dec.up2.w"], P["dec.up2.b"])
    g = _torch_causal_conv(_torch_up(g), P["dec.up1.w"], P["dec.up1.b"])
    g = rb(rb(g, "dec.rb1"), "dec.rb2")
    xh = _torch_causal_conv(g, P["dec.conv_out.w"], P["dec.conv_out.b"])
    loss = (xh - x).abs().mean() + 0.1 * ((zt - c.detach()) ** 2).mean()
    loss.backward()
    return float(loss), {k: v.grad.numpy() for k, v in P.items()}


def test_gradient_matches_torch_autograd(tiny):
    u8, p, keep = tiny
    loss, tape = B.train_forward(u8, p, keep)
    grads, _ = B.train_backward(tape, p)
    tl, tg = _torch_loss(u8, p, keep)
    assert abs(loss - tl) < 1e-12
    for name, _, _ in synth.param_spec():
        ref = tg[name]
        np.testing.assert_allclose(grads[name], ref, rtol=0,
                                   atol=1e-10 * max(1.0, np.abs(ref).max()), err_msg=name)


def _surrogate_fd(u8, p, keep, frozen, direction, h=1e-6):
    pp = {k: v + h * direction.get(k, 0.0) for k, v in p.items()}
    pm = {k: v - h * direction.get(k, 0.0) for k, v in p.items()}
    lp, _ = B.train_forward(u8, pp, keep, frozen)
    lm, _ = B.train_forward(u8, pm, keep, frozen)
    return (lp - lm) / (2 * h)


def _frozen(tape):
    return (tape["codes"] - tape["zt"], tape["codes"])


def test_gradient_finite_difference_per_tensor(tiny):
    """One random unit direction per parameter tensor (38 tensors), rel 1e-6."""
    u8, p, keep = tiny
    loss, tape = B.train_forward(u8, p, keep)
    grads, _ = B.train_backward(tape, p)
    frozen = _frozen(tape)
    rng = np.random.default_rng(11)
    for name, _, shape in synth.param_spec():
        v = rng.standard_normal(shape)
        v /= np.linalg.norm(v)
        fd = _surrogate_fd(u8, p, keep, frozen, {name: v})
        an = float(np.vdot(grads[name], v))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-4 * np.linalg.norm(grads[name]), 1e-9), (name, fd, an)


def test_gradient_finite_difference_coordinates(tiny):
    """20 random single weights."""
    u8, p, keep = tiny
    loss, tape = B.train_forward(u8, p, keep)
    grads, _ = B.train_backward(tape, p)
    frozen = _frozen(tape)
    rng = np.random.default_rng(12)
    spec = synth.param_spec()
    for _ in range(20):
        name, _, shape = spec[int(rng.integers(len(spec)))]
        idx = tuple(int(rng.integers(s)) for s in shape)
        e = np.zeros(shape)
        e[idx] = 1.0
        fd = _surrogate_fd(u8, p, keep, frozen, {name: e})
        an = float(grads[name][idx])
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.abs(grads[name]).max(), 1e-9), (name, idx, fd, an)


@pytest.mark.slow
def test_gradient_finite_difference_config0_clip():
    """The 1x9x64x64 clip: 2 global random directions + 20 input pixels
    (the input gradient, through the encoder)."""
    u8 = synth.make_batch([0], 9, 64, 64)
    p = {k: v.astype(np.float64) for k, v in synth.make_weights(1).items()}
    keep = O.keep_mask(O.DROP_BERNOULLI, 0.25, 3, [0], 3, 16, 16)
    loss, tape = B.train_forward(u8, p, keep)
    grads, dx = B.train_backward(tape, p)
    frozen = _frozen(tape)
    rng = np.random.default_rng(13)
    for _ in range(2):
        d = {name: rng.standard_normal(shape) for name, _, shape in synth.param_spec()}
        nrm = np.sqrt(sum(float((v * v).sum()) for v in d.values()))
        d = {k: v / nrm for k, v in d.items()}
        fd = _surrogate_fd(u8, p, keep, frozen, d)
        an = sum(float(np.vdot(grads[k], d[k])) for k in d)
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
    assert dx.shape == (1, 9, 64, 64, 3)


def test_outputs_backward_finite_difference(tiny):
    """The adjoint for gradients from outside (the codec's gradient interface):
    F = <g_xhat, x_hat> + <g_codes, keep c> + <g_z, z> on the frozen-rounding
    surrogate, one random direction per parameter tensor and the input, rel 1e-6;
    with g_codes = g_z = 0 it is train_backward's adjoint from the same seed."""
    u8, p, keep = tiny
    _, tape = B.train_forward(u8, p, keep)
    rng = np.random.default_rng(21)
    gx = rng.standard_normal(tape["xhat"].shape)
    gc = rng.standard_normal(tape["dec_in"].shape)
    gz = rng.standard_normal(tape["z"].shape)
    grads, dx = B.outputs_backward(tape, p, gx, gc, gz)
    frozen = _frozen(tape)

    def F(pp, u=None):
        _, t = B.train_forward(u8 if u is None else u, pp, keep, frozen)
        return float(np.vdot(gx, t["xhat"]) + np.vdot(gc, t["dec_in"]) + np.vdot(gz, t["z"]))

    h = 1e-6
    for name, _, shape in synth.param_spec():
        v = rng.standard_normal(shape)
        v /= np.linalg.norm(v)
        fd = (F({**p, name: p[name] + h * v}) - F({**p, name: p[name] - h * v})) / (2 * h)
        an = float(np.vdot(grads[name], v))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-4 * np.linalg.norm(grads[name]), 1e-9), (name, fd, an)
    # the zero-seed special case reduces to the loss adjoint's structure
    g0, dx0 = B.outputs_backward(tape, p, gx)
    g1, dx1 = B._adjoint(tape, p, gx)
    for k in g0:
        np.testing.assert_array_equal(g0[k], g1[k])
    np.testing.assert_array_equal(dx0, dx1)


def test_fsq_ste_backward_finite_difference():
    """dz~/dz by central differences of b / floor(L/2) away from saturation."""
    z = np.linspace(-2.0, 2.0, 61)[:, None] * np.ones((1, 6))
    dd = O.fsq_constants()[3]
    zt = lambda v: O.fsq(v)[3] / dd  # noqa: E731  (b of the quantiser's forward, normalised)
    eps = 1e-6
    fd = (zt(z + eps) - zt(z - eps)) / (2 * eps)
    np.testing.assert_allclose(B.fsq_ste_backward(z, np.ones_like(z)), fd, rtol=1e-8, atol=1e-12)
