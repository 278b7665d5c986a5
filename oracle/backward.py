"""FP64 training step of the stand-in tokenizer: loss and its hand-written adjoint.

TEST INFRASTRUCTURE ONLY.

Paper anchors: the appendix trains the codec with an l1 pixel loss (Eq. 5;
the optical-flow and adversarial terms need networks the stand-in does not
have) and, in the drop-robust stage (Eq. 7), decodes the zero-filled token
tensor while gradients flow back into the encoder through the codec's
"internal gradient interface" (Sec. 4.1).  The stand-in's loss is

    L = mean |x_hat - x| + 0.1 * mean (z~ - sg(c))^2

with z~ = b / floor(L/2) the unrounded normalised code, c = rint(b)/floor(L/2)
its quantised value, and a straight-through estimator dc/dz~ = 1.  The
decoder consumes keep * c, so dropped tokens pass no decoder gradient.
sign(0) = 0 is the l1 subgradient.
"""
from __future__ import annotations

import numpy as np

from .tokenizer import (COMMIT_WEIGHT, _pad_causal, conv3d, conv_out_shape, fsq, fsq_constants,
                        group_norm, pixels_to_input, sigmoid, silu, upsample, GN_GROUPS, GN_EPS)

# ---------------------------------------------------------------------------
# Adjoints of the elementary operations
# ---------------------------------------------------------------------------


def conv3d_dgrad(gy, w, in_shape, stride=(1, 1)):
    """Adjoint of the bias-free causal conv with respect to its input.
    Scatter each tap's contribution into the padded input, then fold the two
    replicated time-pad frames back onto frame 0 and drop the spatial pad."""
    w = np.asarray(w, np.float64)
    N, T, H, W_, Ci = in_shape
    Co = w.shape[0]
    if w.shape[2:] == (1, 1, 1):
        return (gy.reshape(-1, Co) @ np.ascontiguousarray(w[:, :, 0, 0, 0])).reshape(in_shape)
    st, ss = stride
    To, Ho, Wo = conv_out_shape(T, H, W_, stride)
    wt = np.ascontiguousarray(w.transpose(2, 3, 4, 0, 1))  # [kt, kh, kw, Co, Ci]
    gp = np.zeros((N, T + 2, H + 2, W_ + 2, Ci))
    for n in range(N):
        for t in range(To):
            g2 = np.ascontiguousarray(gy[n, t]).reshape(-1, Co)
            for kt in range(3):
                for kh in range(3):
                    for kw in range(3):
                        contrib = (g2 @ wt[kt, kh, kw]).reshape(Ho, Wo, Ci)
                        gp[n, st * t + kt, kh:kh + ss * (Ho - 1) + 1:ss,
                           kw:kw + ss * (Wo - 1) + 1:ss, :] += contrib
    gx = gp[:, 2:, 1:-1, 1:-1].copy()
    gx[:, 0] += gp[:, 0, 1:-1, 1:-1] + gp[:, 1, 1:-1, 1:-1]
    return gx


def conv3d_wgrad(x, gy, wshape, stride=(1, 1)):
    """dL/dW[o,i,kt,kh,kw] = sum over output positions of gy[o] * x~[tap, i];
    dL/db[o] = sum of gy[o]."""
    x = np.asarray(x, np.float64)
    N, T, H, W_, Ci = x.shape
    Co = wshape[0]
    gw = np.zeros(wshape)
    gb = gy.reshape(-1, Co).sum(axis=0)
    if wshape[2:] == (1, 1, 1):
        gw[:, :, 0, 0, 0] = gy.reshape(-1, Co).T @ x.reshape(-1, Ci)
        return gw, gb
    st, ss = stride
    To, Ho, Wo = conv_out_shape(T, H, W_, stride)
    xp = _pad_causal(x)
    for n in range(N):
        for t in range(To):
            g2t = np.ascontiguousarray(gy[n, t].reshape(-1, Co).T)
            for kt in range(3):
                frame = xp[n, st * t + kt]
                for kh in range(3):
                    for kw in range(3):
                        sl = frame[kh:kh + ss * (Ho - 1) + 1:ss, kw:kw + ss * (Wo - 1) + 1:ss, :]
                        gw[:, :, kt, kh, kw] += g2t @ np.ascontiguousarray(sl).reshape(-1, Ci)
    return gw, gb


def upsample_adjoint(g):
    """Adjoint of the nearest x2 upsample: sum each 2x2 spatial block and the
    time frames that copy the same source frame (t = 2m-1 and 2m; t = 0 alone)."""
    N, Tu, Hu, Wu, C = g.shape
    T = (Tu + 1) // 2
    gs = g.reshape(N, Tu, Hu // 2, 2, Wu // 2, 2, C).sum(axis=(3, 5))
    out = np.zeros((N, T, Hu // 2, Wu // 2, C))
    tidx = (np.arange(Tu) + 1) // 2
    for t in range(Tu):
        out[:, tidx[t]] += gs[:, t]
    return out


def group_norm_backward(x, gamma, gy, groups=GN_GROUPS, eps=GN_EPS):
    """Adjoint of the per-frame GroupNorm: returns (dx, dgamma, dbeta)."""
    N, T, H, W_, C = x.shape
    cg = C // groups
    xg = x.reshape(N, T, H, W_, groups, cg)
    mu = xg.mean(axis=(2, 3, 5), keepdims=True)
    var = ((xg - mu) ** 2).mean(axis=(2, 3, 5), keepdims=True)
    rstd = 1.0 / np.sqrt(var + eps)
    xh = (xg - mu) * rstd
    gyg = gy.reshape(xg.shape)
    gam = np.asarray(gamma, np.float64).reshape(groups, cg)
    gxh = gyg * gam
    m1 = gxh.mean(axis=(2, 3, 5), keepdims=True)
    m2 = (gxh * xh).mean(axis=(2, 3, 5), keepdims=True)
    dx = (rstd * (gxh - m1 - xh * m2)).reshape(x.shape)
    dgamma = (gyg * xh).sum(axis=(0, 1, 2, 3)).reshape(C)
    dbeta = gyg.sum(axis=(0, 1, 2, 3)).reshape(C)
    return dx, dgamma, dbeta


def fsq_ste_backward(z, g_zt):
    """Gradient with respect to z of the quantiser under the straight-through
    rule: c = rint(b) / floor(L/2) passes dL/dc unchanged to
    z~ = b / floor(L/2), and b = tanh(z + s) h - o, so
    dL/dz = dL/dz~ * (h / floor(L/2)) * (1 - tanh^2(z + s))."""
    h, o, s, dd = fsq_constants()
    th = np.tanh(np.asarray(z, np.float64) + s)
    return g_zt * (h / dd) * (1.0 - th * th)


def silu_backward(a, g):
    s = sigmoid(a)
    return g * s * (1.0 + a * (1.0 - s))


# ---------------------------------------------------------------------------
# Residual block with tape
# ---------------------------------------------------------------------------


def resblock_fwd(x, p, name):
    gn_a = group_norm(x, p[name + ".gn_a.gamma"], p[name + ".gn_a.beta"])
    s1 = silu(gn_a)
    c1 = conv3d(s1, p[name + ".a.w"], p[name + ".a.b"])
    gn_b = group_norm(c1, p[name + ".gn_b.gamma"], p[name + ".gn_b.beta"])
    s2 = silu(gn_b)
    c2 = conv3d(s2, p[name + ".b.w"], p[name + ".b.b"])
    return x + c2, dict(x=x, gn_a=gn_a, s1=s1, c1=c1, gn_b=gn_b, s2=s2)


def resblock_bwd(tape, p, name, gy, grads):
    gw, gb = conv3d_wgrad(tape["s2"], gy, p[name + ".b.w"].shape)
    grads[name + ".b.w"], grads[name + ".b.b"] = gw, gb
    g = conv3d_dgrad(gy, p[name + ".b.w"], tape["s2"].shape)
    g = silu_backward(tape["gn_b"], g)
    g, grads[name + ".gn_b.gamma"], grads[name + ".gn_b.beta"] = group_norm_backward(
        tape["c1"], p[name + ".gn_b.gamma"], g)
    gw, gb = conv3d_wgrad(tape["s1"], g, p[name + ".a.w"].shape)
    grads[name + ".a.w"], grads[name + ".a.b"] = gw, gb
    g = conv3d_dgrad(g, p[name + ".a.w"], tape["s1"].shape)
    g = silu_backward(tape["gn_a"], g)
    gx, grads[name + ".gn_a.gamma"], grads[name + ".gn_a.beta"] = group_norm_backward(
        tape["x"], p[name + ".gn_a.gamma"], g)
    return gy + gx


# ---------------------------------------------------------------------------
# Whole training step
# ---------------------------------------------------------------------------


def train_forward(u8, p, keep=None, frozen=None):
    """Forward pass of the training objective with everything kept for the
    backward.  keep: (N,T2,H2,W2) token mask (None = keep all).

    frozen: optional (offset, codes0) taken at a reference point.  The
    decoder then consumes keep * (z~ + offset) and the commitment term uses
    the constant codes0.  That surrogate is smooth in the parameters, equals
    the real loss at the reference point, and its exact gradient there equals
    the straight-through gradient, which is what finite differences check.
    """
    tape = {}
    x = pixels_to_input(u8)
    tape["x"] = x
    h0 = conv3d(x, p["enc.conv_in.w"], p["enc.conv_in.b"])
    e1, tape["enc.rb1"] = resblock_fwd(h0, p, "enc.rb1")
    e2, tape["enc.rb2"] = resblock_fwd(e1, p, "enc.rb2")
    d1 = conv3d(e2, p["enc.down1.w"], p["enc.down1.b"], stride=(2, 2))
    d2 = conv3d(d1, p["enc.down2.w"], p["enc.down2.b"], stride=(2, 2))
    z = conv3d(d2, p["enc.proj.w"], p["enc.proj.b"])
    tape.update(e2=e2, d1=d1, d2=d2, z=z)
    codes, idx, q, b = fsq(z)
    h, o, s, dd = fsq_constants()
    zt = b / dd
    dec_codes = codes
    if frozen is not None:
        dec_codes = zt + frozen[0]
        codes = np.asarray(frozen[1], np.float64)
    if keep is None:
        keep = np.ones(z.shape[:-1], np.uint8)
    kf = np.asarray(keep, np.float64)[..., None]
    dec_in = dec_codes * kf
    tape.update(b=b, zt=zt, codes=codes, idx=idx, keep=kf, dec_in=dec_in)
    g = conv3d(dec_in, p["dec.proj_in.w"], p["dec.proj_in.b"])
    ug = upsample(g)
    u2 = conv3d(ug, p["dec.up2.w"], p["dec.up2.b"])
    uu2 = upsample(u2)
    u1 = conv3d(uu2, p["dec.up1.w"], p["dec.up1.b"])
    r1, tape["dec.rb1"] = resblock_fwd(u1, p, "dec.rb1")
    r2, tape["dec.rb2"] = resblock_fwd(r1, p, "dec.rb2")
    xhat = conv3d(r2, p["dec.conv_out.w"], p["dec.conv_out.b"])
    tape.update(ug=ug, uu2=uu2, r2=r2, xhat=xhat)
    l1 = float(np.mean(np.abs(xhat - x)))
    commit = float(np.mean((zt - codes) ** 2))
    loss = l1 + COMMIT_WEIGHT * commit
    tape.update(l1=l1, commit=commit)
    return loss, tape


def train_backward(tape, p, gx_hat=None):
    """Hand-written adjoint of train_forward: returns (grads dict, dx).

    gx_hat: optional dL/dx_hat to use instead of the l1 subgradient
    sign(x_hat - x) / numel.  The l1 term is not differentiable where
    x_hat = x (its subgradient there is any value in [-1, 1] / numel), so a
    caller can evaluate the gradient for another valid choice at such pixels;
    everything after the seed is the same adjoint.
    """
    x, xhat = tape["x"], tape["xhat"]
    if gx_hat is None:
        gx_hat = np.sign(xhat - x) / xhat.size
    zt, codes = tape["zt"], tape["codes"]
    g_commit = 2.0 * COMMIT_WEIGHT * (zt - codes) / zt.size
    return _adjoint(tape, p, gx_hat, g_zt_extra=g_commit)


def outputs_backward(tape, p, g_xhat, g_codes=None, g_z=None):
    """Adjoint of the codec's outputs for gradients that come from outside
    (a loss computed by the caller; the gradient interface of Sec. 4.1):
    returns (grads dict, dx) of the scalar
        <g_xhat, x_hat> + <g_codes, keep * c> + <g_z, z>
    where keep * c is the zero-filled code tensor the decoder reads (Eq. 7),
    z the pre-quantisation latent, and the straight-through rule dc/dz~ = 1
    applies.  No loss term of train_forward's own enters."""
    return _adjoint(tape, p, g_xhat, g_dec_extra=g_codes, g_z_extra=g_z)


def _adjoint(tape, p, gx_hat, g_dec_extra=None, g_zt_extra=None, g_z_extra=None):
    """Back-propagation from dL/dx_hat through decoder, quantiser and encoder.
    g_dec_extra is added to the gradient of the decoder input keep * c,
    g_zt_extra to that of z~, g_z_extra to that of z."""
    grads = {}
    gw, gb = conv3d_wgrad(tape["r2"], gx_hat, p["dec.conv_out.w"].shape)
    grads["dec.conv_out.w"], grads["dec.conv_out.b"] = gw, gb
    g = conv3d_dgrad(gx_hat, p["dec.conv_out.w"], tape["r2"].shape)
    g = resblock_bwd(tape["dec.rb2"], p, "dec.rb2", g, grads)
    g = resblock_bwd(tape["dec.rb1"], p, "dec.rb1", g, grads)
    gw, gb = conv3d_wgrad(tape["uu2"], g, p["dec.up1.w"].shape)
    grads["dec.up1.w"], grads["dec.up1.b"] = gw, gb
    g = upsample_adjoint(conv3d_dgrad(g, p["dec.up1.w"], tape["uu2"].shape))
    gw, gb = conv3d_wgrad(tape["ug"], g, p["dec.up2.w"].shape)
    grads["dec.up2.w"], grads["dec.up2.b"] = gw, gb
    g = upsample_adjoint(conv3d_dgrad(g, p["dec.up2.w"], tape["ug"].shape))
    gw, gb = conv3d_wgrad(tape["dec_in"], g, p["dec.proj_in.w"].shape)
    grads["dec.proj_in.w"], grads["dec.proj_in.b"] = gw, gb
    g_dec_in = conv3d_dgrad(g, p["dec.proj_in.w"], tape["dec_in"].shape)
    if g_dec_extra is not None:
        g_dec_in = g_dec_in + g_dec_extra
    # straight-through: d(codes)/d(z~) = 1; the mask multiplies the decoder path
    g_zt = g_dec_in * tape["keep"]
    if g_zt_extra is not None:
        g_zt = g_zt + g_zt_extra
    g_z = fsq_ste_backward(tape["z"], g_zt)
    if g_z_extra is not None:
        g_z = g_z + g_z_extra
    gw, gb = conv3d_wgrad(tape["d2"], g_z, p["enc.proj.w"].shape)
    grads["enc.proj.w"], grads["enc.proj.b"] = gw, gb
    g = conv3d_dgrad(g_z, p["enc.proj.w"], tape["d2"].shape)
    gw, gb = conv3d_wgrad(tape["d1"], g, p["enc.down2.w"].shape, stride=(2, 2))
    grads["enc.down2.w"], grads["enc.down2.b"] = gw, gb
    g = conv3d_dgrad(g, p["enc.down2.w"], tape["d1"].shape, stride=(2, 2))
    gw, gb = conv3d_wgrad(tape["e2"], g, p["enc.down1.w"].shape, stride=(2, 2))
    grads["enc.down1.w"], grads["enc.down1.b"] = gw, gb
    g = conv3d_dgrad(g, p["enc.down1.w"], tape["e2"].shape, stride=(2, 2))
    g = resblock_bwd(tape["enc.rb2"], p, "enc.rb2", g, grads)
    g = resblock_bwd(tape["enc.rb1"], p, "enc.rb1", g, grads)
    gw, gb = conv3d_wgrad(tape["x"], g, p["enc.conv_in.w"].shape)
    grads["enc.conv_in.w"], grads["enc.conv_in.b"] = gw, gb
    dx = conv3d_dgrad(g, p["enc.conv_in.w"], tape["x"].shape)
    return grads, dx
