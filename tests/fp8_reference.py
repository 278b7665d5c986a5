"""FP64 model of the fp8 decoder's operand rounding (test infrastructure).

The oracle computes the decoder exactly; the fp8 decoder rounds its conv
operands by a stated rule.  This module applies that rule to the oracle's
definitions and computes everything else in float64, so the GPU's fp8 decode
can be compared with it element by element: what remains between the two is
the GPU's fp32 accumulation and transcendental rounding, and the quantisation
decisions those tiny differences flip.  The rule:

  weights      per output channel c: scale_c = max |w_c| / 448 (fp32), each
               weight becomes e4m3(w * fp32(1 / scale_c)) * scale_c; for the
               upsampling convs the weights are first folded into their
               polyphase form (per output parity the 3 taps of each
               dimension sum into 2, fp32 sums in kt, kh, kw order) and the
               scale covers the folded weights;
  activations  conv inputs in MX-FP8: per position and block of 32 channels
               the smallest power of two 2^e with max |v| 2^-e <= 448 (e from
               the fp32 product max |v| * fp32(1/448)), each value
               e4m3(v 2^-e) 2^e;
  e4m3         OCP E4M3 (bias 7, 3 mantissa bits, subnormals, max 448),
               round to nearest even;
  bf16 stores  the residual stream between convs (up1's output, the first
               residual block's convs, the second block's first conv) in
               bf16, round to nearest even from the fp32 value.

Nothing here is shared with the library; the oracle's conv, upsample,
GroupNorm and SiLU are reused as they are."""
from __future__ import annotations

import numpy as np
import torch

from oracle import tokenizer as O

F32 = np.float32
_INV448 = F32(1.0) / F32(448.0)


def e4m3(x):
    """Round float64 values (already scaled into [-448, 448]) to the nearest
    OCP E4M3 value, ties to even."""
    x = np.asarray(x, np.float64)
    a = np.abs(x)
    _, ex = np.frexp(np.where(a > 0, a, 1.0))
    E = np.maximum(ex - 1, -6)            # binade exponent; below 2^-6 the subnormal quantum stays 2^-9
    q = np.ldexp(1.0, E - 3)
    v = np.minimum(np.round(a / q) * q, 448.0)   # np.round: half to even
    return np.where(a > 0, np.copysign(v, x), 0.0)


def bf16(x):
    """fp32 -> bf16 (round to nearest even) -> float64."""
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(x, F32)))
    return t.to(torch.bfloat16).to(torch.float64).numpy()


def block_exp(am):
    """Exponent of the smallest power of two bringing max |v| to <= 448, as the
    fp32 bits of max |v| * fp32(1/448) give it (0 for an all-zero block)."""
    am = np.asarray(am, F32)
    p = (am * _INV448).astype(F32)
    b = p.view(np.uint32).astype(np.int64)
    e = ((b >> 23) & 255) - 127 + ((b & 0x7FFFFF) != 0)
    return np.where(am > 0, np.clip(e, -127, 127), 0)


def quantize_mx(v):
    """MX-FP8 of fp32 values (..., C), C a multiple of 32; returns the
    represented values in float64."""
    v = np.asarray(v, F32)
    sh = v.shape
    vb = v.reshape(sh[:-1] + (sh[-1] // 32, 32))
    e = block_exp(np.abs(vb).max(axis=-1))
    s = np.ldexp(1.0, -e)[..., None]
    return (e4m3(vb.astype(np.float64) * s) / s).reshape(sh)


def _channel_quant(vals, axis_c=0):
    """Per-output-channel e4m3 weights: vals float32 with the output channel on
    axis 0; returns float64 represented values."""
    vals = np.asarray(vals, F32)
    am = np.abs(vals).reshape(vals.shape[0], -1).max(axis=1)
    scale = np.where(am > 0, (am / F32(448.0)).astype(F32), F32(1.0)).astype(F32)
    inv = (F32(1.0) / scale).astype(F32)
    shp = (-1,) + (1,) * (vals.ndim - 1)
    q = e4m3((vals * inv.reshape(shp)).astype(F32))
    return q * scale.astype(np.float64).reshape(shp)


# fold ranges of the 3 taps onto the 2 source positions d of output parity p
_LO = {(0, 0): 0, (0, 1): 1, (1, 0): 0, (1, 1): 2}
_HI = {(0, 0): 0, (0, 1): 2, (1, 0): 1, (1, 1): 2}
_KEYS = [(pt, ph, pw, dt, dh, dw) for pt in (0, 1) for ph in (0, 1) for pw in (0, 1)
         for dt in (0, 1) for dh in (0, 1) for dw in (0, 1)]


def fold_up(w, dtype=F32):
    """Polyphase weights of nearest-x2 upsample + causal 3x3x3 conv: for
    output parities (pt, ph, pw) and source offsets (dt, dh, dw) the sum of
    the taps that read that source position, accumulated in `dtype` in
    kt, kh, kw order.  Returns an array (2,2,2,2,2,2,Co,Ci)."""
    w = np.asarray(w, dtype)
    Co, Ci = w.shape[:2]
    out = np.zeros((2,) * 6 + (Co, Ci), dtype)
    for k in _KEYS:
        pt, ph, pw, dt, dh, dw = k
        v = np.zeros((Co, Ci), dtype)
        for kt in range(_LO[pt, dt], _HI[pt, dt] + 1):
            for kh in range(_LO[ph, dh], _HI[ph, dh] + 1):
                for kw in range(_LO[pw, dw], _HI[pw, dw] + 1):
                    v = (v + w[:, :, kt, kh, kw]).astype(dtype)
        out[k] = v
    return out


def upconv_poly(x, wf, b):
    """Upsample x2 (time map t -> ceil(t/2)) then causal 3x3x3 conv, evaluated
    in polyphase form from folded weights wf (2,2,2,2,2,2,Co,Ci), float64."""
    x = np.asarray(x, np.float64)
    N, Ts, Hs, Ws, Ci = x.shape
    Co = wf.shape[-2]
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (0, 0)))
    To = 2 * Ts - 1
    out = np.empty((N, To, 2 * Hs, 2 * Ws, Co))
    bias = np.zeros(Co) if b is None else np.asarray(b, np.float64)
    for t in range(To):
        j, pt = t // 2, t % 2
        src = [(j + dt) if pt else max(j - 1 + dt, 0) for dt in (0, 1)]
        for ph in (0, 1):
            for pw in (0, 1):
                acc = np.broadcast_to(bias, (N, Hs, Ws, Co)).copy()
                for dt in (0, 1):
                    for dh in (0, 1):
                        for dw in (0, 1):
                            sl = xp[:, src[dt], dh + ph:dh + ph + Hs, dw + pw:dw + pw + Ws, :]
                            acc += sl.reshape(-1, Ci) .dot(np.asarray(wf[pt, ph, pw, dt, dh, dw], np.float64).T
                                                          ).reshape(N, Hs, Ws, Co)
                out[:, t, ph::2, pw::2, :] = acc
    return out


def quant_s1(w):
    return _channel_quant(w)


def quant_up(w):
    f = fold_up(w)
    # the scale of output channel c covers every folded weight of c
    ff = np.moveaxis(f, 6, 0)                      # (Co, 2,2,2,2,2,2, Ci)
    q = _channel_quant(ff)
    return np.moveaxis(q, 0, 6)


def _proj_in_f32(codes, w, b):
    """1x1 6 -> 128 as an fp32 fused multiply-add chain from the bias."""
    c = np.asarray(codes, F32)
    w = np.asarray(w, F32)[:, :, 0, 0, 0]
    a = np.broadcast_to(np.asarray(b, F32), c.shape[:-1] + (w.shape[0],)).astype(F32)
    for k in range(6):
        a = (a.astype(np.float64) + c[..., k:k + 1].astype(np.float64) * w[:, k].astype(np.float64)).astype(F32)
    return a


def decode_fp8(codes, p, noise=None):
    """The fp8 decoder's arithmetic on codes (N,T2,H2,W2,6) with parameters p
    (float32 dict).  noise: optional (rng, rel) perturbing every conv sum by a
    relative uniform error of at most rel before it is rounded (a model of
    fp32 accumulation-order differences)."""
    def acc(v):
        if noise is None:
            return v
        rng, rel = noise
        return v * (1.0 + rel * rng.uniform(-1.0, 1.0, v.shape))

    def f32(v):
        return np.asarray(v, np.float64).astype(F32)

    def s1(x, name, resid=None):
        y = acc(O.conv3d(x, quant_s1(p[name + ".w"]), None)) + np.asarray(p[name + ".b"], np.float64)
        return y if resid is None else y + resid

    def gn_silu(x, name):
        g = O.group_norm(x, np.asarray(p[name + ".gamma"], np.float64), np.asarray(p[name + ".beta"], np.float64))
        return quantize_mx(f32(acc(O.silu(g))))

    P = quantize_mx(_proj_in_f32(codes, p["dec.proj_in.w"], p["dec.proj_in.b"]))
    U2 = quantize_mx(f32(acc(upconv_poly(P, quant_up(p["dec.up2.w"]), None)) +
                         np.asarray(p["dec.up2.b"], np.float64)))
    A = bf16(f32(acc(upconv_poly(U2, quant_up(p["dec.up1.w"]), None)) + np.asarray(p["dec.up1.b"], np.float64)))
    # residual block 1: bf16 stream
    C = bf16(f32(s1(gn_silu(A, "dec.rb1.gn_a"), "dec.rb1.a")))
    A = bf16(f32(s1(gn_silu(C, "dec.rb1.gn_b"), "dec.rb1.b", A)))
    # residual block 2: its output feeds conv_out in MX-FP8
    C = bf16(f32(s1(gn_silu(A, "dec.rb2.gn_a"), "dec.rb2.a")))
    Cq = quantize_mx(f32(s1(gn_silu(C, "dec.rb2.gn_b"), "dec.rb2.b", A)))
    return s1(Cq, "dec.conv_out")
