"""Seeded synthetic inputs shared by the FP64 oracle and the HIP library.

This module only draws inputs: pixels, weights, random test tensors and the
serving workload.  It contains none of the tokenizer's arithmetic (no
convolution, normalisation, quantisation or masking), so the oracle and the
GPU path can both consume it without sharing any computation.

The paper gives no tokenizer architecture or data (the codec is built on a
pretrained vision foundation model, Sec. 7), so the inputs are a seeded
stand-in with the shapes of the paper's workloads: 1 + 4k frame clips
(9 / 17 / 33 frames, matching the 9-frame GoP of Sec. 4.3) at 640x360,
960x540, 1280x720 and 1920x1080 (the RSA resolutions of Sec. 5 and the
training resolutions of the appendix).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np

# ---------------------------------------------------------------------------
# Architecture table: the parameter layout of the stand-in tokenizer.
# Each entry is (name, kind, shape).  kind: "conv" weight [Cout, Cin, kt, kh, kw],
# "bias" [Cout], "gamma"/"beta" [C].  The flat FP32 weight blob handed to the
# library is the concatenation of these tensors in this order.
# ---------------------------------------------------------------------------

C_LAT = 6            # latent channels (FSQ dimensions)
C0 = 64              # level-0 width
C1 = 128             # level-1 / level-2 width
GN_GROUPS = 32
FSQ_LEVELS = (8, 8, 8, 5, 5, 5)


def _conv(name, cout, cin, k):
    return [(name + ".w", "conv", (cout, cin, k, k, k)), (name + ".b", "bias", (cout,))]


def _rb(prefix, c):
    out = []
    out += [(prefix + ".gn_a.gamma", "gamma", (c,)), (prefix + ".gn_a.beta", "beta", (c,))]
    out += _conv(prefix + ".a", c, c, 3)
    out += [(prefix + ".gn_b.gamma", "gamma", (c,)), (prefix + ".gn_b.beta", "beta", (c,))]
    out += _conv(prefix + ".b", c, c, 3)
    return out


def param_spec():
    """Canonical parameter order: module order, encoder then decoder."""
    s = []
    s += _conv("enc.conv_in", C0, 3, 3)
    s += _rb("enc.rb1", C0)
    s += _rb("enc.rb2", C0)
    s += _conv("enc.down1", C1, C0, 3)
    s += _conv("enc.down2", C1, C1, 3)
    s += _conv("enc.proj", C_LAT, C1, 1)
    s += _conv("dec.proj_in", C1, C_LAT, 1)
    s += _conv("dec.up2", C1, C1, 3)
    s += _conv("dec.up1", C0, C1, 3)
    s += _rb("dec.rb1", C0)
    s += _rb("dec.rb2", C0)
    s += _conv("dec.conv_out", 3, C0, 3)
    return s


def param_count():
    return int(sum(np.prod(shape) for _, _, shape in param_spec()))


def make_weights(seed: int = 1, random_affine: bool = False):
    """He-normal conv weights (std sqrt(2/fan_in)) drawn in module order from
    default_rng(seed); biases 0, GroupNorm gamma 1 and beta 0.

    random_affine=True additionally draws non-trivial biases and GroupNorm
    affine parameters from a second generator (seed + 1000), so that those
    code paths are exercised; the conv weights are unchanged by it.
    Returns an ordered dict name -> float32 array.
    """
    rng = np.random.default_rng(seed)
    rng2 = np.random.default_rng(seed + 1000)
    out = {}
    for name, kind, shape in param_spec():
        if kind == "conv":
            fan_in = int(np.prod(shape[1:]))
            out[name] = (rng.standard_normal(shape) * np.sqrt(2.0 / fan_in)).astype(np.float32)
        elif kind == "bias":
            out[name] = np.zeros(shape, np.float32)
        elif kind == "gamma":
            out[name] = np.ones(shape, np.float32)
        elif kind == "beta":
            out[name] = np.zeros(shape, np.float32)
    if random_affine:
        for name, kind, shape in param_spec():
            if kind == "bias":
                out[name] = (0.1 * rng2.standard_normal(shape)).astype(np.float32)
            elif kind == "gamma":
                out[name] = (1.0 + 0.2 * rng2.standard_normal(shape)).astype(np.float32)
            elif kind == "beta":
                out[name] = (0.1 * rng2.standard_normal(shape)).astype(np.float32)
    return out


def flatten_weights(w: dict) -> np.ndarray:
    """Concatenate a weight dict into the canonical flat FP32 blob."""
    parts = []
    for name, _, shape in param_spec():
        a = np.asarray(w[name], np.float32)
        assert a.shape == tuple(shape), (name, a.shape, shape)
        parts.append(a.reshape(-1))
    return np.concatenate(parts)


def unflatten_weights(flat: np.ndarray) -> dict:
    out, off = {}, 0
    for name, _, shape in param_spec():
        n = int(np.prod(shape))
        out[name] = np.asarray(flat[off:off + n]).reshape(shape)
        off += n
    assert off == flat.size
    return out


# ---------------------------------------------------------------------------
# Pixels: 8 drifting sinusoids + Gaussian noise, uint8 NDHWC.
# ---------------------------------------------------------------------------

def make_clip(seed: int, T: int, H: int, W: int) -> np.ndarray:
    """uint8 clip of shape (T, H, W, 3).

    For k = 0..7 draw a direction theta_k ~ U[0, 2pi), a spatial frequency
    f_k ~ U[1/64, 1/8] cycles/px and phases phi_{k,c} ~ U[0, 2pi) for c = 0..2;
    v(t,y,x,c) = 1/8 sum_k sin(2 pi f_k (x cos theta_k + y sin theta_k - t) + phi_{k,c})
    (each sinusoid drifts 1 px per frame along its own direction), then
    u = clip(rint(127.5 + 100 v + n), 0, 255) with n ~ N(0, 2^2) i.i.d.
    """
    rng = np.random.default_rng(seed)
    theta = np.empty(8)
    freq = np.empty(8)
    phase = np.empty((8, 3))
    for k in range(8):
        theta[k] = rng.uniform(0.0, 2.0 * np.pi)
        freq[k] = rng.uniform(1.0 / 64.0, 1.0 / 8.0)
        phase[k] = rng.uniform(0.0, 2.0 * np.pi, size=3)
    yy = np.arange(H, dtype=np.float64)[:, None]
    xx = np.arange(W, dtype=np.float64)[None, :]
    out = np.empty((T, H, W, 3), np.uint8)
    for t in range(T):
        v = np.zeros((H, W, 3))
        for k in range(8):
            arg = 2.0 * np.pi * freq[k] * (xx * np.cos(theta[k]) + yy * np.sin(theta[k]) - t)
            for c in range(3):
                v[:, :, c] += np.sin(arg + phase[k, c])
        v /= 8.0
        noise = rng.normal(0.0, 2.0, size=(H, W, 3))
        out[t] = np.clip(np.rint(127.5 + 100.0 * v + noise), 0, 255).astype(np.uint8)
    return out


def make_batch(seeds, T: int, H: int, W: int) -> np.ndarray:
    """uint8 (N, T, H, W, 3); clip i uses seeds[i]."""
    return np.stack([make_clip(s, T, H, W) for s in seeds])


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# ---------------------------------------------------------------------------
# Generic seeded tensors for per-operation tests.
# ---------------------------------------------------------------------------

def randn(seed: int, shape, scale: float = 1.0, dtype=np.float32) -> np.ndarray:
    return (np.random.default_rng(seed).standard_normal(shape) * scale).astype(dtype)


def uniform(seed: int, shape, lo: float, hi: float, dtype=np.float32) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=shape).astype(dtype)


# ---------------------------------------------------------------------------
# Serving workload: Poisson arrivals, mixed resolutions and drop rates.
# ---------------------------------------------------------------------------

SERVE_RESOLUTIONS = ((360, 640), (540, 960), (720, 1280), (1080, 1920))


@dataclass
class Request:
    clip_id: int
    arrival_s: float
    H: int
    W: int
    T: int
    drop_rate: float
    pixel_seed: int


def make_requests(n: int = 256, rate_per_s: float = 40.0, T: int = 17, seed: int = 3,
                  resolutions=SERVE_RESOLUTIONS, max_drop: float = 0.5):
    """n requests with exponential inter-arrival times (Poisson process),
    resolution uniform over `resolutions`, drop fraction ~ U[0, max_drop];
    everything drawn from default_rng(seed) in that order per request."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_per_s)
        H, W = resolutions[int(rng.integers(len(resolutions)))]
        p = float(rng.uniform(0.0, max_drop))
        reqs.append(Request(i, t, H, W, T, p, i))
    return reqs
