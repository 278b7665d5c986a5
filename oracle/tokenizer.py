"""FP64 oracle of the stand-in video tokenizer: encode -> FSQ -> token drop -> decode,
the training loss and its hand-written backward.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module.

Paper anchors (arXiv 2602.03529):
  * Sec. 2.4: the encoder f_phi maps a (1+T) x H x W x 3 clip to a
    (1+T') x H' x W' x C latent with spatial factor s_HW and temporal factor
    s_T; the decoder g_theta maps it back.
  * Sec. 1 (challenge C2): the codec's compute is causal residual blocks
    (plus wavelets / attention, which the stand-in does not have).
  * Sec. 4.3: the first frame of a GoP is compressed spatially only and the
    following frames jointly; tokens form an H' x W' matrix per latent frame.
  * Sec. 6.2: dropped tokens and tokens of lost packets (one packet per
    token-matrix row) are zero-filled before decoding.
  * Appendix, Eq. 5 and Eq. 7: L_pixel is the l1 reconstruction loss, and
    the drop-robust loss backpropagates through the zero-filled decoder input
    into the encoder.
The paper fixes neither the layer list nor the quantiser; the readings used
here (layer list, finite scalar quantisation, causal padding, per-frame
GroupNorm, hash-based Bernoulli masks, commitment term) are the stand-in's
definition and are listed with the oracle's other readings in the design
notes.

Layout: every activation is (N, T, H, W, C) float64 ("NDHWC").
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

GN_GROUPS = 32
GN_EPS = 1e-6
FSQ_LEVELS = (8, 8, 8, 5, 5, 5)
FSQ_EPS = 1e-3
COMMIT_WEIGHT = 0.1

# ---------------------------------------------------------------------------
# Elementary operations
# ---------------------------------------------------------------------------


def pixels_to_input(u8):
    """uint8 pixels -> [-1, 1]:  x = u / 127.5 - 1."""
    return np.asarray(u8, np.float64) / 127.5 - 1.0


def _pad_causal(x):
    """Causal pad for a k=3 conv: two copies of frame 0 in front (replicate),
    one zero row/column on each spatial side."""
    x = np.concatenate([x[:, :1], x[:, :1], x], axis=1)
    return np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (0, 0)))


def conv_out_shape(T, H, W, stride):
    st, ss = stride
    assert (T - 1) % st == 0 and H % ss == 0 and W % ss == 0
    return (T - 1) // st + 1, H // ss, W // ss


def conv3d(x, w, b=None, stride=(1, 1)):
    """Causal 3-D convolution.

    y[n,t,h,w,o] = b[o] + sum_{kt,kh,kw,i} W[o,i,kt,kh,kw] * x~[n, s_t t + kt - 2, s_s h + kh - 1, s_s w + kw - 1, i]
    where x~ reads frame 0 for negative time indices and 0 outside the
    spatial range.  A 1x1x1 kernel is a per-position matrix product.
    Evaluated tap by tap: each tap is one matrix product over all output
    positions of one output frame.
    """
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    N, T, H, W_, Ci = x.shape
    Co = w.shape[0]
    assert w.shape[1] == Ci
    if w.shape[2:] == (1, 1, 1):
        assert stride == (1, 1)
        y = x.reshape(-1, Ci) @ np.ascontiguousarray(w[:, :, 0, 0, 0].T)
        if b is not None:
            y = y + np.asarray(b, np.float64)
        return y.reshape(N, T, H, W_, Co)
    st, ss = stride
    To, Ho, Wo = conv_out_shape(T, H, W_, stride)
    xp = _pad_causal(x)
    wt = np.ascontiguousarray(w.transpose(2, 3, 4, 1, 0))  # [kt, kh, kw, Ci, Co]
    y = np.zeros((N, To, Ho, Wo, Co))
    if b is not None:
        y += np.asarray(b, np.float64)
    for n in range(N):
        for t in range(To):
            acc = y[n, t].reshape(-1, Co)
            for kt in range(3):
                frame = xp[n, st * t + kt]
                for kh in range(3):
                    for kw in range(3):
                        sl = frame[kh:kh + ss * (Ho - 1) + 1:ss, kw:kw + ss * (Wo - 1) + 1:ss, :]
                        acc += np.ascontiguousarray(sl).reshape(-1, Ci) @ wt[kt, kh, kw]
    return y


def conv3d_bruteforce(x, w, b=None, stride=(1, 1)):
    """The same causal convolution as seven nested loops (tiny tensors only)."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    N, T, H, W_, Ci = x.shape
    Co, _, KT, KH, KW = w.shape
    st, ss = stride
    if KT == 1:
        To, Ho, Wo = T, H, W_
    else:
        To, Ho, Wo = conv_out_shape(T, H, W_, stride)
    y = np.zeros((N, To, Ho, Wo, Co))
    for n in range(N):
        for t in range(To):
            for h in range(Ho):
                for ww in range(Wo):
                    for o in range(Co):
                        s = 0.0 if b is None else float(b[o])
                        for kt in range(KT):
                            for kh in range(KH):
                                for kw in range(KW):
                                    if KT == 1:
                                        ti, hi, wi = t, h, ww
                                    else:
                                        ti = max(st * t + kt - 2, 0)
                                        hi = ss * h + kh - 1
                                        wi = ss * ww + kw - 1
                                    if hi < 0 or hi >= H or wi < 0 or wi >= W_:
                                        continue
                                    for i in range(Ci):
                                        s += w[o, i, kt, kh, kw] * x[n, ti, hi, wi, i]
                        y[n, t, h, ww, o] = s
    return y


def upsample(x):
    """Nearest x2 in t, h, w with the duplicate of frame 0 dropped:
    U(x)[n,t,h,w,c] = x[n, ceil(t/2), floor(h/2), floor(w/2), c], t in [0, 2T-2]."""
    T = x.shape[1]
    tidx = (np.arange(2 * T - 1) + 1) // 2
    y = x[:, tidx]
    return np.repeat(np.repeat(y, 2, axis=2), 2, axis=3)


def group_norm(x, gamma, beta, groups=GN_GROUPS, eps=GN_EPS):
    """GroupNorm per frame: for each (n, t, g) mean and biased variance over
    h, w and the channels of group g; (x - mu)/sqrt(var + eps) * gamma + beta."""
    N, T, H, W_, C = x.shape
    xg = x.reshape(N, T, H, W_, groups, C // groups)
    mu = xg.mean(axis=(2, 3, 5), keepdims=True)
    var = ((xg - mu) ** 2).mean(axis=(2, 3, 5), keepdims=True)
    xh = ((xg - mu) / np.sqrt(var + eps)).reshape(x.shape)
    return xh * np.asarray(gamma, np.float64) + np.asarray(beta, np.float64)


def silu(x):
    """x * sigmoid(x), evaluated without overflow for large |x|."""
    e = np.exp(-np.abs(x))
    sig = np.where(x >= 0, 1.0 / (1.0 + e), e / (1.0 + e))
    return x * sig


def sigmoid(x):
    e = np.exp(-np.abs(x))
    return np.where(x >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def resblock(x, p, name):
    """Pre-activation residual block with two units:
    x + C_b(SiLU(GN_b(C_a(SiLU(GN_a(x))))))."""
    h = silu(group_norm(x, p[name + ".gn_a.gamma"], p[name + ".gn_a.beta"]))
    h = conv3d(h, p[name + ".a.w"], p[name + ".a.b"])
    h = silu(group_norm(h, p[name + ".gn_b.gamma"], p[name + ".gn_b.beta"]))
    h = conv3d(h, p[name + ".b.w"], p[name + ".b.b"])
    return x + h


# ---------------------------------------------------------------------------
# Encoder / decoder (the stand-in architecture)
# ---------------------------------------------------------------------------


def latent_shape(T, H, W):
    """Latent grid for a (T, H, W) clip: two stride-2 stages, first frame kept."""
    assert (T - 1) % 4 == 0 and H % 4 == 0 and W % 4 == 0
    T1 = (T - 1) // 2 + 1
    T2 = (T1 - 1) // 2 + 1
    return T2, H // 4, W // 4


def encode(u8, p):
    """f_phi: uint8 (N,T,H,W,3) -> pre-quantisation latent z (N,T2,H/4,W/4,6)."""
    x = pixels_to_input(u8)
    h = conv3d(x, p["enc.conv_in.w"], p["enc.conv_in.b"])
    h = resblock(h, p, "enc.rb1")
    h = resblock(h, p, "enc.rb2")
    h = conv3d(h, p["enc.down1.w"], p["enc.down1.b"], stride=(2, 2))
    h = conv3d(h, p["enc.down2.w"], p["enc.down2.b"], stride=(2, 2))
    return conv3d(h, p["enc.proj.w"], p["enc.proj.b"])


def decode(codes, p):
    """g_theta: codes (N,T2,H2,W2,6) -> reconstruction (N,4(T2-1)+1,4H2,4W2,3)."""
    h = conv3d(codes, p["dec.proj_in.w"], p["dec.proj_in.b"])
    h = conv3d(upsample(h), p["dec.up2.w"], p["dec.up2.b"])
    h = conv3d(upsample(h), p["dec.up1.w"], p["dec.up1.b"])
    h = resblock(h, p, "dec.rb1")
    h = resblock(h, p, "dec.rb2")
    return conv3d(h, p["dec.conv_out.w"], p["dec.conv_out.b"])


# ---------------------------------------------------------------------------
# Finite scalar quantisation (Mentzer et al., arXiv:2309.15505; the paper only
# says "tokens", so the quantiser is the stand-in's reading).
# ---------------------------------------------------------------------------


def fsq_constants(levels=FSQ_LEVELS, eps=FSQ_EPS):
    """Per channel: half-range h, offset o, shift s, code half-width d = floor(L/2)."""
    L = np.asarray(levels, np.float64)
    h = (L - 1.0) * (1.0 - eps) / 2.0
    o = np.where(np.asarray(levels) % 2 == 0, 0.5, 0.0)
    s = np.arctanh(o / h)
    d = np.floor(L / 2.0)
    return h, o, s, d


def fsq_basis(levels=FSQ_LEVELS):
    """Mixed-radix place values: beta_c = prod_{j<c} L_j (1, 8, 64, 512, 2560, 12800)."""
    return np.concatenate([[1], np.cumprod(levels)[:-1]]).astype(np.int64)


def fsq_bound(z, levels=FSQ_LEVELS, eps=FSQ_EPS):
    """b = tanh(z + s) * h - o, per channel (last axis)."""
    h, o, s, _ = fsq_constants(levels, eps)
    return np.tanh(np.asarray(z, np.float64) + s) * h - o


def fsq(z, levels=FSQ_LEVELS, eps=FSQ_EPS):
    """Quantise z (..., 6): q = rint(b) (half to even), codes = q / floor(L/2),
    idx = sum_c (q_c + floor(L_c/2)) beta_c.  Returns (codes, idx, q, b)."""
    b = fsq_bound(z, levels, eps)
    q = np.rint(b)
    _, _, _, d = fsq_constants(levels, eps)
    codes = q / d
    idx = ((q + d).astype(np.int64) * fsq_basis(levels)).sum(axis=-1)
    return codes, idx, q, b


def fsq_indices_to_codes(idx, levels=FSQ_LEVELS):
    idx = np.asarray(idx, np.int64)
    _, _, _, d = fsq_constants(levels)
    digits = []
    for c, L in enumerate(levels):
        digits.append((idx // fsq_basis(levels)[c]) % L)
    q = np.stack(digits, axis=-1).astype(np.float64) - d
    return q / d


def fsq_boundary_distance(b):
    """Distance of the bounded value from the nearest rounding boundary
    (k + 1/2): | b - floor(b) - 1/2 |."""
    return np.abs(b - np.floor(b) - 0.5)


# ---------------------------------------------------------------------------
# Token-drop masks (Sec. 6.2: a dropped token and a lost one both become 0).
# ---------------------------------------------------------------------------

U64 = np.uint64
GOLDEN = 0x9E3779B97F4A7C15
DROP_NONE, DROP_BERNOULLI, DROP_ROWS, DROP_EXTERNAL, DROP_SIMILARITY = 0, 1, 2, 3, 4
ROW_SALT = 0x5A5A5A5A00000000


def splitmix64(x):
    """First output of a SplitMix64 generator whose state is x
    (Steele, Lea, Flood, OOPSLA 2014), vectorised over uint64 arrays."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=U64) + U64(GOLDEN)
        z = (z ^ (z >> U64(30))) * U64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> U64(27))) * U64(0x94D049BB133111EB)
        return z ^ (z >> U64(31))


def drop_threshold(rate):
    """Integer threshold on the 24-bit uniform: floor(rate * 2^24), clamped."""
    r = min(max(float(rate), 0.0), 1.0)
    return int(np.floor(r * 16777216.0))


def _hash24(seed, clip_id, key):
    with np.errstate(over="ignore"):
        base = U64(seed) ^ (U64(clip_id) * U64(GOLDEN))
    return splitmix64(base ^ np.asarray(key, dtype=U64)) >> U64(40)


def keep_mask(mode, rate, seed, clip_ids, T2, H2, W2, protect_iframe=False, external=None):
    """keep (N, T2, H2, W2) uint8.

    BERNOULLI: token i = (t' H2 + h') W2 + w' of clip c is dropped when
      splitmix64(seed ^ c*GOLDEN ^ i) >> 40 < floor(rate 2^24).
    ROWS: one draw per token-matrix row (the packet of Sec. 6.2), key
      ROW_SALT | (t' H2 + h'); a dropped row zeroes all W2 tokens.
    EXTERNAL: the given mask.  protect_iframe keeps latent frame 0.
    """
    N = len(clip_ids)
    if mode == DROP_NONE:
        keep = np.ones((N, T2, H2, W2), np.uint8)
    elif mode == DROP_EXTERNAL:
        keep = (np.asarray(external).reshape(N, T2, H2, W2) != 0).astype(np.uint8)
    else:
        thr = drop_threshold(rate)
        keep = np.empty((N, T2, H2, W2), np.uint8)
        for n, c in enumerate(clip_ids):
            if mode == DROP_BERNOULLI:
                i = np.arange(T2 * H2 * W2, dtype=np.uint64)
                u = _hash24(seed, c, i).reshape(T2, H2, W2)
            elif mode == DROP_ROWS:
                r = np.arange(T2 * H2, dtype=np.uint64) | U64(ROW_SALT)
                u = np.repeat(_hash24(seed, c, r).reshape(T2, H2, 1), W2, axis=2)
            else:
                raise ValueError(mode)
            keep[n] = (u >= U64(thr)).astype(np.uint8)
    if protect_iframe:
        keep[:, 0] = 1
    return keep


def similarity_order_key(vp, vi):
    """A key that orders tokens exactly as the cosine similarity of Eq. 3,
    S = vp . vi / (|vp| |vi|) (S = 0 when either norm is 0): sign(dot) *
    dot^2 / (|vp|^2 |vi|^2), an exact rational for the integer vectors
    vp = 4 c_P, vi = 4 c_I (FSQ codes times 4 are integers in [-4, 4])."""
    dot = int(np.dot(vp, vi))
    nn = int(np.dot(vp, vp)) * int(np.dot(vi, vi))
    if nn == 0 or dot == 0:
        return Fraction(0)
    return Fraction(dot * dot, nn) * (1 if dot > 0 else -1)


def similarity_drop_count(rate, n_p):
    """Tokens to drop among n_p P tokens: ceil(rate * n_p), rate clamped to [0, 1]."""
    r = min(max(float(np.float32(rate)), 0.0), 1.0)
    return min(int(math.ceil(r * n_p)), n_p)


def similarity_keep(codes, rate):
    """keep (N, T2, H2, W2) of similarity-based token selection (Sec. 4.3,
    Eq. 3).  Latent frame 0 of a clip is the I-frame token matrix and is
    never dropped; every later latent frame is a P-frame matrix whose token
    at (h', w') is scored by its cosine similarity to the I token at the
    same location.  Per clip, the ceil(rate * N_P) P tokens with the highest
    similarity are dropped (the paper's threshold tau set by the bandwidth
    budget, expressed as a drop count), ties going to the lower token index
    i = (t' H2 + h') W2 + w' first."""
    c = np.asarray(codes, np.float64)
    N, T2, H2, W2, _ = c.shape
    v = np.rint(4.0 * c).astype(np.int64)
    keep = np.ones((N, T2, H2, W2), np.uint8)
    n_p = (T2 - 1) * H2 * W2
    d = similarity_drop_count(rate, n_p)
    for n in range(N):
        scored = []
        for t in range(1, T2):
            for h in range(H2):
                for w in range(W2):
                    scored.append((-similarity_order_key(v[n, t, h, w], v[n, 0, h, w]), (t * H2 + h) * W2 + w))
        scored.sort()
        for _, i in scored[:d]:
            t, rem = divmod(i, H2 * W2)
            keep[n, t, rem // W2, rem % W2] = 0
    return keep


def apply_keep(codes, keep):
    """Zero-fill: codes * keep over all latent channels."""
    return np.asarray(codes, np.float64) * np.asarray(keep, np.float64)[..., None]


def reassemble_rows(rows_received, masks, payloads, T2, H2, W2, C=6):
    """Receiver side of Sec. 6.2 for one clip: packet r = t' H2 + h' carries a
    W2-bit mask and the valid tokens in order; tokens at mask zeros and all
    tokens of rows never received are zero-filled."""
    out = np.zeros((T2, H2, W2, C))
    for r, m, pay in zip(rows_received, masks, payloads):
        t, h = divmod(int(r), H2)
        cols = np.nonzero(np.asarray(m))[0]
        out[t, h, cols] = np.asarray(pay, np.float64).reshape(len(cols), C)
    return out


def roundtrip(u8, p, mode=DROP_NONE, rate=0.0, seed=0, clip_ids=None, protect_iframe=False,
              external=None):
    """encode -> FSQ -> mask -> decode; returns a dict of every stage."""
    N, T, H, W_, _ = np.asarray(u8).shape
    z = encode(u8, p)
    codes, idx, q, b = fsq(z)
    T2, H2, W2 = latent_shape(T, H, W_)
    if clip_ids is None:
        clip_ids = list(range(N))
    keep = keep_mask(mode, rate, seed, clip_ids, T2, H2, W2, protect_iframe, external)
    dec_in = apply_keep(codes, keep)
    xhat = decode(dec_in, p)
    return dict(z=z, b=b, q=q, codes=codes, idx=idx, keep=keep, dec_in=dec_in, xhat=xhat)


def psnr(a, b, peak=2.0):
    """PSNR with peak 2 (the [-1, 1] range), unclamped, MSE over all values."""
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(peak * peak / mse)
