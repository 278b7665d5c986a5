"""FP64 oracle of the token-level and pixel-level coding steps around the
tokenizer: row packets and their reassembly, the pixel-residual layer and
GoP-boundary blending.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module.

Paper anchors (arXiv 2602.03529):
  * Sec. 6.2 (intelligent packetization): an H x W token matrix is sent as H
    packets, one per row; a packet's header holds the row's index and a
    W-bit position mask (1 = valid token, 0 = proactively dropped), its
    payload the valid tokens.  The receiver puts each valid token back at
    its column, zero-fills masked positions and every token of a row whose
    packet never arrived.
  * Sec. 4.3, Eq. 4 (pixel residuals): r = x - x_hat; the residuals of a
    temporal window of T frames are averaged per (h, w, c); entries with
    magnitude below a threshold theta are set to zero, leaving a sparse
    matrix (its entropy coding is out of scope); the receiver adds the
    averaged residual back to every frame of the window.
  * Sec. 4.2, Eq. 2 (GoP-boundary blending): frame i = 1..n of the current
    GoP's reconstruction becomes alpha_i * (frame T-n+i of the previous
    GoP's reconstruction) + (1 - alpha_i) * (frame i of the current one),
    with alpha_i = (n - i) / n.

The paper fixes no byte format for packets.  The stand-in's wire format
(little-endian, every field 4-byte aligned), for the token matrices of a
batch of N clips whose rows are numbered g = (n T2 + t') H2 + h' (for one
clip, the row of its token matrices):

    u32  g
    u8   mask[ceil(W2 / 8)]    bit w & 7 of byte w >> 3 is column w's keep bit
    u8   0 ...                 up to a multiple of 4 bytes
    u16  idx[count]            FSQ code index of each valid token, by column
    u16  0                     if count is odd

Packets follow each other in row order with no gaps.
"""
from __future__ import annotations

import numpy as np

from .tokenizer import fsq_indices_to_codes, pixels_to_input

# ---------------------------------------------------------------------------
# Sec. 6.2: row packets
# ---------------------------------------------------------------------------


def mask_bytes(W2):
    """Bytes of the mask field, padding included: 4 * ceil(ceil(W2 / 8) / 4)."""
    return 4 * (((W2 + 7) // 8 + 3) // 4)


def packet_bytes(W2, count):
    """Size of one packet carrying `count` valid tokens."""
    return 4 + mask_bytes(W2) + 4 * ((count + 1) // 2)


def packetize(idx, keep):
    """Packets of every token-matrix row of a batch, as a list of
    (g, mask, payload): mask the row's W2 keep bits, payload the FSQ indices
    of its valid tokens in column order.  idx, keep: (N, T2, H2, W2)."""
    idx = np.asarray(idx, np.int64)
    keep = np.asarray(keep)
    N, T2, H2, W2 = idx.shape
    packets = []
    for n in range(N):
        for t in range(T2):
            for h in range(H2):
                g = (n * T2 + t) * H2 + h
                m = [int(keep[n, t, h, w] != 0) for w in range(W2)]
                pay = [int(idx[n, t, h, w]) for w in range(W2) if m[w]]
                packets.append((g, m, pay))
    return packets


def serialize(packets, W2):
    """The packets' bytes in the wire format above and the byte offset of each
    packet (plus the total as a last entry)."""
    out = bytearray()
    offsets = []
    for g, m, pay in packets:
        offsets.append(len(out))
        out += int(g).to_bytes(4, "little")
        field = bytearray(mask_bytes(W2))
        for w, bit in enumerate(m):
            if bit:
                field[w >> 3] |= 1 << (w & 7)
        out += field
        for v in pay:
            out += int(v).to_bytes(2, "little")
        if len(pay) % 2:
            out += b"\x00\x00"
    offsets.append(len(out))
    return bytes(out), offsets


def parse_packet(buf, offset, W2):
    """(g, mask, payload) of the packet at `offset`, or None if it does not
    fit inside buf."""
    head = offset + 4 + mask_bytes(W2)
    if offset < 0 or head > len(buf):
        return None
    g = int.from_bytes(buf[offset:offset + 4], "little")
    m = [(buf[offset + 4 + (w >> 3)] >> (w & 7)) & 1 for w in range(W2)]
    count = sum(m)
    if offset + packet_bytes(W2, count) > len(buf):
        return None
    pay = [int.from_bytes(buf[head + 2 * k:head + 2 * k + 2], "little") for k in range(count)]
    return g, m, pay


def reassemble(buf, offsets, N, T2, H2, W2):
    """Receiver: codes (N, T2, H2, W2, 6) and keep (N, T2, H2, W2) from the
    packets found at `offsets` (the ones that arrived, in any order).  Every
    token starts as the zero code vector with keep 0; a packet whose row
    number is out of range or which does not fit inside buf is ignored."""
    codes = np.zeros((N, T2, H2, W2, 6))
    keep = np.zeros((N, T2, H2, W2), np.uint8)
    for off in offsets:
        p = parse_packet(buf, int(off), W2)
        if p is None:
            continue
        g, m, pay = p
        if g >= N * T2 * H2:
            continue
        nt, h = divmod(g, H2)
        n, t = divmod(nt, T2)
        k = 0
        for w in range(W2):
            if m[w]:
                codes[n, t, h, w] = fsq_indices_to_codes(pay[k])
                keep[n, t, h, w] = 1
                k += 1
    return codes, keep


# ---------------------------------------------------------------------------
# Sec. 4.3, Eq. 4: pixel residuals
# ---------------------------------------------------------------------------


def residual_compress(u8, xhat, theta):
    """Sender side of the residual layer for clips u8 (N, T, H, W, 3) uint8
    with reconstructions xhat (N, T, H, W, 3), the window being the clip's T
    frames.  Returns r_comp (N, H, W, 3) = (1/T) sum_t (x_t - xhat_t) with
    x the clip scaled to [-1, 1], r_sparse = r_comp with every entry of
    magnitude below theta set to 0, and per clip the sparse list
    (flat index (h W + w) 3 + c, value) of r_sparse's non-zero entries in
    increasing index order."""
    x = pixels_to_input(u8)
    xh = np.asarray(xhat, np.float64)
    N, T = x.shape[:2]
    r_comp = np.zeros(x.shape[:1] + x.shape[2:])
    for t in range(T):
        r_comp += x[:, t] - xh[:, t]
    r_comp /= T
    r_sparse = np.where(np.abs(r_comp) < theta, 0.0, r_comp)
    lists = []
    for n in range(N):
        flat = r_sparse[n].reshape(-1)
        nz = np.nonzero(flat)[0]
        lists.append((nz.astype(np.int64), flat[nz]))
    return r_comp, r_sparse, lists


def residual_apply(xhat, r_sparse):
    """Receiver side: the window's averaged residual added to every frame,
    xhat (N, T, H, W, 3) + r_sparse (N, H, W, 3)."""
    return np.asarray(xhat, np.float64) + np.asarray(r_sparse, np.float64)[:, None]


# ---------------------------------------------------------------------------
# Sec. 4.2, Eq. 2: GoP-boundary blending
# ---------------------------------------------------------------------------


def blend_weights(n):
    """alpha_i = (n - i) / n for i = 1..n."""
    return [(n - i) / n for i in range(1, n + 1)]


def gop_blend(xhat_prev, xhat_curr, n=2):
    """The current GoP's reconstruction (N, T, H, W, 3) with its first n
    frames blended with the last n of the previous GoP's: frame i (1-based)
    becomes alpha_i prev[T_prev - n + i] + (1 - alpha_i) curr[i]; frames
    after n are unchanged."""
    prev = np.asarray(xhat_prev, np.float64)
    out = np.array(xhat_curr, np.float64)
    Tp = prev.shape[1]
    for i, a in enumerate(blend_weights(n), start=1):
        out[:, i - 1] = a * prev[:, Tp - n + i - 1] + (1.0 - a) * out[:, i - 1]
    return out
