"""GPU parity of similarity-based token selection (Sec. 4.3, Eq. 3).

The keep mask and the zero-filled codes must equal the oracle's exact
rational selection bit for bit, at sizes that span several workgroup tiles
with ragged tails, for rates that drop none, some and all P tokens.  At the
round-trip benchmark's latent shape (4 clips x 5 x 180 x 320), where the
oracle's per-token Fractions are slow, the selection is checked by what
holds at any size: exactly D drops per clip, the I frame kept, every dropped
token at least as similar as every kept one, and among equal similarities the
dropped tokens are the lowest indices.  Those checks use sign(dot) dot^2 / nn
in float64, which orders exactly: division is correctly rounded, so equal
rationals give equal doubles, and two different ones (denominators <= 96^2)
differ by far more than a rounding error.

Inputs: seeded FSQ-valid codes with the structure of temporally redundant
video latents: P tokens that repeat the I token at their location (ties at
S = 1), negated copies (S = -1), zero tokens (S = 0, also zero I tokens),
scaled copies (equal cosines from different integer vectors) and uniformly
drawn codes."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import tokenizer as O  # noqa: E402

pytestmark = pytest.mark.gpu

LEVELS = np.array([8, 8, 8, 5, 5, 5])
HALF = LEVELS // 2


@pytest.fixture(scope="module")
def tk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2602_03529_amd import tok
    return tok


def redundant_codes(seed, N, T2, H2, W2):
    rng = np.random.default_rng(seed)
    q = np.floor(rng.uniform(size=(N, T2, H2, W2, 6)) * LEVELS).astype(np.int64) - HALF
    c = q / HALF
    cat = rng.choice(5, size=(N, T2, H2, W2), p=[0.35, 0.05, 0.05, 0.05, 0.5])
    cat[:, 0] = 4                                                      # the I frame itself is drawn
    i_frame = np.broadcast_to(c[:, :1], c.shape)
    c = np.where((cat == 0)[..., None], i_frame, c)                    # copy of the I token
    c = np.where((cat == 1)[..., None], -i_frame, c)                   # negated copy
    c = np.where((cat == 2)[..., None], 0.0, c)                        # zero token
    half_i = np.trunc(i_frame * 2.0) / 2.0                             # a coarser copy: 4c even
    c = np.where((cat == 3)[..., None], half_i, c)
    c[:, 0][rng.uniform(size=(N, H2, W2)) < 0.05] = 0.0                # a few zero I tokens
    return np.ascontiguousarray(c, np.float32)


def exact_keys(codes):
    v = np.rint(4.0 * codes.astype(np.float64)).astype(np.int64)
    vi = v[:, :1]
    dot = (v * vi).sum(-1)
    nn = (v * v).sum(-1) * (vi * vi).sum(-1)
    key = np.where(nn > 0, np.sign(dot) * (dot * dot).astype(np.float64) / np.maximum(nn, 1), 0.0)
    return key[:, 1:].reshape(codes.shape[0], -1)  # (N, NP), P token j has index j + H2 W2


def check_selection_properties(codes, keep, rate):
    N, T2, H2, W2, _ = codes.shape
    n_p = (T2 - 1) * H2 * W2
    d = O.similarity_drop_count(rate, n_p)
    assert (keep[:, 0] == 1).all()
    keys = exact_keys(codes)
    kp = keep[:, 1:].reshape(N, -1)
    for n in range(N):
        dropped = kp[n] == 0
        assert int(dropped.sum()) == d
        if 0 < d < n_p:
            kstar = keys[n][dropped].min()
            assert keys[n][~dropped].max() <= kstar
            tie = keys[n] == kstar
            idx = np.arange(n_p)
            assert idx[tie & dropped].max() < idx[tie & ~dropped].min(initial=n_p)


def gpu_select(tk, codes_np, rate, keep=True):
    c = torch.from_numpy(codes_np).cuda()
    kp = tk.select_similar(c, rate, keep=keep)
    torch.cuda.synchronize()
    return c.cpu().numpy(), None if kp is None else kp.cpu().numpy()


CASES = [
    (0, 2, 3, 4, 5, 0.3),       # tiny: one tile
    (1, 2, 5, 36, 40, 0.25),    # 5760 P tokens per clip: 3 histogram tiles, ragged tail
    (2, 3, 9, 16, 24, 0.5),
    (3, 1, 2, 45, 80, 0.999),   # one P frame, nearly all dropped
    (4, 2, 4, 12, 20, 0.0),     # nothing dropped
    (5, 2, 4, 12, 20, 1.0),     # every P token dropped
    (6, 2, 1, 8, 8, 0.5),       # I frame only: nothing to drop
    (7, 1, 3, 1, 1, 0.5),       # one token per frame
    (8, 4, 3, 20, 28, 1e-4),    # a single drop per clip
]


@pytest.mark.parametrize("seed,N,T2,H2,W2,rate", CASES)
def test_selection_matches_oracle(tk, seed, N, T2, H2, W2, rate):
    print("case", seed, N, T2, H2, W2, rate, flush=True)
    codes = redundant_codes(seed, N, T2, H2, W2)
    ref_keep = O.similarity_keep(codes, rate)
    out, keep = gpu_select(tk, codes, rate)
    np.testing.assert_array_equal(keep, ref_keep)
    np.testing.assert_array_equal(out, O.apply_keep(codes, ref_keep).astype(np.float32))


def test_uniform_codes_and_clamped_rates(tk):
    rng = np.random.default_rng(9)
    q = np.floor(rng.uniform(size=(2, 3, 10, 14, 6)) * LEVELS).astype(np.int64) - HALF
    codes = np.ascontiguousarray(q / HALF, np.float32)
    for rate in (-0.5, float("nan"), 0.37, 2.0):
        out, keep = gpu_select(tk, codes, rate)
        ref = O.similarity_keep(codes, 0.0 if rate != rate else rate)
        np.testing.assert_array_equal(keep, ref)
        np.testing.assert_array_equal(out, O.apply_keep(codes, ref).astype(np.float32))


def test_clips_are_independent_and_keep_is_optional(tk):
    codes = redundant_codes(11, 3, 5, 12, 16)
    out, keep = gpu_select(tk, codes, 0.4)
    for n in range(3):
        o1, k1 = gpu_select(tk, np.ascontiguousarray(codes[n:n + 1]), 0.4)
        np.testing.assert_array_equal(k1[0], keep[n])
        np.testing.assert_array_equal(o1[0], out[n])
    o2, k2 = gpu_select(tk, codes, 0.4, keep=False)
    assert k2 is None
    np.testing.assert_array_equal(o2, out)


def test_selection_at_benchmark_latent_shape(tk):
    """4 clips x 17 frames x 1280x720 -> latents (5, 180, 320)."""
    codes = redundant_codes(21, 4, 5, 180, 320)
    for rate in (0.3, 0.05):
        out, keep = gpu_select(tk, codes, rate)
        check_selection_properties(codes, keep, rate)
        np.testing.assert_array_equal(out, codes * keep[..., None].astype(np.float32))


def test_encode_with_similarity_equals_encode_then_select(tk):
    import synth
    from paper_2602_03529_amd.tok import Drop, TokModel
    from tests import gpu_common as G
    m = TokModel(synth.flatten_weights(G.weights(True)), "f32")
    x = torch.from_numpy(G.clip((0, 1), 9, 48, 64)).cuda()
    a = m.encode(x, Drop(mode=4, rate=0.35))
    b = m.encode(x)
    kb = tk.select_similar(b["codes"], 0.35)
    torch.cuda.synchronize()
    assert torch.equal(a["keep"], kb) and torch.equal(a["codes"], b["codes"])
    assert torch.equal(a["idx"], b["idx"]) and torch.equal(a["z"], b["z"])
    # streamed (one latent frame per chunk) encode selects after the last chunk
    ws = torch.empty(m.workspace_size(2, 9, 48, 64, what=1, stream=True), dtype=torch.uint8, device="cuda")
    c = m.encode(x, Drop(mode=4, rate=0.35), ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(c["keep"], kb) and torch.equal(c["codes"], b["codes"])


def test_selection_errors(tk):
    from paper_2602_03529_amd import _lib as L
    lib = L.lib()
    codes = torch.zeros((1, 3, 4, 4, 6), dtype=torch.float32, device="cuda")
    d = L.DropDesc(4, 0.5, 0, 0, 0, None)
    assert lib.tok_drop(C.byref(d), C.c_void_p(codes.data_ptr()), None, 1, 3, 4, 4, None) == -1
    need = tk.select_workspace_size(1, 3, 4, 4)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    assert lib.tok_select_similar(C.c_float(0.5), C.c_void_p(codes.data_ptr()), None, 1, 3, 4, 4,
                                  C.c_void_p(ws.data_ptr()), need - 1, None) == -7
    assert lib.tok_select_similar(C.c_float(0.5), None, None, 1, 3, 4, 4, C.c_void_p(ws.data_ptr()), need,
                                  None) == -1
    assert lib.tok_select_similar(C.c_float(0.5), C.c_void_p(codes.data_ptr()), None, 0, 3, 4, 4,
                                  C.c_void_p(ws.data_ptr()), need, None) == -2
    torch.cuda.synchronize()
