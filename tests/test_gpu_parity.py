"""GPU parity: the HIP library through its C ABI against the FP64 oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import tokenizer as O  # noqa: E402
from tests import gpu_common as G  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2602_03529_amd import tok
    return tok


@pytest.fixture(scope="module")
def models(tk):
    m = {}
    for prec in ("f32", "bf16"):
        for ra in (False, True):
            m[(prec, ra)] = tk.TokModel(synth.flatten_weights(G.weights(ra)), prec)
    return m


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# ---------------------------------------------------------------------------
# FSQ and masks
# ---------------------------------------------------------------------------

def test_quantize_matches_oracle(tk):
    rng = np.random.default_rng(0)
    z = rng.normal(0, 2.0, (70001, 6)).astype(np.float32)
    z[:100] = 0.0
    z[100:200] = 50.0
    z[200:300] = -50.0
    codes, idx = tk.quantize(_cuda(z))
    torch.cuda.synchronize()
    rc, ri, rq, rb = O.fsq(z.astype(np.float64))
    mism, agree, band = G.idx_agreement(idx.cpu().numpy(), ri, rb)
    assert mism == 0, (mism, agree, band)
    ok = ~G.in_band(rb)
    np.testing.assert_array_equal(codes.cpu().numpy()[ok], rc[ok].astype(np.float32))


def test_quantize_empty(tk):
    z = torch.empty((0, 6), dtype=torch.float32, device="cuda")
    codes, idx = tk.quantize(z)
    assert codes.numel() == 0 and idx.numel() == 0


@pytest.mark.parametrize("mode,rate,protect", [(1, 0.3, False), (1, 0.0, False), (1, 1.0, False),
                                               (2, 0.4, False), (1, 0.9, True)])
def test_drop_masks_bit_exact(tk, mode, rate, protect):
    N, T2, H2, W2 = 3, 5, 23, 37
    codes = synth.randn(5, (N, T2, H2, W2, 6))
    c = _cuda(codes)
    d = tk.Drop(mode=mode, rate=rate, seed=12345, clip_id0=7, protect_iframe=protect)
    keep = tk.drop(c, d)
    torch.cuda.synchronize()
    ref = O.keep_mask(mode, rate, 12345, [7, 8, 9], T2, H2, W2, protect)
    np.testing.assert_array_equal(keep.cpu().numpy(), ref)
    np.testing.assert_array_equal(c.cpu().numpy(), (codes * ref[..., None]).astype(np.float32))


def test_drop_external_mask(tk):
    N, T2, H2, W2 = 2, 3, 8, 8
    ext = (np.random.default_rng(1).random((N, T2, H2, W2)) > 0.5).astype(np.uint8)
    codes = synth.randn(6, (N, T2, H2, W2, 6))
    c = _cuda(codes)
    keep = tk.drop(c, tk.Drop(mode=3, ext_keep=_cuda(ext)))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(keep.cpu().numpy(), ext)
    np.testing.assert_array_equal(c.cpu().numpy(), (codes * ext[..., None]).astype(np.float32))


# ---------------------------------------------------------------------------
# Encoder / decoder, FP32 path
# ---------------------------------------------------------------------------

SHAPES = [((0,), 9, 64, 64, False),        # the 1x9x64x64 configuration
          ((0, 1), 5, 40, 72, True),       # ragged tiles in h and w, random bias / affine
          ((3,), 1, 16, 132, True),        # single frame, W not a multiple of the 64-wide tile
          ((2,), 13, 24, 24, False),       # more frames, several latent frames
          ((1,), 1, 4, 4, True),           # the smallest frame: one latent position, tiles almost all padding
          ((0,), 5, 4, 8, False)]          # one latent row of two positions


@pytest.mark.parametrize("seeds,T,H,W,ra", SHAPES)
def test_encode_f32_matches_oracle(tk, models, seeds, T, H, W, ra):
    ref = G.oracle_roundtrip(seeds, T, H, W, ra)
    x = _cuda(G.clip(seeds, T, H, W))
    out = models[("f32", ra)].encode(x)
    torch.cuda.synchronize()
    z = out["z"].cpu().numpy()
    zerr = np.abs(z - ref["z"]).max()
    assert zerr <= 1e-4 * max(1.0, np.abs(ref["z"]).max()), zerr
    mism, agree, band = G.idx_agreement(out["idx"].cpu().numpy(), ref["idx"], ref["b"])
    assert mism == 0, (mism, agree, band)
    assert out["keep"].cpu().numpy().all()


@pytest.mark.parametrize("seeds,T,H,W,ra", SHAPES)
def test_decode_f32_matches_oracle_on_identical_codes(tk, models, seeds, T, H, W, ra):
    ref = G.oracle_roundtrip(seeds, T, H, W, ra)
    codes = _cuda(ref["codes"].astype(np.float32))
    xh = models[("f32", ra)].decode(codes)
    torch.cuda.synchronize()
    err = np.abs(xh.cpu().numpy() - ref["xhat"]).max()
    assert err <= G.F32_RECON_TOL, err


def test_encode_with_bernoulli_drop(tk, models):
    seeds, T, H, W = (0, 1), 5, 40, 72
    x = _cuda(G.clip(seeds, T, H, W))
    d = tk.Drop(mode=1, rate=0.3, seed=99, clip_id0=10)
    out = models[("f32", False)].encode(x, drop=d)
    torch.cuda.synchronize()
    T2, H2, W2 = O.latent_shape(T, H, W)
    ref_keep = O.keep_mask(1, 0.3, 99, [10, 11], T2, H2, W2)
    keep = out["keep"].cpu().numpy()
    np.testing.assert_array_equal(keep, ref_keep)
    codes = out["codes"].cpu().numpy()
    assert np.all(codes[keep == 0] == 0.0)
    c2, _ = tk.quantize(out["z"])
    np.testing.assert_array_equal(codes[keep == 1], c2.cpu().numpy()[keep == 1])


# ---------------------------------------------------------------------------
# BF16 path
# ---------------------------------------------------------------------------

def test_bf16_roundtrip_psnr(tk, models):
    seeds, T, H, W = (0,), 9, 64, 64
    ref = G.oracle_roundtrip(seeds, T, H, W, False)
    x = _cuda(G.clip(seeds, T, H, W))
    m = models[("bf16", False)]
    out = m.encode(x)
    xh = m.decode(out["codes"])
    xd = m.decode(_cuda(ref["codes"].astype(np.float32)))
    torch.cuda.synchronize()
    src = O.pixels_to_input(G.clip(seeds, T, H, W))
    p_gpu = O.psnr(xh.cpu().numpy(), src)
    p_ref = O.psnr(ref["xhat"], src)
    assert abs(p_gpu - p_ref) <= 0.5, (p_gpu, p_ref)
    # decode of the oracle's codes: PSNR of the bf16 reconstruction against the
    # oracle's, floor derived from bf16's precision (tests/test_gpu_fullframe.py)
    p_dec = O.psnr(xd.cpu().numpy(), ref["xhat"])
    assert p_dec >= 32.0, p_dec
    _, agree, _ = G.idx_agreement(out["idx"].cpu().numpy(), ref["idx"], ref["b"])
    assert agree > 0.9, agree


# ---------------------------------------------------------------------------
# Structural properties on the GPU path
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_encoder_causality_gpu(tk, models, prec):
    u8 = G.clip((4,), 9, 32, 48)
    m = models[(prec, True)]
    z1 = m.encode(_cuda(u8))["z"].cpu().numpy()
    u2 = u8.copy()
    u2[:, 5] = 255 - u2[:, 5]
    z2 = m.encode(_cuda(u2))["z"].cpu().numpy()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(z1[:, :2], z2[:, :2])
    assert not np.array_equal(z1[:, 2], z2[:, 2])


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_batch_invariance(tk, models, prec):
    """A clip's outputs do not depend on its batch-mates (bit-exact)."""
    u8 = G.clip((0, 1, 2), 5, 32, 40)
    m = models[(prec, False)]
    full = m.encode(_cuda(u8))
    alone = m.encode(_cuda(u8[1:2]))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(full["z"][1:2].cpu().numpy(), alone["z"].cpu().numpy())
    np.testing.assert_array_equal(full["idx"][1:2].cpu().numpy(), alone["idx"].cpu().numpy())
    xf = m.decode(full["codes"])
    xa = m.decode(alone["codes"])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(xf[1:2].cpu().numpy(), xa.cpu().numpy())


def test_repeat_runs_bit_identical(tk, models):
    u8 = G.clip((0,), 9, 64, 64)
    m = models[("bf16", True)]
    a = m.decode(m.encode(_cuda(u8))["codes"]).cpu().numpy()
    b = m.decode(m.encode(_cuda(u8))["codes"]).cpu().numpy()
    np.testing.assert_array_equal(a, b)


def test_shape_errors(tk, models):
    from paper_2602_03529_amd._lib import TokError
    m = models[("f32", False)]
    with pytest.raises(TokError):
        m.encode(torch.zeros((1, 4, 16, 16, 3), dtype=torch.uint8, device="cuda"))
    with pytest.raises(TokError):
        m.encode(torch.zeros((1, 5, 18, 16, 3), dtype=torch.uint8, device="cuda"))


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_chunked_streaming_equals_whole_clip(tk, models, prec):
    """Causal temporal chunking (one latent frame at a time, per-layer frame
    caches) gives bit-identical results to whole-clip processing."""
    seeds, T, H, W = (0, 1), 13, 40, 72
    m = models[(prec, True)]
    x = _cuda(G.clip(seeds, T, H, W))
    d = tk.Drop(mode=1, rate=0.2, seed=5, clip_id0=3)
    ws_whole = torch.empty(m.workspace_size(2, T, H, W), dtype=torch.uint8, device="cuda")
    ws_stream = torch.empty(m.workspace_size(2, T, H, W, stream=True), dtype=torch.uint8, device="cuda")
    assert ws_stream.numel() < ws_whole.numel()
    a = m.encode(x, drop=d, ws=ws_whole)
    b = m.encode(x, drop=d, ws=ws_stream)
    xa = m.decode(a["codes"], ws=ws_whole)
    xb = m.decode(a["codes"], ws=ws_stream)
    torch.cuda.synchronize()
    for k in ("z", "codes", "idx", "keep"):
        np.testing.assert_array_equal(a[k].cpu().numpy(), b[k].cpu().numpy(), err_msg=k)
    np.testing.assert_array_equal(xa.cpu().numpy(), xb.cpu().numpy())
