"""GPU parity of the coding steps around the tokenizer against the FP64
oracle (oracle/coding.py):

* row packets (Sec. 6.2): the sender's bytes and offsets bit-exact, the
  receiver's codes and keep bit-exact, with lost, reordered and malformed
  packets; at the round-trip benchmark's latent shape (4 x 5 x 180 x 320),
  the stream's packet sizes and the reassembled tensor are checked by what
  holds at any size;
* the pixel-residual layer (Sec. 4.3, Eq. 4): the averaged residual within a
  bound derived from fp32 rounding (below), the same zero pattern except for
  entries whose exact magnitude lies within that bound of theta (either
  decision is correct there), the sparse list exactly the non-zero entries of
  the GPU's own residual in index order; at the benchmark's clip shape
  (4 x 17 x 720 x 1280) on sampled rows;
* GoP-boundary blending (Sec. 4.2, Eq. 2): within 4 ulp-scale units of the
  operands, later frames untouched.

fp32 bound of the residual: each term x_t - xhat_t carries at most three
roundings of relative size 2^-24 of |x_t| + |xhat_t| + 1 (the pixel scaling,
its offset, the difference), the sum of T terms at most T - 1 more of the
running sum and the division one more, so per entry
|r_gpu - r| <= (T + 4) 2^-24 mean_t(|x_t| + |xhat_t| + 1).

Inputs are seeded: FSQ indices uniform over the 64000 codes with Bernoulli
keep masks (p = 0.7); pixels uniform uint8 with reconstructions
x + N(0, 0.05) noise in float32."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import coding as K  # noqa: E402
from oracle import tokenizer as O  # noqa: E402

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


@pytest.fixture(scope="module")
def tk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2602_03529_amd import tok
    return tok


def idx_keep(seed, N, T2, H2, W2, p_keep=0.7):
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, 64000, (N, T2, H2, W2)).astype(np.int32)
    keep = (rng.random((N, T2, H2, W2)) < p_keep).astype(np.uint8)
    return idx, keep


def gpu_packets(tk, idx, keep):
    buf, offs = tk.packetize(torch.from_numpy(idx).cuda(), None if keep is None else torch.from_numpy(keep).cuda())
    torch.cuda.synchronize()
    offs = offs.cpu().numpy().astype(np.int64)
    return buf.cpu().numpy()[:offs[-1]].tobytes(), offs


PK_CASES = [(0, 1, 3, 5, 7), (1, 2, 2, 4, 16), (2, 2, 3, 10, 70), (3, 1, 2, 3, 130), (4, 3, 2, 6, 64), (5, 1, 1, 1, 1)]


@pytest.mark.parametrize("seed,N,T2,H2,W2", PK_CASES)
def test_packets_match_oracle_bytes(tk, seed, N, T2, H2, W2):
    print("case", seed, N, T2, H2, W2, flush=True)
    idx, keep = idx_keep(seed, N, T2, H2, W2)
    keep[0, 0, 0] = 0                      # a row with no valid token
    ref, ref_offs = K.serialize(K.packetize(idx, keep), W2)
    got, offs = gpu_packets(tk, idx, keep)
    assert offs.tolist() == ref_offs
    assert got == ref


def test_packets_without_mask_carry_every_token(tk):
    idx, _ = idx_keep(6, 2, 3, 4, 9)
    ref, ref_offs = K.serialize(K.packetize(idx, np.ones_like(idx, np.uint8)), 9)
    got, offs = gpu_packets(tk, idx, None)
    assert got == ref and offs.tolist() == ref_offs


@pytest.mark.parametrize("seed,N,T2,H2,W2", PK_CASES[:4])
def test_reassembly_matches_oracle_with_loss_reorder_and_garbage(tk, seed, N, T2, H2, W2):
    idx, keep = idx_keep(seed + 10, N, T2, H2, W2)
    ref_buf, ref_offs = K.serialize(K.packetize(idx, keep), W2)
    G = N * T2 * H2
    rng = np.random.default_rng(seed)
    recv = [ref_offs[g] for g in range(G) if rng.random() > 0.25]
    bad = bytearray(ref_buf)
    if G > 1:                              # one packet names a row outside the batch
        bad[ref_offs[1]:ref_offs[1] + 4] = (G + 5).to_bytes(4, "little")
        recv.append(ref_offs[1])
    recv += [len(bad) - 2, len(bad) + 100]  # truncated and out-of-buffer offsets
    rng.shuffle(recv)
    ref_codes, ref_keep = K.reassemble(bytes(bad), recv, N, T2, H2, W2)
    buf = torch.from_numpy(np.frombuffer(bytes(bad), np.uint8).copy()).cuda()
    offs = torch.from_numpy(np.array(recv, np.uint64)).cuda()
    codes, kp = tk.reassemble(buf, offs, (N, T2, H2, W2))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(kp.cpu().numpy(), ref_keep)
    np.testing.assert_array_equal(codes.cpu().numpy(), ref_codes.astype(np.float32))


def test_packets_at_benchmark_latent_shape(tk):
    N, T2, H2, W2 = 4, 5, 180, 320
    idx, keep = idx_keep(31, N, T2, H2, W2)
    got, offs = gpu_packets(tk, idx, keep)
    count = keep.reshape(-1, W2).sum(1)
    sizes = 4 + 4 * (((W2 + 7) // 8 + 3) // 4) + 4 * ((count + 1) // 2)
    np.testing.assert_array_equal(np.diff(offs), sizes)
    assert offs[0] == 0 and offs[-1] == len(got)
    heads = np.frombuffer(got, np.uint8)[offs[:-1, None] + np.arange(4)].astype(np.int64)
    np.testing.assert_array_equal(heads[:, 0] | heads[:, 1] << 8 | heads[:, 2] << 16 | heads[:, 3] << 24,
                                  np.arange(N * T2 * H2))
    buf = torch.from_numpy(np.frombuffer(got, np.uint8).copy()).cuda()
    lost = np.random.default_rng(3).random(N * T2 * H2) < 0.1
    sel = torch.from_numpy(offs[:-1][~lost].astype(np.uint64)).cuda()
    codes, kp = tk.reassemble(buf, sel, (N, T2, H2, W2))
    torch.cuda.synchronize()
    eff = keep * (~lost).reshape(N, T2, H2, 1)
    np.testing.assert_array_equal(kp.cpu().numpy(), eff)
    np.testing.assert_array_equal(codes.cpu().numpy(),
                                  O.apply_keep(O.fsq_indices_to_codes(idx), eff).astype(np.float32))


# ---- pixel residuals ---------------------------------------------------------------

def clip_and_recon(seed, N, T, H, W, noise=0.05):
    rng = np.random.default_rng(seed)
    u8 = rng.integers(0, 256, (N, T, H, W, 3)).astype(np.uint8)
    xhat = (O.pixels_to_input(u8) + rng.normal(0, noise, u8.shape)).astype(np.float32)
    return u8, xhat


def residual_bound(u8, xhat):
    T = u8.shape[1]
    mag = (np.abs(O.pixels_to_input(u8)) + np.abs(xhat.astype(np.float64)) + 1.0).mean(axis=1)
    return (T + 4) * U * mag


def check_residual(u8, xhat, theta, out):
    r_ref, rs_ref, _ = K.residual_compress(u8, xhat, theta)
    tol = residual_bound(u8, xhat)
    r = out["r"].cpu().numpy().astype(np.float64)
    band = np.abs(np.abs(r_ref) - theta) <= tol
    assert ((r != 0) == (rs_ref != 0))[~band].all()
    both = (r != 0) & (rs_ref != 0)
    assert (np.abs(r - r_ref)[both] <= tol[both]).all()
    print("residual: %d entries, %d non-zero, %d in the theta band, max err / bound %.3g" %
          (r.size, int((r != 0).sum()), int(band.sum()),
           float((np.abs(r - r_ref)[both] / tol[both]).max(initial=0))), flush=True)
    return r


def check_sparse_list(r, out, capacity=None):
    N = r.shape[0]
    co = out["clip_offsets"].cpu().numpy().astype(np.int64)
    idx = out["index"].cpu().numpy().astype(np.int64)
    val = out["value"].cpu().numpy()
    cap = idx.size if capacity is None else capacity
    assert co[0] == 0
    for n in range(N):
        flat = r[n].reshape(-1)
        nz = np.nonzero(flat)[0]
        assert co[n + 1] - co[n] == nz.size
        a, b = co[n], min(co[n + 1], cap)
        if b > a:
            np.testing.assert_array_equal(idx[a:b], nz[:b - a])
            np.testing.assert_array_equal(val[a:b], flat[nz[:b - a]].astype(np.float32))


RS_CASES = [(0, 1, 5, 8, 12, 0.02), (1, 2, 9, 36, 64, 0.03), (2, 3, 17, 20, 28, 0.01), (3, 1, 1, 4, 4, 0.0)]


@pytest.mark.parametrize("seed,N,T,H,W,theta", RS_CASES)
def test_residual_matches_oracle(tk, seed, N, T, H, W, theta):
    print("case", seed, N, T, H, W, theta, flush=True)
    u8, xhat = clip_and_recon(seed, N, T, H, W)
    out = tk.residual_compress(torch.from_numpy(u8).cuda(), torch.from_numpy(xhat).cuda(), theta)
    torch.cuda.synchronize()
    r = check_residual(u8, xhat, theta, out)
    check_sparse_list(r, out)


def test_residual_truncated_list_and_extreme_thresholds(tk):
    u8, xhat = clip_and_recon(7, 2, 5, 12, 16)
    x, xh = torch.from_numpy(u8).cuda(), torch.from_numpy(xhat).cuda()
    full = tk.residual_compress(x, xh, 0.02)
    part = tk.residual_compress(x, xh, 0.02, capacity=100)
    none = tk.residual_compress(x, xh, float("inf"))
    torch.cuda.synchronize()
    r = full["r"].cpu().numpy()
    check_sparse_list(r, part, capacity=100)
    assert torch.equal(full["clip_offsets"].cpu(), part["clip_offsets"].cpu())
    assert not none["r"].any() and int(none["clip_offsets"].cpu()[-1]) == 0


def test_residual_apply_matches_oracle(tk):
    rng = np.random.default_rng(8)
    xhat = rng.normal(0, 1, (2, 5, 8, 12, 3)).astype(np.float32)
    r = (rng.normal(0, 0.05, (2, 8, 12, 3)) * (rng.random((2, 8, 12, 3)) < 0.3)).astype(np.float32)
    ref = K.residual_apply(xhat, r)
    got = tk.residual_apply(torch.from_numpy(r).cuda(), torch.from_numpy(xhat).cuda()).cpu().numpy()
    assert (np.abs(got - ref) <= U * np.abs(ref)).all()


def test_residual_at_benchmark_clip_shape_sampled_rows(tk):
    N, T, H, W = 4, 17, 720, 1280
    rng = np.random.default_rng(9)
    u8 = rng.integers(0, 256, (N, T, H, W, 3), dtype=np.uint8)
    xhat = (O.pixels_to_input(u8).astype(np.float32) + rng.normal(0, 0.05, u8.shape).astype(np.float32))
    out = tk.residual_compress(torch.from_numpy(u8).cuda(), torch.from_numpy(xhat).cuda(), 0.03)
    torch.cuda.synchronize()
    r = out["r"].cpu().numpy().astype(np.float64)
    co = out["clip_offsets"].cpu().numpy().astype(np.int64)
    assert (np.diff(co) == (r != 0).reshape(N, -1).sum(1)).all()
    for n, h in zip(rng.integers(0, N, 24), rng.integers(0, H, 24)):
        sub = {"r": torch.from_numpy(r[n:n + 1, h:h + 1].astype(np.float32))}
        check_residual(u8[n:n + 1, :, h:h + 1], xhat[n:n + 1, :, h:h + 1], 0.03, sub)


# ---- GoP blending ------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3])
def test_blend_matches_oracle(tk, n):
    rng = np.random.default_rng(n)
    prev = rng.normal(0, 1, (2, 9, 8, 12, 3)).astype(np.float32)
    cur = rng.normal(0, 1, (2, 5, 8, 12, 3)).astype(np.float32)
    ref = K.gop_blend(prev, cur, n)
    got = tk.gop_blend(torch.from_numpy(prev).cuda(), torch.from_numpy(cur).cuda(), n).cpu().numpy()
    np.testing.assert_array_equal(got[:, n:], cur[:, n:])
    tol = 4 * U * (np.abs(prev[:, -n:]).astype(np.float64) + np.abs(cur[:, :n]))
    assert (np.abs(got[:, :n] - ref[:, :n]) <= tol).all()


def test_coding_errors(tk):
    from paper_2602_03529_amd._lib import TokError
    with pytest.raises(TokError):
        tk.gop_blend(torch.zeros((1, 1, 4, 4, 3), device="cuda"), torch.zeros((1, 5, 4, 4, 3), device="cuda"), 2)
    with pytest.raises(TokError):
        tk.residual_compress(torch.zeros((1, 3, 6, 8, 3), dtype=torch.uint8, device="cuda"),
                             torch.zeros((1, 3, 6, 8, 3), device="cuda"), 0.1)


# ---- blending fused into the decoder's last conv (tok_decode_blend) ------------------

def uniform_codes(seed, N, T2, H2, W2):
    rng = np.random.default_rng(seed)
    levels = np.array([8, 8, 8, 5, 5, 5])
    q = np.floor(rng.uniform(size=(N, T2, H2, W2, 6)) * levels).astype(np.int64) - levels // 2
    return np.ascontiguousarray(q / (levels // 2), np.float32)


@pytest.fixture(scope="module")
def f32_model(tk):
    import synth
    from tests import gpu_common as G
    return tk.TokModel(synth.flatten_weights(G.weights(True)), "f32")


def test_fused_blend_matches_oracle_decode_then_blend(tk, f32_model):
    """FP32 decode of seeded codes with the previous GoP's frames blended in
    C_out's epilogue, against the oracle's decode followed by its blend:
    within the FP32 reconstruction tolerance."""
    from tests import gpu_common as G
    codes = uniform_codes(40, 1, 3, 16, 16)
    rng = np.random.default_rng(41)
    prev = rng.normal(0, 1, (1, 9, 64, 64, 3)).astype(np.float32)
    ref = K.gop_blend(prev, O.decode(codes.astype(np.float64), G.weights64(True)), 2)
    got = f32_model.decode(torch.from_numpy(codes).cuda(), prev=torch.from_numpy(prev).cuda(), blend_n=2)
    got = got.cpu().numpy()
    err = float(np.abs(got - ref).max())
    print("fused blend vs oracle: max-abs %.3g" % err, flush=True)
    assert err <= G.F32_RECON_TOL


@pytest.mark.parametrize("prec,n", [("f32", 2), ("f32", 3), ("bf16", 2), ("fp8", 2)])
def test_fused_blend_equals_decode_then_blend_kernel(tk, prec, n):
    import synth
    from tests import gpu_common as G
    m = tk.TokModel(synth.flatten_weights(G.weights(True)), prec)
    codes = torch.from_numpy(uniform_codes(42, 2, 3, 12, 20)).cuda()
    prev = torch.from_numpy(np.random.default_rng(43).normal(0, 1, (2, 5, 48, 80, 3)).astype(np.float32)).cuda()
    plain = m.decode(codes)
    fused = m.decode(codes, prev=prev, blend_n=n)
    sep = tk.gop_blend(prev, plain.clone(), n)
    torch.cuda.synchronize()
    assert torch.equal(fused[:, n:], plain[:, n:])
    p, f, s = prev[:, -n:].double().abs(), fused[:, :n].double(), sep[:, :n].double()
    assert bool(((f - s).abs() <= 4 * U * (p + plain[:, :n].double().abs())).all())


def test_gop_stream_and_chunked_decode(tk, f32_model):
    codes = [torch.from_numpy(uniform_codes(50 + k, 1, 3, 8, 12)).cuda() for k in range(3)]
    st = tk.GopStream(f32_model, n=2)
    outs = [st.decode(c).clone() for c in codes]
    ws = torch.empty(f32_model.workspace_size(1, 9, 32, 48, stream=True), dtype=torch.uint8, device="cuda")
    for k in range(3):
        plain = f32_model.decode(codes[k])
        if k == 0:
            assert torch.equal(outs[0], plain)
            continue
        prev = outs[k - 1][:, -2:].contiguous()
        whole = f32_model.decode(codes[k], prev=prev, blend_n=2)
        chunked = f32_model.decode(codes[k], prev=prev, blend_n=2, ws=ws)
        torch.cuda.synchronize()
        assert torch.equal(outs[k], whole) and torch.equal(chunked, whole)
        assert torch.equal(whole[:, 2:], plain[:, 2:]) and not torch.equal(whole[:, :1], plain[:, :1])


def test_fused_blend_errors(tk, f32_model):
    from paper_2602_03529_amd._lib import TokError
    codes = torch.from_numpy(uniform_codes(60, 1, 2, 4, 4)).cuda()
    with pytest.raises(TokError):
        f32_model.decode(codes, prev=torch.zeros((1, 1, 16, 16, 3), device="cuda"), blend_n=2)
    with pytest.raises(TokError):
        f32_model.decode(codes, prev=torch.zeros((1, 9, 16, 16, 3), device="cuda"), blend_n=6)


@pytest.mark.parametrize("prec", ["f32", "bf16", "fp8"])
def test_fused_residual_equals_decode_then_residual(tk, prec):
    """decode_residual equals decode followed by residual_compress bit for
    bit: x_hat, the thresholded mean r, the clip offsets and the sparse list.
    bf16: the residual sums are formed by the decoder's last conv as it writes
    each frame (Sec. 4.3 Eq. 4), also when the decode runs in temporal chunks
    (the sums carried from chunk to chunk); f32 / fp8 run decode then the
    separate pass."""
    import synth
    from tests import gpu_common as G
    m = tk.TokModel(synth.flatten_weights(G.weights(True)), prec)
    N, T2, H2, W2 = 2, 3, 12, 20
    T, H, W = 4 * (T2 - 1) + 1, 4 * H2, 4 * W2
    codes = torch.from_numpy(uniform_codes(70, N, T2, H2, W2)).cuda()
    x = torch.from_numpy(np.random.default_rng(71).integers(0, 256, (N, T, H, W, 3), dtype=np.uint8)).cuda()
    theta = 0.05
    plain = m.decode(codes)
    ref = tk.residual_compress(x, plain, theta)
    runs = [None]
    if prec != "fp8":
        runs.append(torch.empty(m.workspace_size(N, T, H, W, stream=True), dtype=torch.uint8, device="cuda"))
    for ws in runs:
        got = m.decode_residual(codes, x, theta, ws=ws)
        torch.cuda.synchronize()
        assert torch.equal(got["xhat"], plain)
        assert torch.equal(got["r"], ref["r"])
        assert torch.equal(got["clip_offsets"], ref["clip_offsets"])
        total = int(ref["clip_offsets"][-1].item())
        assert 0 < total < N * H * W * 3
        assert torch.equal(got["index"][:total], ref["index"][:total])
        assert torch.equal(got["value"][:total], ref["value"][:total])


@pytest.mark.parametrize("prec", ["bf16", "f32"])
def test_fused_blend_chunked_equals_whole_clip(tk, prec):
    """A blended decode run in temporal chunks (one latent frame at a time:
    blended frame 1 is written by the second chunk) equals the whole-clip
    blended decode bit for bit."""
    import synth
    from tests import gpu_common as G
    m = tk.TokModel(synth.flatten_weights(G.weights(True)), prec)
    N, T2, H2, W2 = 2, 3, 10, 20
    T, H, W = 4 * (T2 - 1) + 1, 4 * H2, 4 * W2
    codes = torch.from_numpy(uniform_codes(80, N, T2, H2, W2)).cuda()
    prev = torch.from_numpy(np.random.default_rng(81).normal(0, 1, (N, 3, H, W, 3)).astype(np.float32)).cuda()
    ws = torch.empty(m.workspace_size(N, T, H, W, stream=True), dtype=torch.uint8, device="cuda")
    whole = m.decode(codes, prev=prev, blend_n=3)
    chunked = m.decode(codes, prev=prev, blend_n=3, ws=ws)
    plain = m.decode(codes)
    torch.cuda.synchronize()
    assert torch.equal(whole, chunked)
    assert torch.equal(whole[:, 3:], plain[:, 3:]) and not torch.equal(whole[:, 1:3], plain[:, 1:3])
