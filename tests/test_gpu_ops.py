"""GPU parity of the per-operation entry points (tok_op_*) and of the
backward pass for gradients from outside the library (tok_backward_outputs),
through the C ABI, against the FP64 oracle's definitions and adjoints
(oracle/tokenizer.py, oracle/backward.py; the adjoints are pinned by
dot-product tests, torch autograd and finite differences on the CPU).

Inputs are drawn in float32 and rounded to the operation's storage precision
first, so both sides see identical operand values.  Bars:
  fp32: relative L2 error 1e-5 (convolutions, GroupNorm forward, quantiser
        adjoint) and 1e-4 for the GroupNorm input gradient, whose terms
        cancel (dx = rstd (g - m1 - x^ m2)); only the fp32 summation order
        differs from the oracle.
  bf16: the weights are rounded to bf16 when packed and every output is
        stored in bf16, so the reference is the oracle on bf16-rounded
        operands; one bf16 rounding has rms relative error 2^-9 / sqrt 3 =
        1.1e-3, two (the upsample adjoint sums rounded fine-resolution
        values) 1.6e-3: bar relative L2 3e-3.
Shapes span several conv tiles (8 x 64 positions) with ragged tails in h and
w, two clips and several frames."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import backward as B  # noqa: E402
from oracle import tokenizer as O  # noqa: E402
from tests import gpu_common as G  # noqa: E402
from tests.test_gpu_wgrad import rel_l2, storage_round, to_chunked  # noqa: E402

pytestmark = pytest.mark.gpu

BAR = {"f32": 1e-5, "bf16": 3e-3}
GN_DX_BAR = {"f32": 1e-4, "bf16": 3e-3}


@pytest.fixture(scope="module")
def tk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2602_03529_amd import tok
    return tok


def from_chunked(t, C):
    """Chunked device tensor -> dense float64 (N,T,H,W,C) on the host."""
    a = t.float().cpu().numpy()
    N, T, k, H, W, CH = a.shape
    return a.transpose(0, 1, 3, 4, 2, 5).reshape(N, T, H, W, k * CH)[..., :C].astype(np.float64)


def cu(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t if dtype is None else t.to(dtype)).cuda()


# (view, Cin, Cout, input shape N,T,H,W)
CONVS = [
    (0, 64, 64, (2, 5, 20, 72)),
    (0, 128, 64, (2, 3, 20, 72)),
    (0, 3, 64, (2, 5, 20, 72)),
    (0, 64, 3, (2, 5, 20, 72)),
    (0, 64, 3, (1, 9, 17, 130)),       # last layer: nine frames walked, ragged row and column tiles
    (1, 64, 128, (2, 5, 20, 72)),
    (1, 128, 128, (2, 5, 20, 72)),
    (1, 64, 128, (1, 1, 4, 6)),        # one frame: the stride-2 adjoint's frame-0 weight set only
    (1, 128, 128, (1, 7, 18, 130)),    # 4 coarse frames, ragged row and column tiles of the adjoint
    (2, 128, 128, (2, 3, 10, 36)),
    (2, 128, 64, (2, 3, 10, 36)),
    (2, 128, 64, (1, 2, 5, 33)),       # odd source height, ragged tiles of the upsampling adjoint
]


def _out_shape(view, N, T, H, W):
    if view == 0:
        return (N, T, H, W)
    if view == 1:
        return (N, (T - 1) // 2 + 1, H // 2, W // 2)
    return (N, 2 * T - 1, 2 * H, 2 * W)


def _oracle_conv(view, x64, w64, b64):
    if view == 2:
        return O.conv3d(O.upsample(x64), w64, b64)
    return O.conv3d(x64, w64, b64, stride=(2, 2) if view == 1 else (1, 1))


def _conv_operands(view, cin, cout, xs, prec, seed):
    w = storage_round(synth.randn(seed, (cout, cin, 3, 3, 3)) * np.sqrt(2.0 / (27 * cin)), prec)
    b = synth.randn(seed + 1, (cout,)).astype(np.float32)
    if cin == 3:
        u8 = synth.make_batch(list(range(xs[0])), xs[1], xs[2], xs[3])
        # the first layer stages the normalised pixels in its own precision
        return w, b, u8, storage_round(O.pixels_to_input(u8), prec).astype(np.float64)
    x = storage_round(synth.randn(seed + 2, xs + (cin,)), prec)
    return w, b, x, x.astype(np.float64)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("view,cin,cout,xs", CONVS)
def test_conv3d_fwd_matches_oracle(tk, prec, view, cin, cout, xs):
    print("conv fwd", prec, view, cin, cout, xs, flush=True)
    w, b, x, x64 = _conv_operands(view, cin, cout, xs, prec, 10 + view + cin + cout)
    ref = _oracle_conv(view, x64, w.astype(np.float64), b.astype(np.float64))
    xin = cu(x) if cin == 3 else to_chunked(x, prec)
    y = tk.conv3d_fwd(xin, cu(w), cu(b), view, xs, cin, cout, prec)
    torch.cuda.synchronize()
    got = y.cpu().numpy().astype(np.float64) if cout == 3 else from_chunked(y, cout)
    e = rel_l2(got, ref)
    print("  rel-L2 %.2e" % e)
    assert got.shape == ref.shape and e <= BAR[prec]


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_conv3d_fwd_residual(tk, prec):
    xs = (2, 5, 20, 72)
    w, b, x, x64 = _conv_operands(0, 64, 64, xs, prec, 7)
    r = storage_round(synth.randn(8, xs + (64,)), prec)
    ref = O.conv3d(x64, w.astype(np.float64), b.astype(np.float64)) + r
    y = tk.conv3d_fwd(to_chunked(x, prec), cu(w), cu(b), 0, xs, 64, 64, prec, resid=to_chunked(r, prec))
    torch.cuda.synchronize()
    assert rel_l2(from_chunked(y, 64), ref) <= BAR[prec]


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("view,cin,cout,xs", CONVS)
def test_conv3d_dgrad_and_wgrad_match_oracle(tk, prec, view, cin, cout, xs):
    print("conv dgrad/wgrad", prec, view, cin, cout, xs, flush=True)
    w, b, x, x64 = _conv_operands(view, cin, cout, xs, prec, 20 + view + cin + cout)
    ys = _out_shape(view, *xs)
    gy = storage_round(synth.randn(30 + view + cin, ys + (cout,)), prec)
    gy64, w64 = gy.astype(np.float64), w.astype(np.float64)
    if view == 2:
        up = O.upsample(x64)
        ref_dx = B.upsample_adjoint(B.conv3d_dgrad(gy64, w64, up.shape))
        ref_dw, ref_db = B.conv3d_wgrad(up, gy64, w.shape)
    else:
        st = (2, 2) if view == 1 else (1, 1)
        ref_dx = B.conv3d_dgrad(gy64, w64, x64.shape, st)
        ref_dw, ref_db = B.conv3d_wgrad(x64, gy64, w.shape, st)
    gin = cu(gy) if cout == 3 else to_chunked(gy, prec)
    xin = cu(x) if cin == 3 else to_chunked(x, prec)
    dx = tk.conv3d_dgrad(gin, cu(w), view, xs, cin, cout, prec)
    dw, db = tk.conv3d_wgrad_op(xin, gin, view, xs, cin, cout, prec)
    torch.cuda.synchronize()
    got_dx = dx.cpu().numpy().astype(np.float64) if cin == 3 else from_chunked(dx, cin)
    e_dx, e_dw, e_db = rel_l2(got_dx, ref_dx), rel_l2(dw.cpu().numpy(), ref_dw), rel_l2(db.cpu().numpy(), ref_db)
    print("  rel-L2 dx %.2e dw %.2e db %.2e" % (e_dx, e_dw, e_db))
    assert e_dx <= BAR[prec]
    # the weight gradient is accumulated in fp32 from identical operands in either precision
    assert e_dw <= 1e-5 and e_db <= 1e-5


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_conv3d_ops_reject_unsupported_shapes(tk, prec):
    from paper_2602_03529_amd._lib import TokError
    w = torch.zeros((64, 64, 3, 3, 3), dtype=torch.float32, device="cuda")
    x = torch.zeros(tk.act_shape(1, 4, 8, 8, 64, prec), dtype=tk._OP_DTYPES[prec], device="cuda")
    with pytest.raises(TokError) as e:   # stride 2 needs an odd frame count
        tk.conv3d_fwd(x, w, None, 1, (1, 4, 8, 8), 64, 64, prec)
    assert e.value.status == -2
    w2 = torch.zeros((48, 64, 3, 3, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(TokError) as e:   # output channels not whole 64-channel tiles
        tk.conv3d_fwd(x, w2, None, 0, (1, 4, 8, 8), 64, 48, prec)
    assert e.value.status == -6


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_act_pack_unpack(tk, prec):
    a = synth.randn(40, (2, 3, 7, 9, 70)).astype(np.float32)
    t = tk.act_pack(cu(a), prec)
    back = tk.act_unpack(t, 70)
    torch.cuda.synchronize()
    ref = storage_round(a, prec)
    np.testing.assert_array_equal(back.cpu().numpy(), ref)
    np.testing.assert_array_equal(from_chunked(t, 70), ref.astype(np.float64))
    # the padding channels of the last chunk are zero
    k = t.shape[2]
    assert float(t[:, :, k - 1, :, :, 70 - (k - 1) * t.shape[-1]:].abs().max()) == 0.0


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_group_norm_silu_ops_match_oracle(tk, prec):
    xs = (2, 3, 20, 72)
    x = storage_round(synth.randn(50, xs + (64,)) * 1.7 + 0.4, prec)
    gam = (1.0 + 0.3 * synth.randn(51, (64,))).astype(np.float32)
    bet = (0.2 * synth.randn(52, (64,))).astype(np.float32)
    gy = storage_round(synth.randn(53, xs + (64,)), prec)
    x64 = x.astype(np.float64)
    gn = O.group_norm(x64, gam.astype(np.float64), bet.astype(np.float64))
    ref_y = O.silu(gn)
    g_a = B.silu_backward(gn, gy.astype(np.float64))
    ref_dx, ref_dg, ref_db = B.group_norm_backward(x64, gam.astype(np.float64), g_a)
    xg = x64.reshape(2 * 3, 20 * 72, 32, 2)
    ref_mean = xg.mean(axis=(1, 3))
    ref_rstd = 1.0 / np.sqrt(xg.var(axis=(1, 3)) + O.GN_EPS)
    xt = to_chunked(x, prec)
    mr = tk.gn_stats(xt, O.GN_EPS)
    y = tk.gn_apply(xt, mr, cu(gam), cu(bet))
    dx, dg, db = tk.gn_bwd(xt, to_chunked(gy, prec), mr, cu(gam), cu(bet))
    torch.cuda.synchronize()
    m = mr.cpu().numpy().astype(np.float64)
    assert rel_l2(m[..., 0], ref_mean) <= 1e-5 and rel_l2(m[..., 1], ref_rstd) <= 1e-5
    e_y = rel_l2(from_chunked(y, 64), ref_y)
    e_dx = rel_l2(from_chunked(dx, 64), ref_dx)
    e_dg, e_db = rel_l2(dg.cpu().numpy(), ref_dg), rel_l2(db.cpu().numpy(), ref_db)
    print(prec, "gn rel-L2 y %.2e dx %.2e dgamma %.2e dbeta %.2e" % (e_y, e_dx, e_dg, e_db))
    assert e_y <= BAR[prec] and e_dx <= GN_DX_BAR[prec]
    assert e_dg <= GN_DX_BAR[prec] and e_db <= GN_DX_BAR[prec]


def test_fsq_ste_bwd_matches_oracle(tk):
    n = 5000
    z = (2.0 * synth.randn(60, (n, 6))).astype(np.float32)
    gc = synth.randn(61, (n, 6)).astype(np.float32)
    gin = synth.randn(62, (n, 6)).astype(np.float32)
    keep = (synth.randn(63, (n,)) > -0.5).astype(np.uint8)
    ref = gin + keep[:, None] * B.fsq_ste_backward(z.astype(np.float64), gc.astype(np.float64))
    got = tk.fsq_ste_bwd(cu(z), cu(gc), cu(keep), cu(gin))
    got_nokeep = tk.fsq_ste_bwd(cu(z), cu(gc))
    torch.cuda.synchronize()
    assert rel_l2(got.cpu().numpy(), ref) <= 1e-5
    assert rel_l2(got_nokeep.cpu().numpy(), B.fsq_ste_backward(z.astype(np.float64), gc.astype(np.float64))) <= 1e-5


def test_residual_block_composed_from_autograd_ops(tk):
    """A residual block x + conv_b(SiLU(GN_b(conv_a(SiLU(GN_a x))))) built from
    the autograd wrappers, with a loss computed in torch (<y, g>): every
    gradient equals the oracle's resblock adjoint (fp32)."""
    prec, xs = "f32", (2, 5, 20, 72)
    p = {k: v.astype(np.float64) for k, v in G.weights(True).items()}
    name = "dec.rb1"
    x = synth.randn(70, xs + (64,)).astype(np.float32)
    g = synth.randn(71, xs + (64,)).astype(np.float32)
    y_ref, tape = B.resblock_fwd(x.astype(np.float64), p, name)
    grads = {}
    gx_ref = B.resblock_bwd(tape, p, name, g.astype(np.float64), grads)

    P = {k: cu(np.asarray(p[name + "." + k], np.float32)).requires_grad_()
         for k in ("gn_a.gamma", "gn_a.beta", "a.w", "a.b", "gn_b.gamma", "gn_b.beta", "b.w", "b.b")}
    xt = to_chunked(x, prec).requires_grad_()
    h = tk.GroupNormSiLUFn.apply(xt, P["gn_a.gamma"], P["gn_a.beta"])
    h = tk.Conv3dFn.apply(h, P["a.w"], P["a.b"], 0, xs, 64, 64, prec)
    h = tk.GroupNormSiLUFn.apply(h, P["gn_b.gamma"], P["gn_b.beta"])
    y = tk.Conv3dFn.apply(h, P["b.w"], P["b.b"], 0, xs, 64, 64, prec, xt)
    loss = (y * to_chunked(g, prec)).sum()
    loss.backward()
    torch.cuda.synchronize()
    assert rel_l2(from_chunked(y.detach(), 64), y_ref) <= 1e-5
    assert rel_l2(from_chunked(xt.grad, 64), gx_ref) <= 1e-4
    for k, t in P.items():
        e = rel_l2(t.grad.cpu().numpy(), grads[name + "." + k])
        print(k, "rel-L2 %.2e" % e)
        assert e <= 1e-4, k


def test_backward_outputs_matches_oracle(tk):
    """tok_backward_outputs and the Tokenizer autograd stage, with the loss
    computed in torch from x_hat, the zero-filled codes and z, against the
    oracle's adjoint of the same outputs (fp32, 2 x 5 x 36 x 72, 30% of
    the tokens dropped)."""
    seeds, T, H, W, rate = (0, 1), 5, 36, 72, 0.3
    u8 = G.clip(seeds, T, H, W)
    p = G.weights64(True)
    T2, H2, W2 = O.latent_shape(T, H, W)
    keep = O.keep_mask(1, rate, 5, np.arange(len(seeds), dtype=np.uint64), T2, H2, W2)
    _, tape = B.train_forward(u8, p, keep)
    rng = np.random.default_rng(80)
    gx = rng.standard_normal(tape["xhat"].shape).astype(np.float32)
    gc = rng.standard_normal(tape["dec_in"].shape).astype(np.float32)
    gz = rng.standard_normal(tape["z"].shape).astype(np.float32)
    ref, ref_dx = B.outputs_backward(tape, p, gx.astype(np.float64), gc.astype(np.float64), gz.astype(np.float64))
    ref_flat = synth.flatten_weights(ref).astype(np.float64)

    m = tk.TokModel(synth.flatten_weights(G.weights(True)), "f32")
    params = cu(synth.flatten_weights(G.weights(True)).astype(np.float32)).requires_grad_()
    x, kp = cu(u8), cu(np.ascontiguousarray(keep, np.uint8))
    xhat, codes, z = tk.tokenizer(m, params, x, kp)
    loss = (xhat * cu(gx)).sum() + (codes * cu(gc)).sum() + (z * cu(gz)).sum()
    loss.backward()
    f = m.train_forward(x, kp, idx=True)
    direct = m.backward_outputs(x, f["ws"], cu(gx), cu(gc), cu(gz), dx=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(f["idx"].cpu().numpy(), tape["idx"])
    assert float(np.abs(codes.detach().cpu().numpy() - tape["dec_in"]).max()) == 0.0
    got = synth.unflatten_weights(params.grad.cpu().numpy())
    for name, _, _ in synth.param_spec():
        e = rel_l2(got[name], ref[name])
        assert e <= 1e-4, (name, e)
    assert rel_l2(direct["dweights"].cpu().numpy(), ref_flat) <= 1e-4
    assert rel_l2(direct["dx"].cpu().numpy(), ref_dx) <= 1e-4
    # the autograd stage and the direct call run the same kernels in the same order
    np.testing.assert_array_equal(params.grad.cpu().numpy(), direct["dweights"].cpu().numpy())
