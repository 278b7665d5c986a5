"""GPU parity of the training step (tok_train_forward / tok_backward) against
the FP64 oracle's hand-written adjoint (oracle/backward.py, itself pinned by
dot-product tests, torch autograd and central finite differences).

Bars: FP32 loss within rel 1e-5 and every parameter tensor's gradient within
relative L2 error 1e-4 of the oracle's, for the oracle's choice of the l1
subgradient's sign at pixels where x_hat is within the reconstruction
tolerance of x (see L1_BAND); BF16 within the bounds stated in its test.  The loss is a mean, so at any size the gradient of a batch is the mean
of its clips' gradients; that property is checked at the training benchmark
size, where the oracle is too slow."""
import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import backward as B  # noqa: E402
from oracle import tokenizer as O  # noqa: E402
from tests import gpu_common as G  # noqa: E402

pytestmark = pytest.mark.gpu

F32_LOSS_RTOL = 1e-5
F32_GRAD_REL_L2 = 1e-4
# The l1 subgradient sign(x_hat - x) is set-valued where x_hat = x: at pixels
# whose oracle residual is within the FP32 reconstruction tolerance, the GPU's
# x_hat may fall on the other side of x, and either sign is a correct
# subgradient.  The adjoint is affine in the seed, so every such choice is the
# oracle gradient plus a sum of per-pixel flip corrections.
L1_BAND = G.F32_RECON_TOL


@pytest.fixture(scope="module")
def tk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2602_03529_amd import tok
    return tok


def keep_mask(N, T, H, W, rate, seed):
    if rate <= 0:
        return None
    T2, H2, W2 = O.latent_shape(T, H, W)
    return O.keep_mask(1, rate, seed, np.arange(N, dtype=np.uint64), T2, H2, W2)


@functools.lru_cache(maxsize=None)
def oracle_step(seeds, T, H, W, rate):
    u8 = G.clip(seeds, T, H, W)
    p = G.weights64(True)
    keep = keep_mask(len(seeds), T, H, W, rate, 5)
    loss, tape = B.train_forward(u8, p, keep)
    grads, dx = B.train_backward(tape, p)
    return loss, tape, grads, dx, keep


def flat_grads(grads, dx):
    return np.concatenate([synth.flatten_weights(grads).astype(np.float64), dx.ravel()])


@functools.lru_cache(maxsize=None)
def l1_band_flips(seeds, T, H, W, rate):
    """Oracle gradient changes (weights and dx, flattened) from flipping the
    l1 sign at each in-band pixel alone."""
    loss, tape, grads, dx, keep = oracle_step(seeds, T, H, W, rate)
    p = G.weights64(True)
    d = tape["xhat"] - tape["x"]
    zero = np.zeros_like(d)
    g0 = flat_grads(*B.train_backward(tape, p, gx_hat=zero))
    flips = []
    for ix in np.argwhere(np.abs(d) < L1_BAND):
        seed = zero.copy()
        seed[tuple(ix)] = -2.0 * np.sign(d[tuple(ix)]) / d.size
        flips.append(flat_grads(*B.train_backward(tape, p, gx_hat=seed)) - g0)
    return flips


def best_valid_gradient(gpu_flat, ref_flat, flips):
    """The oracle gradient for the choice of in-band signs closest to the GPU's."""
    best, best_e = ref_flat, np.inf
    for mask in range(1 << len(flips)):
        cand = ref_flat + sum((f for k, f in enumerate(flips) if mask >> k & 1), np.zeros_like(ref_flat))
        e = np.linalg.norm(gpu_flat - cand)
        if e < best_e:
            best, best_e = cand, e
    return best


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@functools.lru_cache(maxsize=None)
def model(tk, prec):
    return tk.TokModel(synth.flatten_weights(G.weights(True)), prec)


def gpu_step(tk, prec, u8, keep, dx=True):
    m = model(tk, prec)
    x = torch.from_numpy(u8).cuda()
    kp = None if keep is None else torch.from_numpy(np.ascontiguousarray(keep, np.uint8)).cuda()
    f = m.train_forward(x, kp, idx=True, xhat=True)
    b = m.backward(x, f["ws"], dx=dx)
    torch.cuda.synchronize()
    return dict(loss=f["loss"].cpu().numpy(), idx=f["idx"].cpu().numpy(), xhat=f["xhat"].cpu().numpy(),
                dw=b["dweights"].cpu().numpy(), dx=None if b["dx"] is None else b["dx"].cpu().numpy())


def grads_by_name(flat):
    return synth.unflatten_weights(flat)


CASES = [((0,), 9, 64, 64, 0.0), ((0, 1), 5, 36, 72, 0.3)]


@pytest.mark.parametrize("seeds,T,H,W,rate", CASES)
def test_train_step_f32_matches_oracle(tk, seeds, T, H, W, rate):
    print("case", seeds, T, H, W, rate, flush=True)
    loss, tape, grads, dx, keep = oracle_step(seeds, T, H, W, rate)
    g = gpu_step(tk, "f32", G.clip(seeds, T, H, W), keep)
    # the codes must be the oracle's (no in-band flips at these inputs), else the gradients differ legitimately
    np.testing.assert_array_equal(g["idx"], tape["idx"])
    np.testing.assert_allclose(g["loss"][0], loss, rtol=F32_LOSS_RTOL)
    np.testing.assert_allclose(g["loss"][1], tape["l1"], rtol=F32_LOSS_RTOL)
    np.testing.assert_allclose(g["loss"][2], tape["commit"], rtol=F32_LOSS_RTOL)
    flips = l1_band_flips(seeds, T, H, W, rate)
    nw = g["dw"].size
    ref = best_valid_gradient(np.concatenate([g["dw"], g["dx"].ravel()]).astype(np.float64), flat_grads(grads, dx),
                              flips)
    print("in-band l1 pixels: %d" % len(flips), flush=True)
    gg, rg = grads_by_name(g["dw"]), synth.unflatten_weights(ref[:nw])
    dx = ref[nw:].reshape(dx.shape)
    worst = []
    for name, _, _ in synth.param_spec():
        e = rel_l2(gg[name], rg[name])
        worst.append((e, name))
    for e, name in worst:
        print("  grad rel-L2 %-22s %.3e" % (name, e), flush=True)
    worst.sort(reverse=True)
    assert worst[0][0] <= F32_GRAD_REL_L2, worst[:4]
    assert rel_l2(g["dx"], dx) <= F32_GRAD_REL_L2


def test_train_step_bf16_close_to_oracle(tk):
    """BF16 activations and gradients, fp32 accumulation and statistics:
    the loss within rel 1e-2 and the full gradient vector within relative L2
    error 0.1 of the FP64 oracle (cosine similarity >= 0.995)."""
    seeds, T, H, W, rate = CASES[0]
    loss, tape, grads, dx, keep = oracle_step(seeds, T, H, W, rate)
    g = gpu_step(tk, "bf16", G.clip(seeds, T, H, W), keep, dx=False)
    ref = synth.flatten_weights(grads).astype(np.float64)
    e = rel_l2(g["dw"], ref)
    cos = float(np.dot(g["dw"], ref) / (np.linalg.norm(g["dw"]) * np.linalg.norm(ref)))
    print("bf16 loss %.6g vs %.6g; gradient rel-L2 %.4g, cosine %.6f" % (g["loss"][0], loss, e, cos), flush=True)
    np.testing.assert_allclose(g["loss"][0], loss, rtol=1e-2)
    assert e <= 0.1 and cos >= 0.995


def test_backward_deterministic_and_scaled(tk):
    m = model(tk, "f32")
    u8 = G.clip((0, 1), 5, 36, 72)
    x = torch.from_numpy(u8).cuda()
    f = m.train_forward(x)
    a = m.backward(x, f["ws"])["dweights"].clone()
    b = m.backward(x, f["ws"])["dweights"].clone()
    g = torch.tensor([2.5], dtype=torch.float32, device="cuda")
    c = m.backward(x, f["ws"], gloss=g)["dweights"].clone()
    f2 = m.train_forward(x)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(f["loss"], f2["loss"])
    assert rel_l2(c.cpu().numpy(), 2.5 * a.cpu().numpy().astype(np.float64)) <= 1e-6


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_checkpointed_backward_equals_kept_interiors(tk, prec):
    """The smallest workspace makes the backward recompute each residual
    block's interior (per-block checkpointing); the default one keeps the
    interiors on the tape.  Loss, weight and input gradients agree bit for bit."""
    m = model(tk, prec)
    N, T, H, W = 2, 5, 36, 72
    x = torch.from_numpy(G.clip((0, 1), T, H, W)).cuda()
    full, small = m.train_workspace_size(N, T, H, W), m.train_workspace_size(N, T, H, W, recompute=True)
    assert small < full
    fk = m.train_forward(x)
    gk = m.backward(x, fk["ws"], dx=True)
    ws = torch.empty(small, dtype=torch.uint8, device="cuda")
    fr = m.train_forward(x, ws=ws)
    gr = m.backward(x, ws, dx=True)
    torch.cuda.synchronize()
    assert torch.equal(fk["loss"], fr["loss"])
    assert torch.equal(gk["dweights"], gr["dweights"])
    assert torch.equal(gk["dx"], gr["dx"])


def test_autograd_function_matches_direct_call(tk):
    from paper_2602_03529_amd.tok import tokenizer_loss
    m = tk.TokModel(synth.flatten_weights(G.weights(False)), "f32")
    params = torch.from_numpy(synth.flatten_weights(G.weights(True))).cuda().requires_grad_()
    x = torch.from_numpy(G.clip((0,), 9, 64, 64)).cuda()
    loss = tokenizer_loss(m, params, x)
    (3.0 * loss).backward()
    ref = model(tk, "f32")
    f = ref.train_forward(x)
    d = ref.backward(x, f["ws"])["dweights"]
    torch.cuda.synchronize()
    assert torch.equal(loss.detach().reshape(1), f["loss"][:1])
    assert rel_l2(params.grad.cpu().numpy(), 3.0 * d.cpu().numpy().astype(np.float64)) <= 1e-6
    # an in-place parameter update reloads the weights at the next call
    with torch.no_grad():
        params.mul_(0.5)
    loss2 = tokenizer_loss(m, params, x)
    torch.cuda.synchronize()
    assert float(loss2) != float(loss)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_set_weights_equals_fresh_model(tk, prec):
    w1 = synth.flatten_weights(G.weights(True))
    a = tk.TokModel(w1, prec)
    b = tk.TokModel(synth.flatten_weights(G.weights(False)), prec)
    b.set_weights(torch.from_numpy(w1).cuda())
    x = torch.from_numpy(G.clip((2,), 5, 32, 48)).cuda()
    oa, ob = a.encode(x), b.encode(x)
    ra, rb = a.decode(oa["codes"]), b.decode(ob["codes"])
    torch.cuda.synchronize()
    assert torch.equal(oa["z"], ob["z"]) and torch.equal(ra, rb)


def test_train_errors(tk):
    from paper_2602_03529_amd._lib import TokError
    m = model(tk, "f32")
    x = torch.zeros((1, 4, 32, 32, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(TokError) as e:
        m.train_forward(x)
    assert e.value.status == -2
    x = torch.zeros((1, 5, 32, 32, 3), dtype=torch.uint8, device="cuda")
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(TokError) as e:
        m.train_forward(x, ws=small)
    assert e.value.status == -7


def test_batch_gradient_is_mean_of_clip_gradients_at_bench_size(tk):
    """8 clips of 17 x 256 x 256 (the training benchmark's batch), FP32: the
    batch gradient equals the mean of the 8 single-clip gradients."""
    m = model(tk, "f32")
    N, T, H, W = 8, 17, 256, 256
    u8 = synth.make_batch(list(range(N)), T, H, W)
    x = torch.from_numpy(u8).cuda()
    f = m.train_forward(x)
    gb = m.backward(x, f["ws"])["dweights"].cpu().numpy().astype(np.float64)
    lb = float(f["loss"][0])
    del f
    acc = np.zeros_like(gb)
    ls = 0.0
    ws = torch.empty(m.train_workspace_size(1, T, H, W), dtype=torch.uint8, device="cuda")
    for n in range(N):
        xn = x[n:n + 1].contiguous()
        fn = m.train_forward(xn, ws=ws)
        acc += m.backward(xn, ws)["dweights"].cpu().numpy()
        ls += float(fn["loss"][0])
    e = rel_l2(gb, acc / N)
    print("batch vs mean-of-clips gradient rel-L2 %.3g, loss %.8g vs %.8g" % (e, lb, ls / N), flush=True)
    assert abs(lb - ls / N) <= 1e-5 * abs(lb)
    assert e <= 1e-4
