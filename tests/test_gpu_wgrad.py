"""GPU parity of the weight-gradient kernels (tok_conv3d_wgrad) against the
FP64 oracle's conv3d_wgrad, for the three input views (stride 1, stride 2,
nearest-x2 upsampled) and the channel counts of the tokenizer's layers.
Inputs are drawn in float32 and rounded to the kernel's storage precision
first, so both sides see identical values; the only difference left is the
fp32 accumulation order, bounded here by relative L2 error 1e-5.  bf16
operands with 64-multiple channel counts run on the bf16 MFMA kernel, the
others on the fp32 MFMA kernel."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import backward as B  # noqa: E402
from oracle import tokenizer as O  # noqa: E402

pytestmark = pytest.mark.gpu

REL_L2 = 1e-5


@pytest.fixture(scope="module")
def tk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2602_03529_amd import tok
    return tok


def storage_round(a, prec):
    t = torch.from_numpy(np.ascontiguousarray(a, np.float32))
    if prec == "bf16":
        t = t.to(torch.bfloat16).to(torch.float32)
    return t.numpy()


def to_chunked(a, prec):
    """(N,T,H,W,C) -> chunked device tensor [N][T][C/CH][H][W][CH]."""
    CH = 32 if prec == "bf16" else 16
    N, T, H, W, Cc = a.shape
    k = -(-Cc // CH)
    pad = np.zeros((N, T, H, W, k * CH), np.float32)
    pad[..., :Cc] = a
    c = np.ascontiguousarray(pad.reshape(N, T, H, W, k, CH).transpose(0, 1, 4, 2, 3, 5))
    t = torch.from_numpy(c)
    return (t.to(torch.bfloat16) if prec == "bf16" else t).cuda()


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


VIEWS = {0: "s1", 1: "s2", 2: "up"}
CHANNELS = [(64, 64), (64, 128), (128, 64), (128, 128), (3, 64), (64, 3)]


@pytest.mark.parametrize("prec", ["bf16", "f32"])
@pytest.mark.parametrize("view", [0, 1, 2])
@pytest.mark.parametrize("cin,cout", CHANNELS)
def test_wgrad_matches_oracle(tk, prec, view, cin, cout):
    N = 2
    if view == 0:
        xs, ys = (N, 5, 12, 70), (N, 5, 12, 70)
    elif view == 1:
        xs, ys = (N, 5, 12, 70), (N, 3, 6, 35)
    else:
        xs, ys = (N, 3, 6, 35), (N, 5, 12, 70)
    seed = 100 * view + cin + cout
    x = storage_round(synth.randn(seed, xs + (cin,)), prec)
    dy = storage_round(synth.randn(seed + 1, ys + (cout,)), prec)
    x64, dy64 = x.astype(np.float64), dy.astype(np.float64)
    if view == 2:
        gw, gb = B.conv3d_wgrad(O.upsample(x64), dy64, (cout, cin, 3, 3, 3))
    else:
        gw, gb = B.conv3d_wgrad(x64, dy64, (cout, cin, 3, 3, 3), stride=(2, 2) if view == 1 else (1, 1))
    dw, db = tk.conv3d_wgrad(to_chunked(x, prec), to_chunked(dy, prec), xs, ys, cin, cout, view, prec)
    torch.cuda.synchronize()
    e_w, e_b = rel_l2(dw.cpu().numpy(), gw), rel_l2(db.cpu().numpy(), gb)
    print(prec, VIEWS[view], cin, cout, "rel-L2 dw %.2e db %.2e" % (e_w, e_b), flush=True)
    assert e_w <= REL_L2 and e_b <= REL_L2


@pytest.mark.parametrize("prec", ["bf16", "f32"])
def test_wgrad_upsample_ragged_rows_and_single_odd_frame(tk, prec):
    """Upsampling view with an odd source height (a partial row pair at the
    bottom), a ragged last column tile and Ti = 2 (one odd output frame)."""
    cin, cout = 128, 64
    xs, ys = (1, 2, 5, 33), (1, 3, 10, 66)
    x = storage_round(synth.randn(71, xs + (cin,)), prec)
    dy = storage_round(synth.randn(72, ys + (cout,)), prec)
    gw, gb = B.conv3d_wgrad(O.upsample(x.astype(np.float64)), dy.astype(np.float64), (cout, cin, 3, 3, 3))
    dw, db = tk.conv3d_wgrad(to_chunked(x, prec), to_chunked(dy, prec), xs, ys, cin, cout, 2, prec)
    torch.cuda.synchronize()
    e_w, e_b = rel_l2(dw.cpu().numpy(), gw), rel_l2(db.cpu().numpy(), gb)
    print(prec, "up ragged rel-L2 dw %.2e db %.2e" % (e_w, e_b), flush=True)
    assert e_w <= REL_L2 and e_b <= REL_L2


def test_wgrad_rejects_mismatched_shapes(tk):
    from paper_2602_03529_amd._lib import TokError
    x = torch.zeros((1, 5, 2, 8, 8, 32), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(TokError) as e:
        tk.conv3d_wgrad(x, x, (1, 5, 8, 8), (1, 5, 4, 4), 64, 64, 0, "bf16")
    assert e.value.status == -2
