"""GPU tests of the streaming request loop: every clip's result in a mixed,
batched, overlapping stream equals the same clip run alone (bit-exact, since
the kernels are batch-invariant), admission respects the HBM budget, and an
impossible request is refused without stopping the loop."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from tests import gpu_common as G  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2602_03529_amd import tok
    return tok


@pytest.fixture(scope="module")
def model(tk):
    return tk.TokModel(synth.flatten_weights(G.weights(True)), "bf16")


SHAPES = [(5, 32, 48), (9, 40, 64), (5, 64, 64), (1, 16, 24)]


def _clip(i, T, H, W):
    return torch.from_numpy(synth.make_clip(100 + i, T, H, W)).pin_memory()


def _alone(tk, model, px, drop):
    x = px.cuda()
    out = model.encode(x[None], drop=drop)
    xh = model.decode(out["codes"])
    torch.cuda.synchronize()
    return {k: v[0].cpu().numpy() for k, v in out.items() if k != "z"}, xh[0].cpu().numpy()


@pytest.mark.parametrize("modes", [(1,), (1, 2, 4)])
def test_mixed_stream_equals_alone(tk, model, modes):
    """Bernoulli drops only, and a mix of Bernoulli, lost-row and
    similarity-based (Sec. 4.3, Eq. 3) drops across the clips of the stream."""
    rng = np.random.default_rng(7)
    reqs = []
    for i in range(14):
        T, H, W = SHAPES[int(rng.integers(len(SHAPES)))]
        mode = modes[i % len(modes)]
        d = tk.Drop(mode=mode, rate=float(rng.uniform(0, 0.5)), seed=11, clip_id0=1000 + i)
        reqs.append((i, T, H, W, _clip(i, T, H, W), d))
    budget = 3 * max(model.workspace_size(1, T, H, W) for _, T, H, W, _, _ in reqs) + (64 << 20)
    sv = tk.TokServer(model, budget, slots=3, max_batch=3)
    tickets = []
    for i, T, H, W, px, d in reqs:
        tickets.append(sv.submit(px, d))
        if i % 4 == 3:
            time.sleep(0.002)  # arrivals while earlier work is on the GPU
    batched = 0
    for (i, T, H, W, px, d), t in zip(reqs, tickets):
        r = sv.wait(t, timeout_ms=60000)
        assert r is not None and r["status"] == 0, r
        batched = max(batched, r["batch_size"])
        got = sv.fetch(t, T, H, W)
        torch.cuda.synchronize()
        sv.release(t)
        ref, xh = _alone(tk, model, px, d)
        np.testing.assert_array_equal(got["codes"].cpu().numpy(), ref["codes"])
        np.testing.assert_array_equal(got["idx"].cpu().numpy(), ref["idx"])
        np.testing.assert_array_equal(got["keep"].cpu().numpy(), ref["keep"])
        np.testing.assert_array_equal(got["xhat"].cpu().numpy(), xh)
    st = sv.stats()
    assert st["bytes_peak"] <= budget
    assert st["finished"] == len(reqs) and st["queued"] == 0 and st["running"] == 0
    assert st["bytes_in_use"] == 0
    sv.close()


def test_oversized_request_refused_and_loop_keeps_serving(tk, model):
    from paper_2602_03529_amd._lib import TokError
    small = (5, 32, 32)
    budget = model.workspace_size(1, *small) * 2 + (16 << 20)
    sv = tk.TokServer(model, budget, slots=2, max_batch=2)
    with pytest.raises(TokError) as e:
        sv.submit(_clip(0, 9, 256, 256))
    assert e.value.status == -5  # TOK_EBUDGET
    t = sv.submit(_clip(1, *small))
    r = sv.wait(t, timeout_ms=60000)
    assert r is not None and r["status"] == 0
    sv.release(t)
    sv.close()


def test_budget_bounds_concurrency(tk, model):
    """With room for one clip at a time the clips still all finish, serially."""
    shape = (9, 48, 64)
    probe = tk.TokServer(model, 1 << 30, slots=1, max_batch=1)
    need = probe.request_bytes(*shape)  # streaming workspace + clip buffers
    probe.close()
    budget = int(need * 1.5)
    sv = tk.TokServer(model, budget, slots=4, max_batch=4)
    ts = [sv.submit(_clip(i, *shape)) for i in range(5)]
    for t in ts:
        r = sv.wait(t, timeout_ms=60000)
        assert r is not None and r["status"] == 0 and r["batch_size"] == 1
        sv.release(t)
    assert sv.stats()["bytes_peak"] <= budget
    sv.close()
