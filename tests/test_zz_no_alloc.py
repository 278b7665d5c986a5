"""The selection entry point that allocates nothing
(tok_select_similar_noalloc, static per-GPU scratch) against
tok_select_similar with a caller workspace, through the C ABI: keep masks
and zero-filled codes bit-identical, on two calls in a row with the second
batch smaller than the first (the scratch keeps the first call's contents,
so anything the selection fails to reset would show), and a batch beyond the
scratch rejected before any launch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from tests.test_gpu_similarity import check_selection_properties, redundant_codes  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2602_03529_amd import tok
    return tok


def _pair(tk, codes, rate):
    a = torch.from_numpy(codes).cuda()
    b = a.clone()
    ka = tk.select_similar(a, rate)
    kb = tk.select_similar_noalloc(b, rate)
    torch.cuda.synchronize()
    return a.cpu().numpy(), ka.cpu().numpy(), b.cpu().numpy(), kb.cpu().numpy()


@pytest.mark.parametrize("big,small,rate", [
    ((4, 5, 180, 320), (2, 3, 9, 13), 0.3),
    ((3, 4, 37, 45), (1, 2, 5, 7), 0.61),
])
def test_noalloc_matches_workspace_entry_point(tk, big, small, rate):
    for k, shape in enumerate((big, small)):
        codes = redundant_codes(100 + k, *shape)
        ca, ka, cb, kb = _pair(tk, codes, rate)
        assert np.array_equal(ka, kb), shape
        assert np.array_equal(ca.view(np.uint32), cb.view(np.uint32)), shape
        check_selection_properties(codes, kb, rate)


def test_noalloc_rejects_batches_beyond_the_scratch(tk):
    from paper_2602_03529_amd import _lib as L
    cap = tk.select_scratch_bytes()
    shape = (1, 9, 1080, 1920)  # 8 P frames of 2 M tokens: 66 MB of order keys
    assert tk.select_workspace_size(*shape) > cap
    codes = torch.zeros(shape + (6,), dtype=torch.float32, device="cuda")
    with pytest.raises(L.TokError) as e:
        tk.select_similar_noalloc(codes, 0.3)
    assert e.value.status == -7  # TOK_EWORKSPACE
