"""dtb_topk_noalloc: the top-k entry point that allocates no device memory
(its scores and indices pass through the library's static staging area)
gives the indices of dtb_topk, on consecutive calls of shrinking size."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dtb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2308_01241_amd as m
    m.load()
    return m


def _scores(rng, n):
    s = rng.integers(0, 50, n).astype(np.float32)  # many ties
    s[n // 3] = np.nan
    return s


def test_topk_noalloc_equals_topk_on_consecutive_calls(dtb):
    import torch
    from paper_2308_01241_amd.surrogate import topk, topk_noalloc
    rng = np.random.default_rng(11)
    stream = torch.cuda.current_stream()
    # the second call is smaller than the first: stale staged scores past n
    # must not leak into its selection
    for n, k, st in [(4096, 64, None), (1000, 17, stream), (37, 37, None)]:
        s = _scores(rng, n)
        got = topk_noalloc(s, k, stream=st)
        want = topk(s, k)
        np.testing.assert_array_equal(got, want)
        key = np.where(np.isnan(s), np.inf, s)
        np.testing.assert_array_equal(got, np.lexsort((np.arange(n), key))[:k])


def test_topk_noalloc_rejects_sizes_past_its_staging_area(dtb):
    from paper_2308_01241_amd import DtbError
    from paper_2308_01241_amd.surrogate import topk_noalloc
    with pytest.raises(DtbError, match="4096"):
        topk_noalloc(np.zeros(4097, np.float32), 1)
    with pytest.raises(DtbError):
        topk_noalloc(np.zeros(8, np.float32), 9)
