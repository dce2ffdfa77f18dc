"""The reference streams the benchmark's roofline is compared against (a copy
and a read-only sum of 8-byte words): exact results on empty, odd and even
word counts, through the C ABI."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [0, 1, 2, 7, 1000, 1_048_577, 4_000_000])
def test_stream_copy_and_read(n):
    from paper_2307_08637_amd import lsort
    rng = np.random.default_rng(n + 5)
    h = rng.integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)
    src = torch.from_numpy(h.view(np.int64)).cuda()
    dst = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    lsort.stream_copy(src, dst)
    s = lsort.stream_read(src)
    torch.cuda.synchronize()
    assert np.array_equal(dst.cpu().numpy(), h.view(np.int64))
    want = int(h.sum(dtype=np.uint64)) if n else 0  # wraps mod 2^64
    got = int(s.cpu().view(torch.int64).item()) & (2**64 - 1)
    assert got == want
