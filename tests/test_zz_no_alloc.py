"""The allocation-free entry point (ls_sort_noalloc, fixed scratch array in
the library) against ls_sort: every output word equal, on calls in a row
that share the array, each later one smaller than the one before it."""
import numpy as np
import pytest
import torch

from paper_2307_08637_amd import inputs, lsort
from tests.gpu_helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


def u32(a: np.ndarray, dev) -> torch.Tensor:
    return torch.from_numpy(a.view(np.int32).copy()).to(dev).view(torch.uint32)


def both(keys: np.ndarray, dev, payload: bool, **opts):
    """(noalloc keys, noalloc payload, ls_sort keys, ls_sort payload) on host."""
    n = keys.size
    pay = np.arange(n, dtype=np.uint32) if payload else None
    a, b = to_dev(keys, dev), to_dev(keys, dev)
    pa = u32(pay, dev) if payload else None
    pb = u32(pay, dev) if payload else None
    lsort.sort_noalloc(a, pa, **opts)
    torch.cuda.synchronize()
    assert lsort.stats()["overflow"] == 0
    lsort.sort(b, pb, **opts)
    torch.cuda.synchronize()
    host = lambda p: None if p is None else p.view(torch.int32).cpu().numpy().view(np.uint32)  # noqa: E731
    return to_host(a), host(pa), to_host(b), host(pb)


def same(ga, pa, gb, pb):
    assert np.array_equal(np.ascontiguousarray(ga).view(np.uint64), np.ascontiguousarray(gb).view(np.uint64))
    if pa is not None:
        assert np.array_equal(pa, pb)


@pytest.mark.parametrize("calls", [
    # (law, n, payload): the first call of each row takes the large-array
    # path (first level from the 1% sample, sorted by a nested run), later
    # ones are smaller
    [("normal", 2_200_000, False), ("lognormal", 300_000, True)],
    [("mixgauss", 1_900_000, True), ("u64", 1_000_000, False), ("exponential", 5_000, True)],
])
def test_noalloc_equals_sort(dev, calls):
    for law, n, payload in calls:
        print(f"[case] noalloc {law} n={n} payload={payload}", flush=True)
        keys = inputs.generate(law, n, seed=n % 1000 + 3)
        same(*both(keys, dev, payload))


def test_noalloc_adversarial_and_options(dev):
    for kind, n, opts in (("with_nan", 400_000, {}), ("sparse_specials", 150_000, {"model": "splitter"}),
                          ("few_distinct", 70_000, {"cutoff": 256})):
        print(f"[case] noalloc {kind} n={n} {opts}", flush=True)
        keys = inputs.adversarial(kind, n, seed=5)
        same(*both(keys, dev, True, **opts))


def test_noalloc_rejects_sizes_above_the_array(dev):
    n = 2_400_000
    t = torch.zeros(n, dtype=torch.float64, device=dev)
    need = lsort.workspace_bytes(n, 1, payload=False, fixed_levels=True)
    assert need > 64 << 20
    with pytest.raises(lsort.LsortError, match="scratch"):
        lsort.sort_noalloc(t)
    # nothing was enqueued: the keys are untouched, and the next call works
    assert int(torch.count_nonzero(t).item()) == 0
    keys = inputs.generate("uniform", 50_000, seed=9)
    same(*both(keys, dev, False))
