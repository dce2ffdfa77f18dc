"""Key types and payload widths the partition engine reaches through
order-preserving maps (int64 keys by a sign flip, float32 keys widened to
float64 and narrowed back, 64-bit payloads gathered through the sorted
original indices): every output word equal to the oracle's stable sort."""
import numpy as np
import pytest
import torch

import oracle
from paper_2307_08637_amd import inputs, lsort

pytestmark = pytest.mark.gpu

TORCH = {np.float32: torch.float32, np.int64: torch.int64, np.float64: torch.float64, np.uint64: torch.uint64}


def dev_tensor(a: np.ndarray, dev) -> torch.Tensor:
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64).copy()).to(dev).view(torch.uint64)
    return torch.from_numpy(np.ascontiguousarray(a).copy()).to(dev)


def host_bytes(t: torch.Tensor) -> np.ndarray:
    signed = {torch.uint64: torch.int64, torch.uint32: torch.int32}
    if t.dtype in signed:
        t = t.view(signed[t.dtype])
    return np.ascontiguousarray(t.cpu().numpy()).view(np.uint8)


def run_both(keys: np.ndarray, dev, payload: np.ndarray | None, **opts):
    t = dev_tensor(keys, dev)
    p = None if payload is None else dev_tensor(payload, dev)
    if payload is not None and payload.dtype == np.uint32:
        p = torch.from_numpy(payload.view(np.int32).copy()).to(dev).view(torch.uint32)
    print(f"[case] n={keys.size} {keys.dtype} payload={None if payload is None else payload.dtype} {opts}",
          flush=True)
    lsort.sort(t, p, **opts)
    torch.cuda.synchronize()
    want, wp = oracle.sort(keys, payload)
    assert np.array_equal(host_bytes(t), np.ascontiguousarray(want).view(np.uint8))
    if payload is not None:
        assert np.array_equal(host_bytes(p), np.ascontiguousarray(wp).view(np.uint8))


def f32_law(law, n, seed):
    return inputs.generate(law, n, seed=seed).astype(np.float32)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 1000, 70_000, 300_001, 2_500_000])
@pytest.mark.parametrize("pay", [False, True])
def test_f32_normal(dev, n, pay):
    keys = f32_law("normal", n, seed=n % 101)
    run_both(keys, dev, np.arange(n, dtype=np.uint32) if pay else None)


@pytest.mark.parametrize("law", ["uniform", "lognormal", "exponential", "mixgauss"])
def test_f32_laws(dev, law):
    run_both(f32_law(law, 1_000_000, seed=5), dev, None)


@pytest.mark.parametrize("n", [50, 5000, 200_000, 3_000_000])
def test_f32_specials(dev, n):
    keys = inputs.adversarial("f32_specials", n, seed=n % 13)
    run_both(keys, dev, np.arange(n, dtype=np.uint32))
    run_both(keys, dev, None, model="splitter")


@pytest.mark.parametrize("n", [2, 1000, 150_000, 2_000_003])
def test_i64(dev, n):
    keys = inputs.adversarial("i64_extremes", n, seed=n % 17)
    run_both(keys, dev, np.arange(n, dtype=np.uint32))
    small = np.random.default_rng(n).integers(-1000, 1000, n).astype(np.int64)
    run_both(small, dev, None)


@pytest.mark.parametrize("kdt", [np.float64, np.uint64, np.int64, np.float32])
@pytest.mark.parametrize("n", [7, 4096, 400_000, 2_200_000])
def test_payload64(dev, kdt, n):
    rng = np.random.default_rng(n + 3)
    if kdt == np.float64:
        keys = inputs.generate("lognormal", n, seed=4)
    elif kdt == np.uint64:
        keys = inputs.generate("zipf", n, seed=4)
    elif kdt == np.int64:
        keys = inputs.adversarial("i64_extremes", n, seed=4)
    else:
        keys = inputs.adversarial("f32_specials", n, seed=4)
    pay = rng.integers(0, 2**64, n, dtype=np.uint64, endpoint=False)
    run_both(keys, dev, pay)


def test_f32_segmented_with_payload(dev):
    keys64, off, pay, _ = inputs.segmented(300, seed=43, lo=10, hi=2e5)
    keys = keys64.astype(np.float32)
    t = dev_tensor(keys, dev)
    p = torch.from_numpy(pay.view(np.int32).copy()).to(dev).view(torch.uint32)
    o = torch.from_numpy(off.view(np.int64).copy()).to(dev).view(torch.uint64)
    lsort.sort_segmented(t, o, p)
    torch.cuda.synchronize()
    want, wp = oracle.sort_segmented(keys, off, pay)
    assert np.array_equal(host_bytes(t), want.view(np.uint8))
    assert np.array_equal(p.view(torch.int32).cpu().numpy().view(np.uint32), wp)


def test_i64_f32_noalloc(dev):
    for keys in (inputs.adversarial("i64_extremes", 500_000, seed=8), f32_law("normal", 1_200_000, seed=9)):
        t = dev_tensor(keys, dev)
        lsort.sort_noalloc(t)
        torch.cuda.synchronize()
        assert np.array_equal(host_bytes(t), oracle.sort(keys)[0].view(np.uint8))


def test_type_errors(dev):
    t = torch.zeros(10, dtype=torch.int32, device=dev)
    with pytest.raises(TypeError):
        lsort.sort(t)
    k = torch.zeros(10, dtype=torch.float64, device=dev)
    with pytest.raises(TypeError):
        lsort.sample(k.to(torch.float32), 1, 4)
    p = torch.zeros(9, dtype=torch.uint64, device=dev)
    with pytest.raises(ValueError):
        lsort.sort(k, p)
