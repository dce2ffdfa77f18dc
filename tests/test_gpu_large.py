"""Full-size parity: the benchmark's 1e8-key configuration compared word for
word with the oracle (keys only, and with a payload), the large-array path's
stable scatter with fallback trees, and the two largest workloads -- 1e9
keys of the piecewise law under every first-level model, and the whole
10,000-array batched workload with payload -- checked by properties that pin
a sort at any size: sorted (per array), equal multisets of (key, payload,
array) triples, stability, and the sorted-position definition at sampled
positions."""
import numpy as np
import pytest
import torch

import oracle
from paper_2307_08637_amd import inputs, lsort
from tests.gpu_helpers import is_sorted, multiset_hash, signed_order_key, to_dev, to_host

pytestmark = pytest.mark.gpu


def assert_same_bits(got, want):
    g = np.ascontiguousarray(got).view(np.uint64)
    w = np.ascontiguousarray(want).view(np.uint64)
    assert g.shape == w.shape
    bad = np.flatnonzero(g != w)
    assert bad.size == 0, f"{bad.size} mismatches, first at {bad[:5]}"


def u32(a: np.ndarray, dev) -> torch.Tensor:
    return torch.from_numpy(a.view(np.int32).copy()).to(dev).view(torch.uint32)


def test_1e8_normal_oracle_bitexact(dev):
    """The benchmark's configuration (1e8 normal float64 keys, default
    options): every output word equal to the oracle's."""
    n = 100_000_000
    keys = inputs.generate("normal", n, seed=21)
    t = to_dev(keys, dev)
    print("[case] 1e8 normal vs oracle", flush=True)
    lsort.sort(t)
    torch.cuda.synchronize()
    got = to_host(t)
    del t
    assert_same_bits(got, oracle.sort(keys)[0])


def test_1e8_payload_oracle_bitexact(dev):
    """1e8 lognormal keys with a uint32 payload (the original index): keys
    and payload equal to the oracle's stable sort word for word."""
    n = 100_000_000
    keys = inputs.generate("lognormal", n, seed=22)
    pay = np.arange(n, dtype=np.uint32)
    t, p = to_dev(keys, dev), u32(pay, dev)
    print("[case] 1e8 lognormal + payload vs oracle", flush=True)
    lsort.sort(t, p)
    torch.cuda.synchronize()
    got, gp = to_host(t), p.view(torch.int32).cpu().numpy().view(np.uint32)
    del t, p
    want, wp = oracle.sort(keys, pay)
    assert_same_bits(got, want)
    assert np.array_equal(gp, wp)


@pytest.mark.parametrize("law", ["normal", "exponential"])
def test_large_path_payload_with_fallbacks(dev, law):
    """A large array (first level from the 1% sample, fine second level)
    with a payload and a low fallback threshold, so that oversized buckets
    take splitter trees built from the first-level sample: keys and payload
    equal to the oracle's stable sort."""
    n = 5_000_000
    keys = inputs.generate(law, n, seed=72)
    pay = np.arange(n, dtype=np.uint32)
    t, p = to_dev(keys, dev), u32(pay, dev)
    print(f"[case] 5e6 {law} + payload, fallback 1.5", flush=True)
    lsort.sort(t, p, buckets=1000, fallback_ratio=1.5)
    torch.cuda.synchronize()
    st = lsort.stats()["levels"]
    assert st[0]["learned"] == 1 and st[0]["fallback"] > 0, st[0]
    want, wp = oracle.sort(keys, pay)
    assert_same_bits(to_host(t), want)
    assert np.array_equal(p.view(torch.int32).cpu().numpy().view(np.uint32), wp)


def test_c5_1e9_piecewise_properties(dev):
    """1e9 float64 keys of the 70/20/10 piecewise law (8 GB, sorted in place
    with an 8 GB temporary) under the RMI, the MLP-rooted model and the
    splitter tree: sorted, the same multiset (count and two hashes), and the
    sorted-position definition #{keys < v} <= i < #{keys <= v} at sampled
    positions i."""
    n = 1_000_000_000
    keys = inputs.generate("piecewise", n, seed=81)
    src = to_dev(keys, dev)
    del keys
    h1, h2 = multiset_hash(src), multiset_hash(src, salt=0x5A5A5A5A5A5A5A5)
    sk = signed_order_key(src)
    t = torch.empty_like(src)
    for model in ("auto", "mlp", "splitter"):
        t.copy_(src)
        print(f"[case] 1e9 piecewise model={model}", flush=True)
        lsort.sort(t, model=model)
        torch.cuda.synchronize()
        st = lsort.stats()
        assert st["overflow"] == 0
        if model == "mlp":
            assert st["first_model"] == lsort.MODEL["mlp"]
        assert is_sorted(t)
        assert multiset_hash(t) == h1 and multiset_hash(t, salt=0x5A5A5A5A5A5A5A5) == h2
        out = signed_order_key(t)
        for i in np.random.default_rng(1).integers(0, n, 8).tolist() + [0, n - 1]:
            v = out[i]
            lt = int((sk < v).sum().item())
            le = int((sk <= v).sum().item())
            assert lt <= i < le, (model, i, lt, le)
        del out
    del src, sk, t


def test_c4_full_batched_properties(dev):
    """The whole batched workload: 10,000 arrays, sizes log-uniform in
    [1e3, 1e6] (about 1.45e9 keys), five float64 laws, uint32 payload = index
    within the array: every array sorted, the payload stable, and (key,
    payload, array) triples the same multiset as the input."""
    keys, off, pay, _ = inputs.segmented(10_000, seed=41)
    n, m = keys.size, off.size - 1
    assert m == 10_000 and n > 1_000_000_000
    t = to_dev(keys, dev)
    p = u32(pay, dev)
    o = torch.from_numpy(off.view(np.int64).copy()).to(dev).view(torch.uint64)
    del keys, pay
    seg = torch.repeat_interleave(torch.arange(m, device=dev),
                                  torch.from_numpy(np.diff(off).astype(np.int64)).to(dev))

    def triple_hash(kk, pp, salt=0):
        pv = pp.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        return multiset_hash(kk.view(torch.int64) ^ (pv << 17) ^ (seg << 45), salt=salt)
    h0, h1 = triple_hash(t, p), triple_hash(t, p, salt=0x3C3C3C3C3C3C3C3)
    print(f"[case] C4 full m={m} n={n}", flush=True)
    lsort.sort_segmented(t, o, p)
    torch.cuda.synchronize()
    assert lsort.stats()["overflow"] == 0
    k = signed_order_key(t)
    same = seg[:-1] == seg[1:]
    assert bool(((k[:-1] <= k[1:]) | ~same).all().item())
    tie = same & (k[:-1] == k[1:])
    del k
    pi = p.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    assert bool(((pi[:-1] < pi[1:]) | ~tie).all().item())
    del pi, tie, same
    assert triple_hash(t, p) == h0 and triple_hash(t, p, salt=0x3C3C3C3C3C3C3C3) == h1
    # a few arrays in full against the oracle
    host_k = to_host(t)
    host_p = p.view(torch.int32).cpu().numpy().view(np.uint32)
    keys0, _, pay0, _ = inputs.segmented(10_000, seed=41)
    for s in (0, 1, 4999, 9999):
        a, b = int(off[s]), int(off[s + 1])
        want, wp = oracle.sort(keys0[a:b], pay0[a:b])
        assert_same_bits(host_k[a:b], want)
        assert np.array_equal(host_p[a:b], wp)
    del t, p, o, seg


def _chunked_hash(t: torch.Tensor, salt: int, chunk: int = 1 << 28) -> int:
    h = 0
    for a in range(0, t.numel(), chunk):
        h = (h + multiset_hash(t[a:a + chunk], salt=salt)) % (1 << 64)
    return h


def _chunked_sorted(t: torch.Tensor, chunk: int = 1 << 28) -> bool:
    n = t.numel()
    for a in range(0, n - 1, chunk):
        if not is_sorted(t[a:min(n, a + chunk + 1)]):  # each chunk with the first key of the next
            return False
    return True


def test_beyond_2_32_keys(dev):
    """4.4e9 float64 keys (more than 2^32; 35 GB, normal law, drawn on the
    device from a seeded generator) sorted in place with a caller workspace:
    every count, offset and unit index of the path is 64-bit.  Checked by
    properties that pin the result at any size: sorted, and the same multiset
    (two independent 64-bit hashes)."""
    n = 4_400_000_000
    g = torch.Generator(device=dev)
    g.manual_seed(91)
    t = torch.randn(n, dtype=torch.float64, device=dev, generator=g)
    h1, h2 = _chunked_hash(t, 0), _chunked_hash(t, 0x5A5A5A5A5A5A5A5)
    ws = torch.empty(lsort.workspace_bytes(n), dtype=torch.uint8, device=dev)
    print(f"[case] n={n} workspace {ws.numel() / 1e9:.1f} GB", flush=True)
    try:
        lsort.set_workspace(ws)
        lsort.sort(t)
        torch.cuda.synchronize()
        st = lsort.stats()
    finally:
        lsort.set_workspace(None)
        torch.cuda.synchronize()
    del ws
    assert st["overflow"] == 0
    assert st["levels"][0]["keys"] == n
    assert _chunked_sorted(t)
    assert _chunked_hash(t, 0) == h1 and _chunked_hash(t, 0x5A5A5A5A5A5A5A5) == h2
    del t
    torch.cuda.empty_cache()
