"""The batched (segmented) form: bit-exact parity with the oracle's
per-array stable sort on a mix of array sizes and laws, graph capture and
replay of a fixed-level call, the C4 workload's 2e8-key prefix checked by
properties, and the autotuner's table used by a tuned call."""
import numpy as np
import pytest
import torch

import oracle
from paper_2307_08637_amd import inputs, lsort
from tests.gpu_helpers import multiset_hash, signed_order_key, to_dev, to_host

pytestmark = pytest.mark.gpu


def upload(keys, off, pay, dev):
    t = to_dev(keys, dev)
    p = torch.from_numpy(pay.view(np.int32).copy()).to(dev).view(torch.uint32)
    o = torch.from_numpy(off.view(np.int64).copy()).to(dev).view(torch.uint64)
    return t, o, p


def check(t, p, want, wp):
    assert np.array_equal(to_host(t).view(np.uint64), want.view(np.uint64))
    assert np.array_equal(p.view(torch.int32).cpu().numpy().view(np.uint32), wp)


def test_batched_mix_vs_oracle(dev):
    """2000 arrays, sizes log-uniform in [1e3, 1e5], the five float64 laws,
    payload = index within the array (stability)."""
    keys, off, pay, _ = inputs.segmented(2000, seed=41, lo=1e3, hi=1e5)
    t, o, p = upload(keys, off, pay, dev)
    print(f"[case] batched m=2000 n={keys.size}", flush=True)
    lsort.sort_segmented(t, o, p)
    torch.cuda.synchronize()
    check(t, p, *oracle.sort_segmented(keys, off, pay))


@pytest.mark.parametrize("m,lo,hi", [(300, 10, 2e5), (40, 1e4, 1e6)])
def test_graph_capture_replay(dev, m, lo, hi):
    """A fixed-level call captured into a graph (with a caller-owned
    workspace) replays correctly several times, with other GPU work, host
    synchronisation and a larger eager call on the library's own pool
    between replays; the overflow word read after each replay is zero."""
    keys, off, pay, _ = inputs.segmented(m, seed=43, lo=lo, hi=hi)
    want, wp = oracle.sort_segmented(keys, off, pay)
    t, o, p = upload(keys, off, pay, dev)
    k0, p0 = t.clone(), p.clone()
    opts = dict(fixed_levels=True, stats=False)
    nbytes = lsort.workspace_bytes(keys.size, m, payload=True, fixed_levels=True)
    ws = torch.empty((nbytes + 7) // 8, dtype=torch.int64, device=dev)
    lsort.set_workspace(ws)
    try:
        lsort.sort_segmented(t, o, p, **opts)  # set-up outside capture: look-back words of this layout
        torch.cuda.synchronize()
        check(t, p, want, wp)
        assert lsort.stats()["overflow"] == 0
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            t.copy_(k0)
            p.copy_(p0)
            lsort.sort_segmented(t, o, p, **opts)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        check(t, p, want, wp)
        g = torch.cuda.CUDAGraph()
        print(f"[case] capture m={m} n={keys.size}", flush=True)
        with torch.cuda.graph(g):
            lsort.sort_segmented(t, o, p, **opts)
    finally:
        torch.cuda.synchronize()
        lsort.set_workspace(None)
    big = inputs.generate("normal", 3 * keys.size + 1000, seed=5)
    for r in range(3):
        t.copy_(k0)
        p.copy_(p0)
        junk = torch.arange(1 << 20, device=dev, dtype=torch.float64).sqrt().sum()  # unrelated eager work
        if r == 1:  # a larger eager call grows the library's own pool; the graph does not use it
            tb = to_dev(big, dev)
            lsort.sort(tb)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        print(f"[case] replay {r}", flush=True)
        check(t, p, want, wp)
        del junk
    del g, ws


def test_capture_needs_caller_workspace(dev):
    """Under stream capture the library's own (reallocatable) pool is refused."""
    keys, off, pay, _ = inputs.segmented(20, seed=44, lo=100, hi=1e4)
    t, o, p = upload(keys, off, pay, dev)
    lsort.sort_segmented(t, o, p, fixed_levels=True, stats=False)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(lsort.LsortError, match="ls_set_workspace"):
        with torch.cuda.graph(g):
            lsort.sort_segmented(t, o, p, fixed_levels=True, stats=False)
    torch.cuda.synchronize()
    del g


def test_capture_needs_fixed_levels(dev):
    """Under stream capture a call must launch a fixed number of levels: the
    read-backs between levels cannot be captured, so a call without
    LS_FLAG_FIXED_LEVELS is refused (with a caller-owned workspace set)."""
    keys, off, pay, _ = inputs.segmented(20, seed=45, lo=100, hi=1e4)
    t, o, p = upload(keys, off, pay, dev)
    nbytes = lsort.workspace_bytes(keys.size, off.size - 1, payload=True)
    ws = torch.empty((nbytes + 7) // 8, dtype=torch.int64, device=dev)
    lsort.set_workspace(ws)
    try:
        lsort.sort_segmented(t, o, p, stats=False)  # set-up outside capture: this layout's look-back words
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with pytest.raises(lsort.LsortError, match="FIXED_LEVELS"):
            with torch.cuda.graph(g):
                lsort.sort_segmented(t, o, p, stats=False)
    finally:
        torch.cuda.synchronize()
        lsort.set_workspace(None)
    del g


def test_c4_prefix_properties(dev):
    """The batched workload (10,000 arrays, sizes log-uniform in [1e3, 1e6],
    five laws, payload) up to its first 2e8 keys: every array sorted, the
    payload stable (ascending among equal keys, as it was the index), and
    (key, payload) pairs the same multiset as the input."""
    keys, off, pay, _ = inputs.segmented(10_000, seed=41, max_total=200_000_000)
    n, m = keys.size, off.size - 1
    t, o, p = upload(keys, off, pay, dev)
    seg = torch.repeat_interleave(torch.arange(m, device=dev),
                                  torch.from_numpy(np.diff(off).astype(np.int64)).to(dev))
    def pair_hash(kk, pp):
        pv = pp.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        return multiset_hash(kk.view(torch.int64) ^ (pv << 17) ^ (seg << 45))
    h0 = pair_hash(t, p)
    print(f"[case] C4 prefix m={m} n={n}", flush=True)
    lsort.sort_segmented(t, o, p)
    torch.cuda.synchronize()
    k = signed_order_key(t)
    same = seg[:-1] == seg[1:]
    assert bool(((k[:-1] <= k[1:]) | ~same).all().item())
    tie = same & (k[:-1] == k[1:])
    pi = p.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    assert bool(((pi[:-1] < pi[1:]) | ~tie).all().item())
    assert pair_hash(t, p) == h0


def test_autotune_table_and_tuned_sort(dev, tmp_path):
    path = str(tmp_path / "tuning.json")
    print("[case] autotune", flush=True)
    lsort.autotune(path)
    try:
        import json
        tab = json.load(open(path))
        assert tab["format"] == "lsort-tuning-1" and len(tab["classes"]) == 6
        for e in tab["classes"]:
            assert e["ms"] <= e["default_ms"] * 1.0001
            assert e["tile"] in (32768, 65536, 131072)
        lsort.load_tuning(path)
        keys, off, pay, _ = inputs.segmented(500, seed=47, lo=1e3, hi=1e5)
        t, o, p = upload(keys, off, pay, dev)
        lsort.sort_segmented(t, o, p, tuned=True)
        torch.cuda.synchronize()
        check(t, p, *oracle.sort_segmented(keys, off, pay))
        single = inputs.generate("lognormal", 2_000_000, seed=48)
        ts = to_dev(single, dev)
        lsort.sort(ts, tuned=True)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(ts).view(np.uint64), oracle.sort(single)[0].view(np.uint64))
    finally:
        lsort.load_tuning(None)
