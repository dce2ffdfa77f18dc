"""GPU parity of the full sort against the CPU oracle (bit-exact).

Every case: seeded synthetic input -> liblsort on cuda:0 through the C ABI ->
compare every output word (keys, and payload where given) with the oracle's
stable sort of the same input.  Large inputs, where the oracle would take too
long, are checked by properties that pin a sort at any size: sortedness in
totalOrder plus equal multisets (count and two independent 64-bit hashes).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2307_08637_amd import inputs, lsort
from tests.gpu_helpers import is_sorted, multiset_hash, signed_order_key, to_dev, to_host

pytestmark = pytest.mark.gpu


def gpu_sort(keys, dev, payload=None, **opts):
    t = to_dev(keys, dev)
    p = None
    if payload is not None:
        p = torch.from_numpy(payload.view(np.int32).copy()).to(dev).view(torch.uint32)
    print(f"[case] n={keys.size} dtype={keys.dtype} payload={payload is not None} opts={opts}", flush=True)
    lsort.sort(t, p, **opts)
    torch.cuda.synchronize()
    out = to_host(t)
    pout = None if p is None else p.view(torch.int32).cpu().numpy().view(np.uint32)
    return out, pout


def assert_same_bits(got, want):
    g = np.ascontiguousarray(got).view(np.uint64)
    w = np.ascontiguousarray(want).view(np.uint64)
    assert g.shape == w.shape
    bad = np.flatnonzero(g != w)
    assert bad.size == 0, f"{bad.size} mismatches, first at {bad[:5]}: got {g[bad[:5]]} want {w[bad[:5]]}"


@pytest.mark.parametrize("n", [0, 1, 2, 3, 17, 255, 256, 257, 4095, 4096, 4097, 8191, 8192, 8193,
                               16385, 50_000, 99_999, 100_000, 250_001])
def test_sizes_uniform(dev, n):
    keys = inputs.generate("uniform", n, seed=11)
    got, _ = gpu_sort(keys, dev)
    want, _ = oracle.sort(keys)
    assert_same_bits(got, want)


@pytest.mark.parametrize("cutoff", [1, 16, 256, 4096])
def test_cutoffs(dev, cutoff):
    keys = inputs.generate("normal", 120_000, seed=12)
    got, _ = gpu_sort(keys, dev, cutoff=cutoff)
    assert_same_bits(got, oracle.sort(keys)[0])


def test_config_small_uniform_1e6(dev):
    """N = 1e6 uniform [0,1) float64, 1000 leaves, 1000 buckets, base case below 256 keys."""
    keys = inputs.generate("uniform", 1_000_000, seed=1)
    got, _ = gpu_sort(keys, dev, buckets=1000, leaves=1000, cutoff=256)
    assert_same_bits(got, oracle.sort(keys)[0])
    st = lsort.stats()
    assert len(st["levels"]) >= 1
    assert st["levels"] and st["levels"][0]["learned"] == 1  # Alg. 5 picks the RMI at n = 1e6


@pytest.mark.parametrize("law", inputs.ALL_LAWS)
def test_laws_1e6(dev, law):
    keys = inputs.generate(law, 1_000_000, seed=21)
    got, _ = gpu_sort(keys, dev)
    assert_same_bits(got, oracle.sort(keys)[0])


@pytest.mark.parametrize("law", ["uniform", "lognormal", "rootdups", "zipf"])
def test_payload_stable(dev, law):
    n = 300_000
    keys = inputs.generate(law, n, seed=31)
    pay = np.arange(n, dtype=np.uint32)
    got, gp = gpu_sort(keys, dev, payload=pay)
    want, wp = oracle.sort(keys, pay)
    assert_same_bits(got, want)
    assert np.array_equal(gp, wp)


@pytest.mark.parametrize("kind", inputs.ADVERSARIAL_F64 + inputs.ADVERSARIAL_U64)
@pytest.mark.parametrize("n", [2, 100, 5000, 70_000, 200_000])
def test_adversarial(dev, kind, n):
    keys = inputs.adversarial(kind, n, seed=5)
    pay = np.arange(n, dtype=np.uint32)
    got, gp = gpu_sort(keys, dev, payload=pay)
    want, wp = oracle.sort(keys, pay)
    assert_same_bits(got, want)
    assert np.array_equal(gp, wp)


@pytest.mark.parametrize("kind", inputs.ADVERSARIAL_F64 + inputs.ADVERSARIAL_U64)
@pytest.mark.parametrize("n", [100, 5000, 200_000, 1_000_003])
def test_adversarial_keys_only(dev, kind, n):
    """Keys only: the base case's lane-group sort (binary64 comparators when
    a wavefront's sub-arrays hold no NaN and no -0.0, ordered integers
    otherwise) against the oracle."""
    keys = inputs.adversarial(kind, n, seed=6)
    got, _ = gpu_sort(keys, dev)
    assert_same_bits(got, oracle.sort(keys)[0])


def test_group_items_every_size(dev):
    """Segments of every size 1..2100 (sorted directly by the base case:
    lane groups of 4..64 lanes up to 2048 keys, the workgroup sort above),
    keys only, with and without special values."""
    sizes = np.tile(np.arange(1, 2101, dtype=np.int64), 2)
    off = np.zeros(sizes.size + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    n = int(off[-1])
    parts = [inputs.generate("normal", n, seed=7), inputs.adversarial("sparse_specials", n, seed=8),
             inputs.adversarial("subnormal_mix", n, seed=9)]
    for keys in parts:
        t = to_dev(keys, dev)
        o = torch.from_numpy(off.view(np.int64)).to(dev).view(torch.uint64)
        print(f"[case] group items n={n}", flush=True)
        lsort.sort_segmented(t, o, cutoff=2100)
        torch.cuda.synchronize()
        want, _ = oracle.sort_segmented(keys, off)
        assert_same_bits(to_host(t), want)
    keys = inputs.generate("u64", n, seed=10)
    t = to_dev(keys, dev)
    o = torch.from_numpy(off.view(np.int64)).to(dev).view(torch.uint64)
    lsort.sort_segmented(t, o, cutoff=2100)
    torch.cuda.synchronize()
    assert_same_bits(to_host(t), oracle.sort_segmented(keys, off)[0])


@pytest.mark.parametrize("pay", [False, True])
def test_few_units_level_recut(dev, pay):
    """A level with fewer work units than CUs (here the second level: three
    first-level buckets of ~1e6 keys each, ~90 units) is re-cut by k_model
    into one-tile units; bit-exact against the oracle, with a payload too."""
    n = 3_000_000
    z = inputs.generate("normal", n, seed=71)
    c = (np.arange(n) % 3).astype(np.float64) * 1e3
    keys = np.where(np.arange(n) % 33 == 0, z * 1e4, c + z * 1e-3)  # three tight clusters, 3 % spread wide
    payload = np.arange(n, dtype=np.uint32) if pay else None
    got, gp = gpu_sort(keys, dev, payload, buckets=64, stats=True)
    st = lsort.stats()
    want, wp = oracle.sort(keys, payload)
    assert_same_bits(got, want)
    if pay:
        assert np.array_equal(gp, wp)
    # the second level's work units (at most keys / 32768 + segments) are fewer than the CUs
    lv1 = st["levels"][1]
    assert lv1["keys"] // 32768 + lv1["segments"] < 256, st["levels"]


def test_u64_items_as_differences(dev):
    """uint64 base-case items whose keys span less than the +inf bit pattern
    sort as binary64 differences key - min (the floating-point network):
    segments of every size 1..2100 with narrow ranges (differences up to
    2^52, subnormal as binary64), mixed with wide segments (handed to the
    workgroup sort), and the boundary spans 0x7fef.. (narrow) and 0x7ff0..
    (wide), against the oracle."""
    rng = np.random.default_rng(14)
    sizes = np.tile(np.arange(1, 2101, dtype=np.int64), 2)
    off = np.zeros(sizes.size + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    n = int(off[-1])
    base = rng.integers(0, 2**63, sizes.size, dtype=np.uint64).repeat(sizes)
    narrow = base + (rng.integers(0, 2**52, n, dtype=np.uint64) >> rng.integers(0, 52, n, dtype=np.uint64))
    wide = rng.integers(0, 2**64 - 1, n, dtype=np.uint64, endpoint=True)
    pick = (np.arange(sizes.size) % 3 == 0).repeat(sizes)  # every third segment wide
    edge = np.array([5, 5 + 0x7FEFFFFFFFFFFFFF, 7, 3, 3 + 0x7FF0000000000000, 9, 2**64 - 1, 0], dtype=np.uint64)
    eoff = np.array([0, 3, 6, 8], dtype=np.uint64)
    for keys, o_h in ((narrow, off), (np.where(pick, wide, narrow), off), (edge, eoff)):
        t = to_dev(keys, dev)
        o = torch.from_numpy(o_h.view(np.int64)).to(dev).view(torch.uint64)
        print(f"[case] u64 items n={keys.size}", flush=True)
        lsort.sort_segmented(t, o, cutoff=2100)
        torch.cuda.synchronize()
        assert_same_bits(to_host(t), oracle.sort_segmented(keys, o_h)[0])


def test_pair_items_every_size(dev):
    """Segments of every size 1..600 with a uint32 payload, sorted directly by
    the base case: the wavefront pair network with 1, 2, 4 and 8 (key, index)
    pairs per lane up to 512 keys (every boundary 64/65 .. 512/513), the
    workgroup sort above; stable on a duplicate-heavy law too."""
    sizes = np.tile(np.arange(1, 601, dtype=np.int64), 2)
    off = np.zeros(sizes.size + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    n = int(off[-1])
    for law in ("normal", "rootdups"):
        keys = inputs.generate(law, n, seed=12)
        pay = np.arange(n, dtype=np.uint32)
        t = to_dev(keys, dev)
        p = torch.from_numpy(pay.view(np.int32).copy()).to(dev).view(torch.uint32)
        o = torch.from_numpy(off.view(np.int64)).to(dev).view(torch.uint64)
        print(f"[case] pair items {law} n={n}", flush=True)
        lsort.sort_segmented(t, o, p, cutoff=600)
        torch.cuda.synchronize()
        want, wp = oracle.sort_segmented(keys, off, pay)
        assert_same_bits(to_host(t), want)
        assert np.array_equal(p.view(torch.int32).cpu().numpy().view(np.uint32), wp)


def _seg_sort_pay(keys, off, dev, **opts):
    """Segmented sort with payload = global index on the device, and the oracle's."""
    pay = np.arange(keys.size, dtype=np.uint32)
    t = to_dev(keys, dev)
    p = torch.from_numpy(pay.view(np.int32).copy()).to(dev).view(torch.uint32)
    o = torch.from_numpy(off.view(np.int64)).to(dev).view(torch.uint64)
    print(f"[case] packed pairs n={keys.size} dtype={keys.dtype} segments={off.size - 1} opts={opts}", flush=True)
    lsort.sort_segmented(t, o, p, **opts)
    torch.cuda.synchronize()
    want, wp = oracle.sort_segmented(keys, off, pay)
    assert_same_bits(to_host(t), want)
    assert np.array_equal(p.view(torch.int32).cpu().numpy().view(np.uint32), wp)


def test_pair_items_packed(dev):
    """Payload items whose keys span less than 2^(56 - log2 pairs per lane)
    sort as packed binary64 values (key - min) * 2^IB + index in the numeric
    network, wider ones by the pair network; both must give the stable order.
    uint64 segments of every size 1..600 with spans 2^0 .. 2^63 (either side
    of every class's limit 2^56 / 2^55 / 2^54 / 2^53 / 2^52), spans at and
    just past each limit with both extremes present, and duplicate-heavy
    segments (ties decided by the index bits)."""
    rng = np.random.default_rng(15)
    sizes = np.tile(np.arange(1, 601, dtype=np.int64), 3)
    off = np.zeros(sizes.size + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    n = int(off[-1])
    span_bits = rng.integers(0, 64, sizes.size).repeat(sizes)
    base = rng.integers(0, 2**63, sizes.size, dtype=np.uint64).repeat(sizes)
    r = rng.integers(0, 2**64 - 1, n, dtype=np.uint64, endpoint=True)
    keys = base + (r >> (np.uint64(64) - span_bits.astype(np.uint64)).clip(0, 63))
    dups = (np.arange(sizes.size) % 5 == 0).repeat(sizes)  # every fifth segment: four distinct values
    keys = np.where(dups, base + (r & np.uint64(3)), keys)
    _seg_sort_pay(keys, off, dev, cutoff=600)
    # each class's limit: span 2^L - 1 (packed) and 2^L, 2^(L+1) (pair network)
    segs = []
    for size, lim in ((64, 56), (128, 55), (256, 54), (512, 53), (40, 56), (500, 53)):
        for span in (2**lim - 1, 2**lim, 2**(lim + 1), 2**63 + 5):
            lo = int(rng.integers(0, 2**64 - span, dtype=np.uint64, endpoint=True))
            v = lo + rng.integers(0, span, size, dtype=np.uint64, endpoint=True)
            v[rng.permutation(size)[:4]] = np.array([lo, lo, lo + span, lo + span], dtype=np.uint64)
            segs.append(v)
    keys = np.concatenate(segs)
    off = np.zeros(len(segs) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([v.size for v in segs])
    _seg_sort_pay(keys, off, dev, cutoff=600)


@pytest.mark.parametrize("law", ["narrow_f64", "narrow_u64", "zero_mix"])
def test_pair_items_packed_levels(dev, law):
    """The same after partition levels: segments of 2e3..3e4 keys with a
    payload, whose buckets reach the base case as items of up to 512 keys,
    items and 1024-key chunks of 513..1024 (one wavefront each), and chunk
    merges.  Narrow float64 segments (one binade: packed), narrow uint64 ones,
    and float64 keys around zero with -0.0, subnormals and NaN (the buckets
    spanning zero take the pair network)."""
    rng = np.random.default_rng(16)
    sizes = rng.integers(2000, 30000, 40)
    off = np.zeros(sizes.size + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    n = int(off[-1])
    if law == "narrow_f64":
        c = rng.uniform(1.0, 2.0, sizes.size).repeat(sizes)
        keys = c * (1.0 + rng.uniform(0.0, 1e-3, n))
        keys[rng.random(n) < 0.2] = 1.5  # ties across the payload
    elif law == "narrow_u64":
        keys = rng.integers(0, 2**60, sizes.size, dtype=np.uint64).repeat(sizes) + rng.integers(0, 2**44, n,
                                                                                              dtype=np.uint64)
    else:
        keys = rng.normal(0.0, 1e-300, n) * rng.choice([1.0, 1e-8, 1e300], n)
        keys[rng.random(n) < 0.05] = -0.0
        keys[rng.random(n) < 0.05] = 0.0
        keys[rng.random(n) < 0.01] = np.nan
    _seg_sort_pay(keys, off, dev)


@pytest.mark.parametrize("kind,n,buckets", [("uniform", 200_000, 40), ("normal", 300_000, 64), ("u64", 250_000, 40),
                                             ("lognormal", 400_000, 100), ("sparse_specials", 200_000, 40),
                                             ("subnormal_mix", 150_000, 32), ("few_distinct", 200_000, 40)])
def test_split_merge_items(dev, kind, n, buckets):
    """Keys-only base-case items of 2049..8192 keys (first-level buckets of a
    few thousand keys): sorted as chunks of 2048 keys (the register group
    sort; chunks holding NaN / -0.0 by the workgroup sort), then merged in
    LDS.  Bit-exact against the oracle; the statistics say merges ran."""
    if kind in inputs.ALL_LAWS:
        keys = inputs.generate(kind, n, seed=61)
    else:
        keys = inputs.adversarial(kind, n, seed=61)
    got, _ = gpu_sort(keys, dev, buckets=buckets, stats=True)
    st = lsort.stats()
    assert_same_bits(got, oracle.sort(keys)[0])
    if kind not in ("few_distinct", "subnormal_mix"):  # those laws leave no bucket of that size
        assert st["merged_items"] > 0, st


@pytest.mark.parametrize("kind,n,buckets", [("normal", 300_000, 64), ("uniform", 200_000, 40), ("rootdups", 400_000, 64),
                                             ("twodups", 300_000, 50), ("sparse_specials", 200_000, 40),
                                             ("u64", 250_000, 200), ("lognormal", 500_000, 600)])
def test_split_merge_with_payload(dev, kind, n, buckets):
    """With a payload: base-case items of 513..8192 keys sorted as 1024-key
    chunks (a wavefront's stable pair sort), then merged stably in LDS (ties
    to the earlier run).  Keys and payload bit-exact against the oracle's
    stable sort, also on duplicate-heavy laws; the statistics say merges ran
    where buckets exceed one chunk."""
    keys = inputs.generate(kind, n, seed=62) if kind in inputs.ALL_LAWS else inputs.adversarial(kind, n, seed=62)
    pay = np.arange(keys.size, dtype=np.uint32)
    got, gp = gpu_sort(keys, dev, pay, buckets=buckets, stats=True)
    st = lsort.stats()
    want, wp = oracle.sort(keys, pay)
    assert_same_bits(got, want)
    assert np.array_equal(gp, wp)
    if kind in ("normal", "uniform"):
        assert st["merged_items"] > 0, st


def test_split_merge_segmented_sizes(dev):
    """Segmented arrays whose first-level buckets cover 2049..8192 keys, next
    to arrays small enough for the register sort, in one call."""
    rng = np.random.default_rng(63)
    sizes = np.concatenate([rng.integers(20_000, 120_000, 12), rng.integers(1, 2100, 40)]).astype(np.int64)
    rng.shuffle(sizes)
    off = np.zeros(sizes.size + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    keys = inputs.generate("normal", int(off[-1]), seed=64)
    t = to_dev(keys, dev)
    o = torch.from_numpy(off.view(np.int64)).to(dev).view(torch.uint64)
    print(f"[case] split/merge segmented n={keys.size} m={sizes.size}", flush=True)
    lsort.sort_segmented(t, o, buckets=16, stats=True)
    torch.cuda.synchronize()
    st = lsort.stats()
    assert_same_bits(to_host(t), oracle.sort_segmented(keys, off)[0])
    assert st["merged_items"] > 0, st


@pytest.mark.parametrize("pay", [False, True])
def test_merge_size_classes(dev, pay):
    """Thousands of chunk-and-merge items (600 arrays of 2e4..1.2e5 keys, 16
    first-level buckets each: buckets of ~1e3..8e3 keys), so that the merges
    run as one launch per size class (up to 2048 keys, 2049..4096,
    4097..8192) rather than one launch for all; keys (and payload) against
    the oracle."""
    rng = np.random.default_rng(65)
    sizes = rng.integers(20_000, 120_000, 600).astype(np.int64)
    off = np.zeros(sizes.size + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    n = int(off[-1])
    keys = inputs.generate("lognormal", n, seed=66)
    t = to_dev(keys, dev)
    o = torch.from_numpy(off.view(np.int64)).to(dev).view(torch.uint64)
    pay_h = np.arange(n, dtype=np.uint32) if pay else None
    p = torch.from_numpy(pay_h.view(np.int32).copy()).to(dev).view(torch.uint32) if pay else None
    print(f"[case] merge size classes n={n} pay={pay}", flush=True)
    lsort.sort_segmented(t, o, p, buckets=16, stats=True)
    torch.cuda.synchronize()
    st = lsort.stats()
    want, wp = oracle.sort_segmented(keys, off, pay_h)
    assert_same_bits(to_host(t), want)
    if pay:
        assert np.array_equal(p.view(torch.int32).cpu().numpy().view(np.uint32), wp)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert st["merged_items"] >= 4 * cus, st  # at the class-launch form's threshold or above


@pytest.mark.parametrize("law", ["uniform", "normal", "rootdups", "u64"])
def test_splitter_model(dev, law):
    keys = inputs.generate(law, 400_000, seed=41)
    got, _ = gpu_sort(keys, dev, model="splitter")
    assert_same_bits(got, oracle.sort(keys)[0])
    st = lsort.stats()
    assert st["levels"][0]["learned"] == 0


def test_no_fallback_and_small_buckets(dev):
    keys = inputs.generate("lognormal", 500_000, seed=42)
    got, _ = gpu_sort(keys, dev, no_fallback=True, buckets=64, leaves=32)
    assert_same_bits(got, oracle.sort(keys)[0])


def test_depth_cap_radix(dev):
    # a one-level cap with a 4-way tree leaves buckets of ~1e5 keys, which the
    # range radix (8 bits per level) must finish
    keys = inputs.generate("twodups", 400_000, seed=43)
    got, _ = gpu_sort(keys, dev, max_levels=1, cutoff=64, model="splitter", tree_buckets=4)
    assert_same_bits(got, oracle.sort(keys)[0])
    st = lsort.stats()
    assert any(lv["radix"] > 0 for lv in st["levels"])


def test_repeat_deterministic(dev):
    keys = inputs.generate("mixgauss", 700_000, seed=44)
    a, _ = gpu_sort(keys, dev)
    b, _ = gpu_sort(keys, dev)
    assert_same_bits(a, b)


@pytest.mark.parametrize("law", ["uniform", "normal", "u64", "twodups"])
def test_large_1e7_oracle(dev, law):
    keys = inputs.generate(law, 10_000_000, seed=51)
    got, _ = gpu_sort(keys, dev)
    assert_same_bits(got, oracle.sort(keys)[0])


@pytest.mark.parametrize("law,n,buckets,pay", [("normal", 20_000_000, 100, True), ("exponential", 3_000_000, 0, False),
                                                ("u64", 12_000_000, 60, False)])
def test_refit_per_bucket(dev, law, n, buckets, pay):
    """Every bucket that needs another level gets a model of its own (fresh
    sample and fit, the policy deciding): every output word equal to the
    oracle's, and the children of the large cases are learned models."""
    keys = inputs.generate(law, n, seed=n % 89)
    payload = np.arange(n, dtype=np.uint32) if pay else None
    got, gp = gpu_sort(keys, dev, payload, refit=True, buckets=buckets)
    st = lsort.stats()["levels"]
    if buckets:
        assert len(st) >= 2 and st[1]["learned"] > 0, st[:2]
    want, wp = oracle.sort(keys, payload)
    assert_same_bits(got, want)
    if pay:
        assert np.array_equal(gp, wp)


@pytest.mark.parametrize("law,n,pay", [("normal", 10_000_000, False), ("lognormal", 10_000_000, True),
                                       ("u64", 12_000_000, True), ("exponential", 20_000_000, False),
                                       ("uniform", 1_700_001, True)])
def test_model_base_case(dev, law, n, pay):
    """Base case by the model's placement (counting sort on the RMI's fine
    position, then each key's rank inside its bin): every output word equal
    to the oracle's, and from 1e7 keys (second-level buckets of 64..1024
    keys) most keys went through that kernel."""
    keys = inputs.generate(law, n, seed=n % 83)
    payload = np.arange(n, dtype=np.uint32) if pay else None
    lsort.timing(True)
    try:
        got, gp = gpu_sort(keys, dev, payload, model_base=True)
        rec = lsort.timing_read()
    finally:
        lsort.timing(False)
    if n >= 10_000_000:
        assert rec.get("k_base_model", {}).get("keys", 0) > 0.5 * n, rec.get("k_base_model")
    want, wp = oracle.sort(keys, payload)
    assert_same_bits(got, want)
    if pay:
        assert np.array_equal(gp, wp)


@pytest.mark.parametrize("kind", ["sparse_specials", "with_nan", "few_distinct", "signed_zeros", "subnormal_mix"])
def test_model_base_case_adversarial(dev, kind):
    """Specials, heavy duplicates (bins beyond the limit go to the
    comparison sort) and signed zeros under the model-placed base case."""
    n = 12_000_000
    keys = inputs.adversarial(kind, n, seed=19)
    payload = np.arange(n, dtype=np.uint32)
    got, gp = gpu_sort(keys, dev, payload, model_base=True)
    want, wp = oracle.sort(keys, payload)
    assert_same_bits(got, want)
    assert np.array_equal(gp, wp)


@pytest.mark.parametrize("pct", [0, 50, 100, 1])
def test_first_level_balance_judge(dev, pct):
    """The 70/20/10 piecewise law: its fitted RMI puts most of the sample in
    oversized buckets, so at 50 % (the default, pct 0) the first level takes
    the splitter tree; with the check off (100) the RMI stays, and the normal
    law keeps its RMI at 50 %.  Output equal to the oracle's either way (at
    1 % whichever model the check picks)."""
    for law, n in (("piecewise", 4_000_000), ("normal", 3_000_000)):
        keys = inputs.generate(law, n, seed=23)
        payload = np.arange(n, dtype=np.uint32)
        got, gp = gpu_sort(keys, dev, payload, balance_pct=pct)
        first = lsort.stats()["first_model"]
        if law == "piecewise":
            assert first == (lsort.MODEL["rmi"] if pct == 100 else lsort.MODEL["splitter"]), first
        elif pct != 1:
            assert first == lsort.MODEL["rmi"], first
        want, wp = oracle.sort(keys, payload)
        assert_same_bits(got, want)
        assert np.array_equal(gp, wp)


@pytest.mark.parametrize("tile", [65536, 131072, 524288])
@pytest.mark.parametrize("law,n,pay", [("normal", 2_500_000, False), ("u64", 700_003, True),
                                       ("lognormal", 3_000_017, True)])
def test_tile_option(dev, tile, law, n, pay):
    """Larger first-level work units (the carry spans more tiles, several
    units and a ragged last one): every output word equal to the oracle's."""
    keys = inputs.generate(law, n, seed=n % 97)
    payload = np.arange(n, dtype=np.uint32) if pay else None
    got, gp = gpu_sort(keys, dev, payload, tile=tile)
    want, wp = oracle.sort(keys, payload)
    assert_same_bits(got, want)
    if pay:
        assert np.array_equal(gp, wp)


@pytest.mark.parametrize("law", ["normal", "lognormal", "exponential"])
def test_first_level_fallback_trees(dev, law):
    """A large array's oversized first-level buckets (above 2x the expected
    size) get splitter trees whose sample is the sorted first-level sample's
    run in the bucket: the path must run (fallbacks at level 0, trees at level
    1) and the output must equal the oracle's bit for bit."""
    keys = inputs.generate(law, 5_000_000, seed=71)
    got, _ = gpu_sort(keys, dev, buckets=1000, fallback_ratio=1.5)
    st = lsort.stats()["levels"]
    assert st[0]["learned"] == 1 and st[0]["fallback"] > 0, st[0]
    assert st[1]["tree"] >= st[0]["fallback"], st[1]
    assert_same_bits(got, oracle.sort(keys)[0])


@pytest.mark.parametrize("law", ["uniform", "normal", "lognormal", "exponential", "chisquared", "mixgauss", "u64",
                                 "rootdups", "twodups", "zipf"])
def test_full_size_1e8_properties(dev, law):
    """Full benchmark size (1e8 keys) in the benchmark's launch configuration:
    sorted in totalOrder, the same multiset as the input (count and two
    64-bit hashes), and at sampled output positions i the value's rank in the
    input satisfies #{keys < v} <= i < #{keys <= v} (the sorted-position
    definition, counted directly)."""
    n = 100_000_000
    keys = inputs.generate(law, n, seed=61)
    t = to_dev(keys, dev)
    src = signed_order_key(t.clone())
    h1, h2 = multiset_hash(t), multiset_hash(t, salt=0x5A5A5A5A5A5A5A5)
    print(f"[case] 1e8 {law}", flush=True)
    lsort.sort(t)
    torch.cuda.synchronize()
    assert t.numel() == n
    assert is_sorted(t)
    assert multiset_hash(t) == h1 and multiset_hash(t, salt=0x5A5A5A5A5A5A5A5) == h2
    out = signed_order_key(t)
    for i in np.random.default_rng(0).integers(0, n, 16).tolist() + [0, n - 1]:
        v = out[i]
        lt = int((src < v).sum().item())
        le = int((src <= v).sum().item())
        assert lt <= i < le, (i, lt, le)
    del t, src, out


def test_segmented_small(dev):
    rng = np.random.default_rng(3)
    sizes = np.array([0, 1, 2, 5, 300, 4096, 4097, 9000, 0, 70_000, 1, 250_000, 33], dtype=np.int64)
    off = np.zeros(sizes.size + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    keys = np.concatenate([inputs.generate(["uniform", "normal", "lognormal"][i % 3], int(s), seed=100 + i)
                           for i, s in enumerate(sizes)])
    pay = np.concatenate([np.arange(s, dtype=np.uint32) for s in sizes])
    t = to_dev(keys, dev)
    p = torch.from_numpy(pay.view(np.int32).copy()).to(dev).view(torch.uint32)
    o = torch.from_numpy(off.view(np.int64)).to(dev).view(torch.uint64)
    lsort.sort_segmented(t, o, p)
    torch.cuda.synchronize()
    want, wp = oracle.sort_segmented(keys, off, pay)
    assert_same_bits(to_host(t), want)
    assert np.array_equal(p.view(torch.int32).cpu().numpy().view(np.uint32), wp)
    del rng


@pytest.mark.parametrize("m", [1, 7, 200])
def test_segmented_laws(dev, m):
    keys, off, pay, _ = inputs.segmented(m, seed=77, lo=10, hi=2e5)
    t = to_dev(keys, dev)
    p = torch.from_numpy(pay.view(np.int32).copy()).to(dev).view(torch.uint32)
    o = torch.from_numpy(off.view(np.int64)).to(dev).view(torch.uint64)
    lsort.sort_segmented(t, o, p)
    torch.cuda.synchronize()
    want, wp = oracle.sort_segmented(keys, off, pay)
    assert_same_bits(to_host(t), want)
    assert np.array_equal(p.view(torch.int32).cpu().numpy().view(np.uint32), wp)


def test_errors(dev):
    t = torch.zeros(10, dtype=torch.int32, device=dev)
    with pytest.raises(TypeError):
        lsort.sort(t)
    k = torch.zeros(10, dtype=torch.float64, device=dev)
    with pytest.raises(lsort.LsortError):
        lsort.sort(k, buckets=5000)
    with pytest.raises(lsort.LsortError):
        lsort.sort(k, tree_buckets=100)
