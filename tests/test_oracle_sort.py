"""Pins of the oracle's sort against definitions and library routines.

The oracle must reach the unique result the sort is defined by (Sec. 2.1:
position = number of keys before it; Sec. 2.2: the output must be sorted):
the stable sort in IEEE totalOrder (float64) or numeric order (uint64).
None of these checks reuses the oracle's key transform.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2307_08637_amd import inputs


def bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def f64(u):
    return np.array([u], dtype=np.uint64).view(np.float64)[0]


# IEEE 754-2008 totalOrder (5.10), written out class by class in ascending order.
TOTAL_ORDER = [
    f64(0xFFF8000000000001),   # negative quiet NaN with the larger payload
    f64(0xFFF8000000000000),   # negative quiet NaN
    -np.inf, -1.7976931348623157e308, -1.0, -2.2250738585072014e-308, -2.225073858507201e-308, -5e-324,
    -0.0, 0.0,
    5e-324, 2.225073858507201e-308, 2.2250738585072014e-308, 1.0, 1.7976931348623157e308, np.inf,
    f64(0x7FF8000000000000),   # positive quiet NaN
    f64(0x7FF8000000000001),
]


def test_total_order_classes():
    want = np.array(TOTAL_ORDER)
    rng = np.random.default_rng(0)
    for _ in range(20):
        got, _ = oracle.sort(rng.permutation(want))
        assert np.array_equal(bits(got), bits(want))


@pytest.mark.parametrize("n", [0, 1, 2, 3, 10, 1000, 100_000])
def test_matches_numpy_sort_finite(n):
    rng = np.random.default_rng(n)
    a = rng.normal(0, 1e3, n)
    a = a[a != 0]
    got, _ = oracle.sort(a)
    assert np.array_equal(got, np.sort(a, kind="stable"))
    u = rng.integers(0, 2**64, n, dtype=np.uint64, endpoint=False)
    got, _ = oracle.sort(u)
    assert np.array_equal(got, np.sort(u))


@pytest.mark.parametrize("dtype", ["f64", "u64"])
def test_stable_perm_matches_argsort(dtype):
    rng = np.random.default_rng(1)
    n = 50_000
    if dtype == "f64":
        a = rng.integers(-50, 50, n).astype(np.float64) + 0.5   # duplicates, no zeros
    else:
        a = rng.integers(0, 100, n).astype(np.uint64)
    pay = np.arange(n, dtype=np.uint32)
    got, gp, perm = oracle.sort(a, pay, want_perm=True)
    ref = np.argsort(a, kind="stable")
    assert np.array_equal(perm, ref.astype(np.uint64))
    assert np.array_equal(gp, ref.astype(np.uint32))
    assert np.array_equal(got, a[ref])


def precedes(x, y):
    """x strictly before y in totalOrder, for non-NaN doubles."""
    if x < y:
        return True
    return x == 0 and y == 0 and np.signbit(x) and not np.signbit(y)


def test_dest_closed_form_bruteforce():
    rng = np.random.default_rng(2)
    for n in (1, 2, 7, 64, 500, 2000):
        a = rng.choice(np.array([-3.0, -0.0, 0.0, 1.5, 2.0, 1e300, -1e-300]), n)
        _, _, perm = oracle.sort(a, want_perm=True)
        dest = np.empty(n, dtype=np.int64)
        dest[perm.astype(np.int64)] = np.arange(n)
        for i in range(n):
            before = sum(precedes(a[j], a[i]) for j in range(n))
            ties = sum(1 for j in range(i) if bits(a[j:j + 1])[0] == bits(a[i:i + 1])[0])
            assert dest[i] == before + ties


def test_all_permutations_small():
    alphabet = [-0.0, 0.0, 1.0, 1.0, -2.5, 0.0]
    want = None
    for p in itertools.permutations(range(len(alphabet))):
        a = np.array([alphabet[i] for i in p])
        pay = np.array(p, dtype=np.uint32)
        got, gp = oracle.sort(a, pay)
        if want is None:
            want = bits(got).copy()
        assert np.array_equal(bits(got), want)
        # stable: equal keys keep input order, i.e. payload order within a run
        for v in set(bits(got).tolist()):
            run = gp[bits(got) == v]
            pos = [list(p).index(x) for x in run]
            assert pos == sorted(pos)
    assert np.array_equal(want, bits(np.array([-2.5, -0.0, 0.0, 0.0, 1.0, 1.0])))


@pytest.mark.parametrize("kind", inputs.ADVERSARIAL_F64 + inputs.ADVERSARIAL_U64)
def test_adversarial_invariants(kind):
    a = inputs.adversarial(kind, 20_000, seed=3)
    pay = np.arange(a.size, dtype=np.uint32)
    got, gp = oracle.sort(a, pay)
    # a permutation of the input, with the payload travelling with its key
    assert np.array_equal(np.sort(bits(got)), np.sort(bits(a)))
    assert np.array_equal(bits(a)[gp], bits(got))
    # sorted: non-NaN keys agree with numpy's value order wherever values differ
    if a.dtype == np.float64:
        g = got[~np.isnan(got)]
        assert np.all(g[:-1] <= g[1:])
        nan_sign = np.signbit(got[np.isnan(got)])
        k = int(nan_sign.sum())
        assert np.all(np.isnan(got[:k])) and np.all(np.isnan(got[got.size - (nan_sign.size - k):]))
    else:
        assert np.all(got[:-1] <= got[1:])
    # stable
    b = bits(got)
    same = b[1:] == b[:-1]
    assert np.all(gp[1:][same] > gp[:-1][same])


def test_segmented_matches_per_segment():
    keys, off, pay, _ = inputs.segmented(30, seed=4, lo=1, hi=5000)
    got, gp = oracle.sort_segmented(keys, off, pay)
    for s in range(30):
        a, b = int(off[s]), int(off[s + 1])
        r = np.argsort(keys[a:b], kind="stable")
        assert np.array_equal(got[a:b], keys[a:b][r])
        assert np.array_equal(gp[a:b], pay[a:b][r])


# ---- extra key types (int64, float32) and 64-bit payloads ------------------------

def f32(u):
    return np.array([u], dtype=np.uint32).view(np.float32)[0]


def f32_order(a):
    """int32 whose signed order is IEEE totalOrder of binary32 values: a
    negative value's magnitude bits are reversed so that a larger magnitude
    sorts further down (an independent formula, not the oracle's map)."""
    i = np.ascontiguousarray(a, dtype=np.float32).view(np.int32)
    return np.where(i < 0, i ^ np.int32(0x7FFFFFFF), i)


F32_TOTAL_ORDER = [
    f32(0xFFC00001), f32(0xFFC00000), f32(0xFF800001),   # negative NaNs (quiet, quiet, signalling)
    np.float32(-np.inf), np.float32(-3.4028235e38), np.float32(-1.0), f32(0x80800000), f32(0x807FFFFF),
    f32(0x80000001), np.float32(-0.0), np.float32(0.0), f32(0x00000001), f32(0x007FFFFF), f32(0x00800000),
    np.float32(1.0), np.float32(3.4028235e38), np.float32(np.inf),
    f32(0x7F800001), f32(0x7FC00000), f32(0x7FC00001),  # positive NaNs
]


def bits32(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def test_f32_total_order_classes():
    want = np.array(F32_TOTAL_ORDER, dtype=np.float32)
    assert np.all(np.diff(f32_order(want).astype(np.int64)) > 0)
    rng = np.random.default_rng(10)
    for _ in range(20):
        got, _ = oracle.sort(rng.permutation(want))
        assert got.dtype == np.float32
        assert np.array_equal(bits32(got), bits32(want))


def random_f32_with_specials(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(0, 10, n).astype(np.float32)
    pool = np.array(F32_TOTAL_ORDER, dtype=np.float32)
    sel = rng.random(n) < 0.05
    a[sel] = pool[rng.integers(0, pool.size, int(sel.sum()))]
    a[rng.random(n) < 0.02] = np.float32(-0.0)
    return a


@pytest.mark.parametrize("n", [0, 1, 2, 5, 1000, 60_000])
def test_f32_stable_sort_matches_independent_order(n):
    a = random_f32_with_specials(n, seed=n)
    pay = np.arange(n, dtype=np.uint32)
    got, gp = oracle.sort(a, pay)
    ref = np.argsort(f32_order(a), kind="stable")
    assert np.array_equal(bits32(got), bits32(a)[ref])
    assert np.array_equal(gp, ref.astype(np.uint32))
    # NaN-free, zero-free values: numpy's own float32 sort
    b = a[np.isfinite(a) & (a != 0)]
    got, _ = oracle.sort(b)
    assert np.array_equal(got, np.sort(b, kind="stable"))


def test_f32_dest_closed_form_bruteforce():
    rng = np.random.default_rng(11)
    pool = np.array([-3.0, -0.0, 0.0, 1.5, 2.0, 1e30, -1e-30], dtype=np.float32)
    for n in (1, 2, 9, 300):
        a = rng.choice(pool, n)
        _, _, perm = oracle.sort(a, want_perm=True)
        dest = np.empty(n, dtype=np.int64)
        dest[perm.astype(np.int64)] = np.arange(n)
        key = f32_order(a)
        for i in range(n):
            assert dest[i] == int((key < key[i]).sum()) + int((key[:i] == key[i]).sum())


@pytest.mark.parametrize("n", [1, 3, 1000, 80_000])
def test_i64_matches_numpy(n):
    rng = np.random.default_rng(n + 1)
    a = rng.integers(-2**63, 2**63 - 1, n, dtype=np.int64, endpoint=True)
    ext = np.array([-2**63, -2**63 + 1, -1, 0, 1, 2**63 - 2, 2**63 - 1], dtype=np.int64)
    sel = rng.random(n) < 0.1
    a[sel] = ext[rng.integers(0, ext.size, int(sel.sum()))]
    a[rng.random(n) < 0.3] = rng.integers(-5, 5, 1)[0]   # a run of duplicates
    pay = np.arange(n, dtype=np.uint32)
    got, gp = oracle.sort(a, pay)
    ref = np.argsort(a, kind="stable")
    assert got.dtype == np.int64
    assert np.array_equal(got, a[ref]) and np.array_equal(gp, ref.astype(np.uint32))


@pytest.mark.parametrize("dtype", [np.float64, np.uint64, np.int64, np.float32])
def test_payload64_follows_the_stable_order(dtype):
    rng = np.random.default_rng(12)
    n = 40_000
    a = rng.integers(0, 300, n).astype(dtype)           # many ties
    pay = rng.integers(0, 2**64, n, dtype=np.uint64, endpoint=False)
    got, gp = oracle.sort(a, pay)
    ref = np.argsort(a, kind="stable")
    assert gp.dtype == np.uint64
    assert np.array_equal(got, a[ref]) and np.array_equal(gp, pay[ref])


def test_segmented_f32_i64_payload64():
    rng = np.random.default_rng(13)
    off = np.concatenate([[0], np.cumsum(rng.integers(0, 3000, 25))]).astype(np.uint64)
    n = int(off[-1])
    pay = rng.integers(0, 2**64, n, dtype=np.uint64, endpoint=False)
    for a in (random_f32_with_specials(n, 14), rng.integers(-1000, 1000, n).astype(np.int64)):
        got, gp = oracle.sort_segmented(a, off, pay)
        for s in range(off.size - 1):
            lo, hi = int(off[s]), int(off[s + 1])
            key = f32_order(a[lo:hi]) if a.dtype == np.float32 else a[lo:hi]
            r = np.argsort(key, kind="stable")
            assert np.array_equal(got[lo:hi].view(np.uint8), a[lo:hi][r].view(np.uint8))
            assert np.array_equal(gp[lo:hi], pay[lo:hi][r])
