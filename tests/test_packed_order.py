"""The packed forms the GPU base case sorts with its binary64 network order
exactly as the values they stand for (CPU, no GPU).

Keys-only uint64 items are sorted as the bit patterns key - min when
max - min is below 0x7ff0...0 (the +inf pattern); payload items as
(ordered key - min) * 2^IB + index, IB = log2(pairs per lane) + 6, when the
span is below 2^(62 - IB).  Both rest on IEEE 754: finite non-negative
binary64 numbers, subnormals and zero included, order as their bit
patterns.  Here a numeric sort of the patterns read as float64 is checked
against the integer sort of the same patterns, and the stable (key, index)
order is recovered from packed values, at random spans and at each limit.
"""
import numpy as np
import pytest

PINF = np.uint64(0x7FF0000000000000)


def numeric_order(bits: np.ndarray) -> np.ndarray:
    """Sort bit patterns by the binary64 numbers they encode."""
    return np.sort(bits.view(np.float64), kind="stable").view(np.uint64)


def test_finite_nonnegative_patterns_order_as_integers():
    rng = np.random.default_rng(1)
    parts = [rng.integers(0, 1 << 52, 20_000, dtype=np.uint64),            # subnormals and zero
             rng.integers(0, int(PINF), 20_000, dtype=np.uint64),          # any finite non-negative
             np.array([0, 1, (1 << 52) - 1, 1 << 52, int(PINF) - 1], dtype=np.uint64)]
    bits = np.concatenate(parts)
    assert not np.isnan(bits.view(np.float64)).any() and np.isfinite(bits.view(np.float64)).all()
    assert np.array_equal(numeric_order(bits), np.sort(bits))


def test_pads_sort_after_every_packed_value():
    bits = np.array([int(PINF) - 1, 0, 12345], dtype=np.uint64)
    assert np.array_equal(numeric_order(np.concatenate([[PINF], bits]))[-1:], [PINF])


@pytest.mark.parametrize("le", [0, 1, 2, 3, 4])
def test_packed_pairs_give_the_stable_order(le):
    """Items of 64 * 2^le (key, index) pairs: random keys within each span
    class up to the limit 2^(62 - IB) - 1, many equal keys; packing, a numeric
    sort and unpacking give the stable order of the pairs."""
    ib = le + 6
    n = 64 << le
    rng = np.random.default_rng(10 + le)
    for span_bits in (0, 3, 20, 40, 62 - ib):
        span = (1 << span_bits) - 1 if span_bits else 0
        base = int(rng.integers(0, 1 << 63))
        keys = np.uint64(base) + rng.integers(0, span, n, dtype=np.uint64, endpoint=True)
        keys[rng.permutation(n)[: n // 4]] = np.uint64(base)  # duplicates: ties decided by the index
        keys[0] = np.uint64(base + span)                       # both ends of the span present
        mn = keys.min()
        assert int(keys.max() - mn) >> (62 - ib) == 0
        idx = np.arange(n, dtype=np.uint64)
        packed = ((keys - mn) << np.uint64(ib)) | idx
        assert (packed < np.uint64(1 << 62)).all()
        out = numeric_order(packed)
        got_keys = mn + (out >> np.uint64(ib))
        got_idx = out & np.uint64((1 << ib) - 1)
        want = np.lexsort((idx, keys))
        assert np.array_equal(got_idx, idx[want]) and np.array_equal(got_keys, keys[want])


@pytest.mark.parametrize("le", [0, 4])
def test_span_limit(le):
    """At the first span the payload path refuses, the packed value could
    reach 2^62 and beyond: the test the kernel makes rejects exactly those."""
    ib = le + 6
    limit = 1 << (62 - ib)
    assert ((limit - 1) >> (62 - ib)) == 0 and (limit >> (62 - ib)) != 0
    assert ((limit - 1) << ib | ((1 << ib) - 1)) < (1 << 62)
