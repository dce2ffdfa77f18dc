"""The integer form of the RMI bucket that the GPU partition kernels evaluate
equals the stored double form bit for bit (CPU, no GPU).

The stored form (Sec. 2.1 formula, Sec. 4 clamp intervals; the oracle's
rmi_buckets) is
    j = clamp(floor(fma(a_r, x, b_r)), 0, L-1)
    g = clamp(floor(clamp(fma(a_j, x, b_j), c_j, d_j)), 0, R-1).
The kernels use
    j = min(cvt(fma(a_r, x, b_r)), L-1)
    g = med3(cvt(fma(a_j, x, b_j)), lo_j, hi_j)
with cvt the saturating, truncating conversion to uint32 (NaN to 0),
lo_j = G(c_j), hi_j = G(d_j), G(y) = clamp(floor(y), 0, R-1) (a NaN bound
clamps nothing; c_j > d_j leaves only G(d_j)).  Here the integer form is
written out with numpy and compared with the oracle on fitted models and on
parameter tables chosen to reach every clamp: negative, huge and infinite
line values, NaN and crossed bounds.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2307_08637_amd import inputs


def fma(a: float, x: float, b: float) -> float:
    """a * x + b rounded once (exact rational arithmetic, then one rounding)."""
    if not (math.isfinite(a) and math.isfinite(x) and math.isfinite(b)):
        return a * x + b
    v = Fraction(a) * Fraction(x) + Fraction(b)
    try:
        return float(v)
    except OverflowError:
        return math.inf if v > 0 else -math.inf


def cvt_u32(v: float) -> int:
    """Saturating truncation to uint32; NaN to 0."""
    if v != v or v <= 0.0:
        return 0
    if v >= 4294967295.0:
        return 4294967295
    return int(math.trunc(v))


def leaf_range(c: float, d: float, R: float):
    rm1 = R - 1.0
    c = -math.inf if c != c else c
    d = math.inf if d != d else d
    lo = int(min(max(math.floor(c), 0.0), rm1)) if math.isfinite(c) else (0 if c < 0 else int(rm1))
    hi = int(min(max(math.floor(d), 0.0), rm1)) if math.isfinite(d) else (0 if d < 0 else int(rm1))
    return min(lo, hi), hi


def integer_form(scaled: np.ndarray, L: int, R: float, keys: np.ndarray) -> np.ndarray:
    out = np.empty(keys.size, dtype=np.uint32)
    raw = keys.view(np.uint64)
    for n, x in enumerate(keys.astype(np.float64)):
        if not math.isfinite(x):  # first / last bucket by sign
            out[n] = 0 if (int(raw[n]) >> 63) else int(R - 1.0)
            continue
        j = min(cvt_u32(fma(scaled[0], x, scaled[1])), L - 1)
        a, b, c, d = scaled[2 + 4 * j: 6 + 4 * j]
        lo, hi = leaf_range(c, d, R)
        t = cvt_u32(fma(a, x, b))
        out[n] = min(max(t, lo), hi)  # med3 with lo <= hi
    return out


def check(scaled, L, R, keys):
    want = oracle.rmi_buckets(scaled, L, R, keys)
    got = integer_form(scaled, L, R, keys)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, (bad[:5], got[bad[:5]], want[bad[:5]])


@pytest.mark.parametrize("law", ["normal", "lognormal", "mixgauss"])
def test_fitted_models(law):
    keys = inputs.generate(law, 20_000, seed=3)
    smp = np.sort(keys[:2000])
    for L, R in ((16, 64.0), (100, 1000.0 * 512), (1000, 1000.0)):
        _, scaled, _ = oracle.rmi_fit(smp, L, R)
        check(scaled, L, R, keys[:4000])


def test_clamps_and_special_bounds():
    rng = np.random.default_rng(5)
    L, R = 8, 50.0
    xs = np.concatenate([rng.normal(0, 3, 3000), [0.0, -0.0, 1e300, -1e300, 5e-324]])
    keys = np.concatenate([xs, [np.inf, -np.inf, np.nan, -np.nan]])
    for trial in range(40):
        p = np.empty(2 + 4 * L)
        p[0] = rng.choice([0.0, 1.0, 1e6, -2.0, 1e300])
        p[1] = rng.choice([0.0, 3.5, -10.0, 4.0])
        for j in range(L):
            a = rng.choice([0.0, 1.0, 7.3, 1e12, 1e308])
            b = rng.choice([-5.0, 0.0, 12.5, 1e9])
            c = rng.choice([0.0, 3.0, 17.9, 49.99, 50.0, np.nan, -np.inf, 1e20])
            d = rng.choice([0.0, 10.0, 25.5, 50.0, 60.0, np.nan, np.inf, -3.0])
            p[2 + 4 * j: 6 + 4 * j] = (a, b, c, d)
        check(p, L, R, keys)
