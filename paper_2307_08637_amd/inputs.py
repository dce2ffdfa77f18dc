"""Seeded synthetic inputs with the shapes and laws of the paper's benchmark.

This module holds no part of the sort's arithmetic: it only draws keys.  It is
the one piece shared by the GPU tests, the oracle tests and the benchmark.

Laws (Sec. 5, synthetic datasets; N = 1e8 float64 in the paper):
  uniform      U[0, 1)                      (the paper uses U[0, N); the scale
                                             does not change the order statistics)
  normal       N(0, 1)
  lognormal    LogNormal(mu=0, sigma=0.5)
  exponential  Exp(rate 2)
  chisquared   chi^2 with k = 4
  mixgauss     equal-weight mixture of five Gaussians, means U[-100, 100],
               sigmas U[1, 10], component drawn per key
  u64          uniform 64-bit unsigned integers
  rootdups     A[i] = i mod floor(sqrt(N)), shuffled
  twodups      A[i] = (i*i + N/2) mod N, shuffled
  zipf         ranks 1..1e6 with P(k) ~ k^-0.75 (inverse CDF; numpy's zipf
               needs an exponent above 1)
  piecewise    70% LogNormal(0, 2), 20% 1e6 + U[0, 1), 10% N(-5e3, 1), per key

Every array is generated in chunks of CHUNK keys from
SeedSequence([seed, chunk index]) with PCG64, so a prefix of a large draw is
reproducible and memory stays bounded.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK = 10_000_000

F64_LAWS = ("normal", "lognormal", "exponential", "chisquared", "mixgauss")
ALL_LAWS = ("uniform",) + F64_LAWS + ("u64", "rootdups", "twodups", "zipf", "piecewise")


def _rng(seed: int, chunk: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, chunk])))


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunked(n: int, seed: int, draw, dtype) -> np.ndarray:
    """Chunk c of the output is drawn from its own stream (seed, c), so the
    chunks are independent: they are filled by a pool of threads (numpy's
    generators release the interpreter lock) with the same result as a
    sequential loop."""
    out = np.empty(n, dtype=dtype)

    def fill(c):
        lo = c * CHUNK
        hi = min(n, lo + CHUNK)
        out[lo:hi] = draw(_rng(seed, c), hi - lo)

    nchunk = (n + CHUNK - 1) // CHUNK
    if nchunk <= 1:
        for c in range(nchunk):
            fill(c)
    else:
        with ThreadPoolExecutor(min(_workers(), nchunk)) as ex:
            list(ex.map(fill, range(nchunk)))
    return out


def _mixgauss_params(seed: int):
    g = _rng(seed, 1 << 30)
    means = g.uniform(-100.0, 100.0, 5)
    sigmas = g.uniform(1.0, 10.0, 5)
    return means, sigmas


_ZIPF_CDF = {}


def _zipf_cdf(K: int = 1_000_000, s: float = 0.75) -> np.ndarray:
    if (K, s) not in _ZIPF_CDF:
        w = np.arange(1, K + 1, dtype=np.float64) ** (-s)
        c = np.cumsum(w)
        _ZIPF_CDF[(K, s)] = c / c[-1]
    return _ZIPF_CDF[(K, s)]


def generate(law: str, n: int, seed: int) -> np.ndarray:
    """Draw n keys of the given law (float64, or uint64 for the integer laws)."""
    if law == "uniform":
        return _chunked(n, seed, lambda g, m: g.random(m), np.float64)
    if law == "normal":
        return _chunked(n, seed, lambda g, m: g.normal(0.0, 1.0, m), np.float64)
    if law == "lognormal":
        return _chunked(n, seed, lambda g, m: g.lognormal(0.0, 0.5, m), np.float64)
    if law == "exponential":
        return _chunked(n, seed, lambda g, m: g.exponential(0.5, m), np.float64)
    if law == "chisquared":
        return _chunked(n, seed, lambda g, m: g.chisquare(4.0, m), np.float64)
    if law == "mixgauss":
        mu, sd = _mixgauss_params(seed)

        def draw(g, m):
            c = g.integers(0, 5, m)
            return g.normal(0.0, 1.0, m) * sd[c] + mu[c]
        return _chunked(n, seed, draw, np.float64)
    if law == "u64":
        return _chunked(n, seed, lambda g, m: g.integers(0, 2**64, m, dtype=np.uint64, endpoint=False), np.uint64)
    if law == "rootdups":
        r = int(math.isqrt(n)) if n > 0 else 1
        a = (np.arange(n, dtype=np.uint64) % np.uint64(max(r, 1)))
        return _rng(seed, 0).permutation(a)
    if law == "twodups":
        i = np.arange(n, dtype=np.uint64)
        a = (i * i + np.uint64(n // 2)) % np.uint64(max(n, 1))
        return _rng(seed, 0).permutation(a)
    if law == "zipf":
        cdf = _zipf_cdf()

        def draw(g, m):
            k = np.searchsorted(cdf, g.random(m), side="right") + 1
            return np.minimum(k, cdf.size).astype(np.uint64)
        return _chunked(n, seed, draw, np.uint64)
    if law == "piecewise":
        def draw(g, m):
            u = g.random(m)
            a = g.lognormal(0.0, 2.0, m)
            b = 1e6 + g.random(m)
            c = g.normal(-5e3, 1.0, m)
            return np.where(u < 0.7, a, np.where(u < 0.9, b, c))
        return _chunked(n, seed, draw, np.float64)
    raise ValueError(f"unknown law {law!r}")


def segmented(m: int, seed: int, lo: float = 1e3, hi: float = 1e6, laws=F64_LAWS, max_total: int | None = None):
    """Batched workload: m arrays with sizes floor(exp(U[ln lo, ln hi])), each
    drawn from a law picked uniformly from `laws`, concatenated.  Returns
    (keys float64, offsets uint64[m+1], payload uint32 = index within its
    array, law index per array).  With max_total, only the leading arrays up
    to the first one at which the running total reaches max_total."""
    g = _rng(seed, 1 << 31)
    sizes = np.floor(np.exp(g.uniform(math.log(lo), math.log(hi), m))).astype(np.int64)
    which = g.integers(0, len(laws), m)
    if max_total is not None:
        cut = int(np.searchsorted(np.cumsum(sizes), max_total)) + 1
        m = min(m, cut)
        sizes, which = sizes[:m], which[:m]
    off = np.zeros(m + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes, dtype=np.uint64)
    keys = np.empty(int(off[-1]), dtype=np.float64)
    payload = np.empty(int(off[-1]), dtype=np.uint32)

    def fill(s):  # array s has its own stream: any order of filling gives the same result
        a, b = int(off[s]), int(off[s + 1])
        keys[a:b] = generate(laws[which[s]], b - a, seed * 100_003 + s)
        payload[a:b] = np.arange(b - a, dtype=np.uint32)

    if m > 16:
        with ThreadPoolExecutor(_workers()) as ex:
            list(ex.map(fill, range(m), chunksize=64))
    else:
        for s in range(m):
            fill(s)
    return keys, off, payload, which


def adversarial(kind: str, n: int, seed: int = 0) -> np.ndarray:
    """Edge-case inputs: degenerate orders, duplicates and extreme values."""
    g = _rng(seed, 7)
    if kind == "all_equal":
        return np.full(n, 0.5)
    if kind == "sorted":
        return np.sort(g.random(n))
    if kind == "reversed":
        return np.sort(g.random(n))[::-1].copy()
    if kind == "organ_pipe":
        h = np.arange(n, dtype=np.float64)
        return np.minimum(h, n - 1 - h)
    if kind == "two_values":
        return np.where(g.random(n) < 0.5, -1.0, 3.0)
    if kind == "signed_zeros":
        return np.where(g.random(n) < 0.5, -0.0, 0.0)
    if kind == "extremes":
        pool = np.array([0.0, -0.0, 5e-324, -5e-324, 2.2250738585072014e-308, -2.2250738585072014e-308,
                         1.7976931348623157e308, -1.7976931348623157e308, np.inf, -np.inf, 1.0, -1.0])
        return pool[g.integers(0, pool.size, n)]
    if kind == "with_nan":
        a = g.normal(0, 1, n)
        pos_nan = np.frombuffer(np.uint64(0x7ff8000000000001).tobytes(), dtype=np.float64)[0]
        neg_nan = np.frombuffer(np.uint64(0xfff8000000000002).tobytes(), dtype=np.float64)[0]
        u = g.random(n)
        a = np.where(u < 0.05, pos_nan, a)
        a = np.where((u >= 0.05) & (u < 0.1), neg_nan, a)
        a = np.where((u >= 0.1) & (u < 0.12), np.inf, a)
        return np.where((u >= 0.12) & (u < 0.14), -np.inf, a)
    if kind == "u64_extremes":
        pool = np.array([0, 1, 2**63 - 1, 2**63, 2**64 - 2, 2**64 - 1], dtype=np.uint64)
        return pool[g.integers(0, pool.size, n)]
    if kind == "u64_collide":
        # distinct integers that all round to the same double
        return (np.uint64(2**60) + g.integers(0, 2**20, n, dtype=np.uint64))
    if kind == "few_distinct":
        return g.integers(0, 7, n).astype(np.float64)
    if kind == "subnormal_mix":
        # subnormals and the smallest normals of both signs, no -0.0 or NaN:
        # bit patterns with a biased exponent of 0..3 and a random mantissa
        bits = g.integers(1, 1 << 52, n, dtype=np.uint64) | (g.integers(0, 4, n, dtype=np.uint64) << np.uint64(52))
        bits |= g.integers(0, 2, n, dtype=np.uint64) << np.uint64(63)
        return bits.view(np.float64)
    if kind == "sparse_specials":
        # normal keys with rare NaNs (both signs), -0.0 and +0.0
        a = g.normal(0, 1, n)
        pos_nan = np.frombuffer(np.uint64(0x7ff0000000000123).tobytes(), dtype=np.float64)[0]
        neg_nan = np.frombuffer(np.uint64(0xfff8000000000000).tobytes(), dtype=np.float64)[0]
        u = g.random(n)
        a = np.where(u < 1e-4, pos_nan, a)
        a = np.where((u >= 1e-4) & (u < 2e-4), neg_nan, a)
        a = np.where((u >= 2e-4) & (u < 3e-4), -0.0, a)
        return np.where((u >= 3e-4) & (u < 4e-4), 0.0, a)
    if kind == "f32_specials":
        # float32 normal keys with every class of special value: NaNs of both
        # signs with payload bits (quiet and signalling), infinities, signed
        # zeros, subnormals and the extreme normals
        a = g.normal(0, 10, n).astype(np.float32)
        pool = np.array([0xFFC00001, 0xFFC00000, 0xFF800001, 0xFF800000, 0xFF7FFFFF, 0x80800000, 0x807FFFFF,
                         0x80000001, 0x80000000, 0x00000000, 0x00000001, 0x007FFFFF, 0x00800000, 0x7F7FFFFF,
                         0x7F800000, 0x7F800001, 0x7FC00000, 0x7FC00001], dtype=np.uint32).view(np.float32)
        sel = g.random(n) < 0.1
        a[sel] = pool[g.integers(0, pool.size, int(sel.sum()))]
        return a
    if kind == "i64_extremes":
        # int64 keys: the full range, the extremes and a heavy run of one small value
        a = g.integers(-2**63, 2**63 - 1, n, dtype=np.int64, endpoint=True)
        ext = np.array([-2**63, -2**63 + 1, -1, 0, 1, 2**63 - 2, 2**63 - 1], dtype=np.int64)
        sel = g.random(n) < 0.1
        a[sel] = ext[g.integers(0, ext.size, int(sel.sum()))]
        a[g.random(n) < 0.2] = -3
        return a
    raise ValueError(kind)


ADVERSARIAL_F64 = ("all_equal", "sorted", "reversed", "organ_pipe", "two_values", "signed_zeros",
                   "extremes", "with_nan", "few_distinct", "subnormal_mix", "sparse_specials")
ADVERSARIAL_U64 = ("u64_extremes", "u64_collide")
