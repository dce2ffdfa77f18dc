"""Pins of the oracle's per-step functions (sampling, policy, RMI, splitter
tree, range radix, partition, MLP, pivot quality) against closed forms,
library routines, invariants and brute force -- never against a retyped copy
of the oracle's own formula."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2307_08637_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for ln in f:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                rows.append(ln.split())
    return rows


# -- sampling ---------------------------------------------------------------------

def test_splitmix64_reference_outputs():
    for k, hx in read_golden("splitmix64_seed0.txt"):
        assert oracle.splitmix64_at(0, int(k)) == int(hx, 16)


def test_splitmix64_sequence_is_counter_based():
    # output k from state s equals output 0 from state s + k * golden increment
    g = 0x9E3779B97F4A7C15
    for s in (0, 1, 12345, 2**63 + 7):
        for k in (1, 2, 1000):
            assert oracle.splitmix64_at(s, k) == oracle.splitmix64_at((s + k * g) % 2**64, 0)


def test_sample_index_range_and_uniformity():
    n, S = 1000, 200_000
    idx = np.array([oracle.sample_index(77, k, n) for k in range(S)])
    assert idx.min() >= 0 and idx.max() < n
    counts = np.bincount(idx // 10, minlength=100)
    chi2 = ((counts - S / 100) ** 2 / (S / 100)).sum()
    assert chi2 < 200  # 99 dof; p ~ 1e-8 bound
    assert all(oracle.sample_index(5, k, 1) == 0 for k in range(100))


def test_sample_gathers_indexed_keys():
    keys = np.arange(5000, dtype=np.uint64) * 3
    s = oracle.sample(keys, 9, 300)
    want = np.array([keys[oracle.sample_index(9, k, 5000)] for k in range(300)], dtype=np.uint64)
    assert np.array_equal(s, want)


# -- duplicates and policy (Alg. 5) -------------------------------------------------

def test_dup_fraction_bruteforce():
    rng = np.random.default_rng(0)
    for _ in range(50):
        a = np.sort(rng.integers(0, 5, rng.integers(2, 30)).astype(np.float64))
        d = sum(1 for j in range(1, a.size) if a[j] == a[j - 1]) / (a.size - 1)
        assert oracle.dup_fraction(a) == pytest.approx(d, abs=0)
    z = np.array([-0.0, 0.0])  # distinct in totalOrder
    assert oracle.dup_fraction(z) == 0.0


def test_policy_alg5():
    s = np.sort(np.random.default_rng(1).random(1000))
    assert oracle.policy_learned(200_000, s)
    assert not oracle.policy_learned(99_999, s)                     # small input -> tree
    dup = np.sort(np.concatenate([s[:800], np.full(200, 0.5)]))
    assert not oracle.policy_learned(200_000, dup)                  # > 10% duplicates -> tree
    assert not oracle.policy_learned(200_000, np.append(s[:-1], np.inf))
    assert not oracle.policy_learned(200_000, np.full(10, 1.0))


# -- RMI --------------------------------------------------------------------------------

def leaf_lines(raw, L):
    q = raw[2:].reshape(L, 4)
    return q[:, 0], q[:, 1], q[:, 2], q[:, 3]


def test_rmi_root_closed_form_arithmetic_progression():
    for S in (10, 1000, 12345):
        x = np.arange(S, dtype=np.float64)
        raw, _, _ = oracle.rmi_fit(x, 16, 1000.0)
        assert raw[0] == pytest.approx(1.0 / S, rel=1e-12)      # y = i/S = x/S exactly
        assert abs(raw[1]) < 1e-12


@pytest.mark.parametrize("c,d", [(2.5, -7.0), (1e-3, 1e6), (3.0, 0.0)])
def test_rmi_linear_data_perfect_fit(c, d):
    S, L = 4000, 50
    x = c * np.arange(S) + d
    raw, _, counts = oracle.rmi_fit(x, L, 100.0)
    assert raw[0] == pytest.approx(1 / (c * S), rel=1e-9)
    assert raw[1] == pytest.approx(-d / (c * S), rel=1e-9, abs=1e-12)
    a, b, lo_c, hi_d = leaf_lines(raw, L)
    for j in np.flatnonzero(counts >= 2):
        assert a[j] == pytest.approx(1 / (c * S), rel=1e-7)


@pytest.mark.parametrize("law", ["uniform", "lognormal", "normal", "mixgauss", "u64"])
def test_rmi_leaves_match_polyfit(law):
    S, L = 20_000, 200
    s = oracle.sort(inputs.generate(law, S, seed=3))[0]
    x = oracle.model_x(s)
    raw, sc, counts = oracle.rmi_fit(x, L, 1000.0)
    # root = numpy least squares on (x, i/S)
    y = np.arange(S) / S
    ra, rb = np.polyfit(x - x.mean(), y, 1)
    assert raw[0] == pytest.approx(max(ra, 0.0), rel=1e-8)
    assert raw[1] + raw[0] * x.mean() == pytest.approx(rb, rel=1e-8, abs=1e-12)
    a, b, c, d = leaf_lines(raw, L)
    lo = 0
    for j in range(L):
        k = int(counts[j])
        if k >= 3 and np.ptp(x[lo:lo + k]) > 0:
            xs = x[lo:lo + k]
            sa, sb = np.polyfit(xs - xs.mean(), y[lo:lo + k], 1)
            assert a[j] == pytest.approx(max(sa, 0.0), rel=1e-6, abs=1e-12 / max(np.ptp(xs), 1e-300))
        lo += k
    assert counts.sum() == S


@pytest.mark.parametrize("law", ["uniform", "lognormal", "piecewise", "twodups", "u64"])
def test_rmi_invariants(law):
    S, L, R = 10_000, 1000, 1000.0
    s = oracle.sort(inputs.generate(law, S, seed=4))[0]
    x = oracle.model_x(s)
    raw, sc, counts = oracle.rmi_fit(x, L, R)
    a, b, c, d = leaf_lines(raw, L)
    assert raw[0] >= 0 and np.all(a >= 0)
    chain = np.stack([c, d], axis=1).ravel()
    assert np.all(np.diff(chain) >= 0) and chain[0] >= 0 and chain[-1] <= 1
    # leaf membership is contiguous and follows the pre-scaled root
    leaves = np.array([oracle.rmi_leaf(sc[0], sc[1], L, v) for v in x])
    assert np.all(np.diff(leaves) >= 0)
    assert np.array_equal(np.bincount(leaves, minlength=L), counts)
    # the line stays inside its clamp interval except where the clamp cuts it
    lo = 0
    for j in range(L):
        k = int(counts[j])
        if k:
            p0, p1 = a[j] * x[lo] + b[j], a[j] * x[lo + k - 1] + b[j]
            assert c[j] >= min(max(p0, 0), 1) - 1e-12 and d[j] >= min(max(p1, 0), 1) - 1e-12
        lo += k


@pytest.mark.parametrize("law", ["uniform", "normal", "lognormal", "piecewise", "u64", "zipf"])
def test_bucket_monotone_along_sorted_order(law):
    """Sec. 3.1 / Sec. 4: x <= y implies F(x) <= F(y); needs no second implementation."""
    keys = inputs.generate(law, 50_000, seed=5)
    srt = oracle.sort(keys)[0]
    smp = oracle.sort(oracle.sample(keys, 1, 2000))[0]
    if not oracle.policy_learned(10**6, smp):
        smp = np.unique(smp)
    _, sc, _ = oracle.rmi_fit(oracle.model_x(smp), 300, 50_000.0)
    b = oracle.rmi_buckets(sc, 300, 50_000.0, srt)
    assert np.all(np.diff(b.astype(np.int64)) >= 0)
    assert b.max() < 50_000


def test_bucket_nonfinite_routing():
    keys = np.array([-np.inf, np.inf, np.nan, -np.nan, 0.5])
    s = np.sort(np.random.default_rng(0).random(100))
    _, sc, _ = oracle.rmi_fit(s, 10, 100.0)
    b = oracle.rmi_buckets(sc, 10, 100.0, keys)
    assert b[0] == 0 and b[1] == 99 and b[2] == 99 and b[3] == 0


@pytest.mark.parametrize("law", ["uniform", "lognormal", "mixgauss"])
def test_alg4_implicit_pivots_equivalence(law):
    """Sec. 3.3: the learned partition equals a SampleSort partition whose
    splitters are each non-empty bucket's largest key (Alg. 4):
    bucket(x) = bucket of the first pivot >= x."""
    keys = inputs.generate(law, 40_000, seed=6)
    smp = oracle.sort(oracle.sample(keys, 2, 1000))[0]
    R = 256.0
    _, sc, _ = oracle.rmi_fit(oracle.model_x(smp), 64, R)
    b = oracle.rmi_buckets(sc, 64, R, keys)
    piv, has = oracle.implicit_pivots(keys, b, 256)
    nz = np.flatnonzero(has)
    pk = piv[nz]
    assert np.all(np.diff(pk.astype(np.float64)) > 0) or np.all(pk[1:] > pk[:-1])
    pos = np.searchsorted(pk, oracle.ord_keys(keys), side="left")
    assert np.array_equal(nz[pos], b)


def exact_fma(a, x, b):
    return float(Fraction(a) * Fraction(x) + Fraction(b))


def test_two_buckets_is_learned_quicksort_split():
    """Sec. 3.2, Alg. 3: with B = 2 the partition is the two-way split by the
    model's CDF value.  Reading: the floor formula puts F = 0.5 on the right,
    so bucket 0 holds exactly the keys with F(x) < 0.5."""
    rng = np.random.default_rng(7)
    keys = rng.lognormal(0, 1, 3000)
    smp = np.sort(keys[rng.integers(0, 3000, 400)])
    L = 8
    raw, sc, _ = oracle.rmi_fit(smp, L, 2.0)
    b = oracle.rmi_buckets(sc, L, 2.0, keys)
    a_, b_, c_, d_ = leaf_lines(raw, L)
    for x, got in zip(keys, b):
        j = oracle.rmi_leaf(sc[0], sc[1], L, x)
        F = min(max(exact_fma(a_[j], x, b_[j]), c_[j]), d_[j])
        assert got == (0 if F < 0.5 else 1)


# -- splitter tree ------------------------------------------------------------------------

def test_splitters_closed_form_ranks():
    S, B = 256 * 7, 256
    s = np.arange(S, dtype=np.uint64) * 5
    u, eq = oracle.splitters(s, B)
    assert np.array_equal(u, (np.arange(1, B) * 7 * 5).astype(np.uint64))
    assert not eq.any()


def test_splitter_buckets_upper_bound():
    rng = np.random.default_rng(8)
    s = np.sort(rng.random(5000))
    u, eq = oracle.splitters(s, 128)
    assert not eq.any()
    keys = rng.random(20_000)
    keys[:100] = s[rng.integers(0, 5000, 100)]    # some keys equal a splitter
    b = oracle.splitter_buckets(u, eq, keys)
    assert np.array_equal(b, np.searchsorted(u, oracle.ord_keys(keys), side="right"))


def test_equality_buckets():
    rng = np.random.default_rng(9)
    keys = rng.choice(np.array([1.0, 2.0, 3.0, 7.0]), 10_000, p=[0.7, 0.1, 0.1, 0.1])
    keys = np.concatenate([keys, rng.random(2000) * 10])
    s = oracle.sort(keys[rng.integers(0, keys.size, 4000)])[0]
    u, eq = oracle.splitters(s, 64)
    assert eq.any()
    b = oracle.splitter_buckets(u, eq, keys)
    nb = u.size + 1 + int(eq.sum())
    assert b.max() < nb
    srt = oracle.sort(keys)[0]
    bs = oracle.splitter_buckets(u, eq, srt)
    assert np.all(np.diff(bs.astype(np.int64)) >= 0)
    # every flagged splitter's value sits alone in its own bucket
    ok = oracle.ord_keys(keys)
    for i in np.flatnonzero(eq):
        ids = np.unique(b[ok == u[i]])
        assert ids.size == 1
        assert np.all(ok[b == ids[0]] == u[i])


# -- range radix ------------------------------------------------------------------------

def test_radix_progress_bound():
    """Eight 8-bit levels make every segment homogeneous (guaranteed progress)."""
    rng = np.random.default_rng(10)
    keys = rng.integers(0, 2**64, 3000, dtype=np.uint64, endpoint=False)
    keys[:500] = keys[0]
    segs = [keys]
    levels = 0
    while any(np.unique(s).size > 1 for s in segs):
        nxt = []
        for s in segs:
            o = oracle.ord_keys(s)
            lo, hi = int(o.min()), int(o.max())
            if lo == hi:
                continue
            sh = oracle.radix_shift(lo, hi, 8)
            b = oracle.radix_buckets(lo, sh, s)
            assert b.max() < 256
            order = np.argsort(o, kind="stable")
            assert np.all(np.diff(b[order].astype(np.int64)) >= 0)
            nxt += [s[b == k] for k in np.unique(b)]
        segs = nxt
        levels += 1
    assert levels <= 8


# -- one partition level ------------------------------------------------------------------

@pytest.mark.parametrize("B", [1, 2, 17, 1000])
def test_partition_is_stable_counting_sort(B):
    rng = np.random.default_rng(B)
    n = 30_000
    keys = rng.random(n)
    ids = rng.integers(0, B, n).astype(np.uint32)
    pay = np.arange(n, dtype=np.uint32)
    ok, op, counts, starts = oracle.partition(keys, ids, B, pay)
    r = np.argsort(ids, kind="stable")
    assert np.array_equal(ok, keys[r])
    assert np.array_equal(op, pay[r])
    assert np.array_equal(counts, np.bincount(ids, minlength=B).astype(np.uint64))
    assert np.array_equal(starts, np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.uint64))


# -- MLP -------------------------------------------------------------------------------------

def rand_params(seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.5, oracle.MLP_NP)
    return p


def test_mlp_gradient_finite_differences():
    rng = np.random.default_rng(11)
    t = np.sort(rng.random(200))
    y = np.arange(200) / 200
    for seed in range(3):
        p = rand_params(seed)
        loss, g = oracle.mlp_loss_grad(p, t, y)
        h = 1e-6
        num = np.empty_like(p)
        for i in range(p.size):
            e = np.zeros_like(p)
            e[i] = h
            num[i] = (oracle.mlp_loss_grad(p + e, t, y)[0] - oracle.mlp_loss_grad(p - e, t, y)[0]) / (2 * h)
        err = np.linalg.norm(num - g) / max(np.linalg.norm(g), 1e-30)
        assert err < 1e-6, err


def test_mlp_forward_is_monotone_and_fp32_close():
    rng = np.random.default_rng(12)
    p = rand_params(4)
    w = np.where(np.isin(np.arange(oracle.MLP_NP), list(range(0, 16)) + list(range(32, 288)) + list(range(304, 320))),
                 np.abs(p), p).astype(np.float32)
    ts = np.sort(rng.random(5000)).astype(np.float32)
    f32 = np.array([oracle.mlp_eval_f32(w, t) for t in ts])
    assert np.all(np.diff(f32) >= 0)
    f64 = np.clip([oracle.mlp_forward(p, float(t)) for t in ts], 0, 1)
    assert np.max(np.abs(f32 - f64)) < 1e-4


def test_adam_closed_form():
    """Kingma & Ba 2015: with bias correction, a constant gradient g moves every
    step by exactly lr * g / (|g| + eps)."""
    p0 = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-9])
    p, m, v = p0.copy(), np.zeros(3), np.zeros(3)
    for k in range(1, 6):
        p, m, v = oracle.adam_step(p, m, v, g, k, lr=0.01)
        step = 0.01 * g / (np.abs(g) + 1e-8)
        assert np.allclose(p, p0 - k * step, rtol=1e-12, atol=1e-15)



@pytest.mark.parametrize("law", ["uniform", "normal", "lognormal", "exponential"])
def test_mlp_init_is_the_octile_interpolant(law):
    """With eps = 0 the start point is the piecewise-linear interpolant of the
    sample CDF through (k_m, m/8): exact at every knot, linear in between,
    flat at 1 beyond the last knot.  Checked with an independent numpy
    interpolation (np.interp)."""
    S = 4096
    t = np.sort(oracle.mlp_inputs(oracle.sort(inputs.generate(law, S, seed=9))[0], 0.0, 1.0).astype(np.float64))
    if law != "uniform":  # map onto [0, 1] the way the model input does
        s = oracle.sort(inputs.generate(law, S, seed=9))[0]
        lo, inv = oracle.mlp_lo_inv(s)
        t = oracle.mlp_inputs(s, lo, inv).astype(np.float64)
    p = oracle.mlp_init(t, eps=0.0)
    knots = [t[m * S // 8] for m in range(8)] + [t[-1]]
    assert min(np.diff(knots)) >= 1e-6  # no segment narrow enough to be widened
    probe = np.unique(np.concatenate([knots, np.linspace(0, 1, 101), (np.array(knots[:-1]) + knots[1:]) / 2]))
    for q in probe:
        f = oracle.mlp_forward(p, float(q))
        seg = [m for m in range(8) if knots[m] <= q <= knots[m + 1]]
        if q >= knots[-1]:
            assert f == pytest.approx(1.0, abs=1e-12)
        elif seg:
            m = seg[0]
            want = m / 8 + (q - knots[m]) / (knots[m + 1] - knots[m]) / 8
            assert f == pytest.approx(want, abs=1e-9), (q, m)
    # with the default eps the start point stays within 2% of the interpolant
    pe = oracle.mlp_init(t, eps=1e-3)
    for q in knots:
        assert abs(oracle.mlp_forward(pe, float(q)) - oracle.mlp_forward(p, float(q))) < 0.02


@pytest.mark.parametrize("law", ["lognormal", "piecewise"])
def test_mlp_step_scale_bounds_preactivation_change(law):
    """One training step from the start point changes every layer-2
    pre-activation, anywhere on t in [0, 1], by at most
    lr * (1 + sum_k (s_k (B_k + 2 lr) + |V2_ik| 2 lr)) with B_k the activation
    bound of unit k -- about 17 lr -- because the step of a layer-2 weight is
    scaled by 1 / B_k.  (Unscaled, a weight feeding a first-layer ramp of
    width 1e-4 would move its pre-activation by ~1e4 lr.)  Also pins the
    composition: the first bias-corrected step of each parameter is exactly
    s * lr * g_s / (|g_s| + eps) with g_s = s g."""
    S, lr = 4096, 1e-2
    s = oracle.sort(inputs.generate(law, S, seed=9))[0]
    lo, inv = oracle.mlp_lo_inv(s)
    t = oracle.mlp_inputs(s, lo, inv).astype(np.float64)
    y = np.arange(S) / S
    p0 = oracle.mlp_init(t)
    sc = oracle.mlp_step_scale(p0)
    p1, _ = oracle.mlp_train(t, y, p0, 1, lr, final=True)
    _, g = oracle.mlp_loss_grad(p0, t, y)
    gs = sc * g
    want = -sc * lr * gs / (np.abs(gs) + 1e-8)
    assert np.all(np.abs((p1 - p0) - want) <= 1e-9 * np.abs(want) + 1e-15 * np.maximum(1.0, np.abs(p0)))
    bound = np.maximum(1.0, np.abs(p0[0:16]) + np.abs(p0[16:32]))
    assert bound.max() > 10  # the case the scale is for: steep first-layer ramps
    V2 = np.abs(p0[32:288]).reshape(16, 16)
    limit = lr * (1 + (sc[32:48] * (bound + 2 * lr)).sum() + 2 * lr * V2.sum(axis=1) / lr)
    for q in np.unique(np.concatenate([t[::64], np.linspace(0, 1, 257)])):
        z0 = oracle.mlp_forward_full(p0, q)[3]
        z1 = oracle.mlp_forward_full(p1, q)[3]
        assert np.all(np.abs(z1 - z0) <= limit * (1 + 1e-9) + 1e-12), q

def mlp_root_case(law, S=20_000, L=200, seed=3, steps=0):
    s = oracle.sort(inputs.generate(law, S, seed=seed))[0]
    x = oracle.model_x(s)
    lo, inv = oracle.mlp_lo_inv(s)
    t = oracle.mlp_inputs(s, lo, inv).astype(np.float64)
    p = oracle.mlp_init(t)
    if steps:
        p, _ = oracle.mlp_train(t[::20], np.arange(0, S, 20) / S, p, steps, 3e-3)
    return s, x, lo, inv, oracle.effective(p)


@pytest.mark.parametrize("law", ["uniform", "lognormal", "piecewise"])
def test_mlp_root_leaves_match_polyfit_and_counting(law):
    """Leaves under the MLP root: every leaf's line is the least-squares line
    of its run (numpy polyfit), the runs are exactly the points the root sends
    to each leaf (direct count), and the clamp chain is non-decreasing."""
    S, L, R = 20_000, 200, 1000.0
    s, x, lo, inv, w = mlp_root_case(law, S, L)
    raw, sc, counts = oracle.mlp_rmi_fit(x, w, lo, inv, L, R)
    leaves = np.array([oracle.mlp_leaf(w, lo, inv, L, v) for v in x])
    assert np.all(np.diff(leaves) >= 0)
    assert np.array_equal(np.bincount(leaves, minlength=L), counts)
    q = raw.reshape(L, 4)
    chain = q[:, 2:].ravel()
    assert np.all(np.diff(chain) >= 0) and chain[0] >= 0 and chain[-1] <= 1
    y = np.arange(S) / S
    start = 0
    for j in range(L):
        k = int(counts[j])
        if k >= 3 and np.ptp(x[start:start + k]) > 0:
            xs = x[start:start + k]
            sa, sb = np.polyfit(xs - xs.mean(), y[start:start + k], 1)
            assert q[j, 0] == pytest.approx(max(sa, 0.0), rel=1e-6, abs=1e-12 / max(np.ptp(xs), 1e-300))
        start += k
    assert np.allclose(sc, R * raw, rtol=1e-15, atol=0)


def test_mlp_root_arithmetic_progression_closed_form():
    """x_i = i with targets i/S is a line: whatever monotone root splits it,
    every leaf with two or more points fits slope 1/S and intercept 0."""
    S, L = 5000, 64
    x = np.arange(S, dtype=np.float64)
    lo, inv = 0.0, 1.0 / (S - 1)
    t = oracle.mlp_inputs(x, lo, inv).astype(np.float64)
    w = oracle.effective(oracle.mlp_init(t))
    raw, _, counts = oracle.mlp_rmi_fit(x, w, lo, inv, L, 1000.0)
    q = raw.reshape(L, 4)
    for j in np.flatnonzero(counts >= 2):
        assert q[j, 0] == pytest.approx(1.0 / S, rel=1e-12)
        assert abs(q[j, 1]) < 1e-12


@pytest.mark.parametrize("law", ["normal", "piecewise", "mixgauss"])
def test_mlp_root_buckets_monotone_and_alg4(law):
    """Sec. 3.1 / Alg. 4 on the MLP-root model: bucket ids are non-decreasing
    along the sorted keys, and every key's bucket is the first bucket whose
    implicit pivot (largest key in it) is not below the key."""
    n, R = 30_000, 1000.0
    s, x, lo, inv, w = mlp_root_case(law, 3000, 100, seed=6)
    _, sc, _ = oracle.mlp_rmi_fit(x, w, lo, inv, 100, R)
    keys = inputs.generate(law, n, seed=7)
    srt = oracle.sort(keys)[0]
    b = oracle.mlp_rmi_buckets(w, lo, inv, sc, 100, R, srt).astype(np.int64)
    assert np.all(np.diff(b) >= 0) and b.max() < R
    piv, has = oracle.implicit_pivots(srt, b.astype(np.uint32), int(R))
    ords = oracle.ord_keys(srt)
    nz = np.flatnonzero(has)
    first = nz[np.searchsorted(piv[nz], ords, side="left")]
    assert np.array_equal(first, b)


def test_mlp_root_gain_over_linear_root_on_piecewise():
    """What the learned root buys on the 70/20/10 piecewise law (three
    clusters over seven orders of magnitude): the linear root sends most keys
    to a few leaves, the MLP root (octile start point, 200 Adam steps) spreads
    them, so the largest of 1000 buckets shrinks severalfold; training also
    beats the untrained start point."""
    n, S, L, R = 400_000, 20_000, 1000, 1000.0
    keys = inputs.generate("piecewise", n, seed=8)
    s = oracle.sort(oracle.sample(keys, 5, S))[0]
    x = oracle.model_x(s)
    lo, inv = oracle.mlp_lo_inv(s)
    t = oracle.mlp_inputs(s, lo, inv).astype(np.float64)
    p, losses = oracle.mlp_train(t[::4], np.arange(0, S, 4) / S, oracle.mlp_init(t), 200, 3e-3)
    assert losses[-1] < losses[0]
    w = oracle.effective(p)
    _, sc_m, _ = oracle.mlp_rmi_fit(x, w, lo, inv, L, R)
    _, sc_r, _ = oracle.rmi_fit(x, L, R)
    mx = lambda b: np.bincount(b.astype(np.int64), minlength=int(R)).max() / (n / R)  # noqa: E731
    mlp_ratio = mx(oracle.mlp_rmi_buckets(w, lo, inv, sc_m, L, R, keys))
    rmi_ratio = mx(oracle.rmi_buckets(sc_r, L, R, keys))
    assert mlp_ratio * 2 < rmi_ratio, (mlp_ratio, rmi_ratio)
    w0 = oracle.effective(oracle.mlp_init(t))
    _, sc_0, _ = oracle.mlp_rmi_fit(x, w0, lo, inv, L, R)
    init_ratio = mx(oracle.mlp_rmi_buckets(w0, lo, inv, sc_0, L, R, keys))
    assert mlp_ratio < init_ratio, (mlp_ratio, init_ratio)

# -- pivot quality (Sec. 3.4, Table 1) ------------------------------------------------------

def test_pivot_quality_learned_beats_random_uniform():
    """Table 1 (qualitative pin): on uniform data the RMI's implicit pivots
    are closer to the perfect splitters than 255 random pivots.  The paper's
    exact values (tests/golden/table1_pivot_quality.txt) are parity unpinned:
    neither IPS4o's sample size nor LearnedSort's exact RMI is given."""
    rows = {r[0]: (float(r[1]), float(r[2])) for r in read_golden("table1_pivot_quality.txt")}
    assert rows["uniform"][1] < rows["uniform"][0]
    n, B = 1_000_000, 256
    keys = inputs.generate("uniform", n, seed=13)
    srt_ord = oracle.ord_keys(oracle.sort(keys)[0])
    smp = oracle.sort(oracle.sample(keys, 3, n // 100))[0]
    _, sc, _ = oracle.rmi_fit(oracle.model_x(smp), 1000, float(B))
    b = oracle.rmi_buckets(sc, 1000, float(B), keys)
    piv, has = oracle.implicit_pivots(keys, b, B)
    learned = oracle.pivot_quality(srt_ord, piv[:B - 1], B)
    rnd = np.sort(oracle.ord_keys(keys[np.random.default_rng(1).integers(0, n, B - 1)]))
    random_q = oracle.pivot_quality(srt_ord, rnd, B)
    assert learned < random_q
    assert math.isfinite(learned) and learned < 1.0


# -- MLP bucket, exact cases -------------------------------------------------------------------

def dyadic_mlp(b3=0.25):
    """Hand-set parameters whose every fp32 product and sum on inputs
    t = k / 1024 is exact (dyadic values with few bits): units 0..7 are
    max(t - i/16, 0), units 8..15 min(t - 1/2 - (i-8)/16, 0); layer-2 weights
    2^-(4 + (i + k) mod 3); output weights 1/8."""
    p = np.zeros(oracle.MLP_NP)
    for i in range(16):
        p[i] = 1.0
        p[16 + i] = -i / 16 if i < 8 else -0.5 - (i - 8) / 16
        p[288 + i] = -1 / 32 if i < 8 else 1 / 32
        p[304 + i] = 1 / 8
        for k in range(16):
            p[32 + 16 * i + k] = 2.0 ** -(4 + (i + k) % 3)
    p[320] = b3
    return p


def exact_forward(p, t):
    """The network's output with exact rational arithmetic (no rounding)."""
    from fractions import Fraction as Fr
    t = Fr(t)
    h1 = []
    for i in range(16):
        z = abs(Fr(p[i])) * t + Fr(p[16 + i])
        h1.append(max(z, Fr(0)) if i < 8 else min(z, Fr(0)))
    out = Fr(p[320])
    for i in range(16):
        z = Fr(p[288 + i]) + sum(abs(Fr(p[32 + 16 * i + k])) * h1[k] for k in range(16))
        h = max(z, Fr(0)) if i < 8 else min(z, Fr(0))
        out += abs(Fr(p[304 + i])) * h
    return out


@pytest.mark.parametrize("R", [1, 2, 1000, 1 << 20])
def test_mlp_bucket_exact_dyadic(R):
    """orc_mlp_bucket against an independent evaluation: the network output F
    in exact rational arithmetic (every fp32 step is exact for these weights
    and inputs, which the test checks), clamped to [0, 1], then
    min(floor(fp32(F) * fp32(R)), R - 1) with numpy's IEEE fp32 product."""
    p = dyadic_mlp()
    w = oracle.effective(p)
    keys = np.arange(0, 1025, dtype=np.float64) / 1024.0
    got = oracle.mlp_buckets(w, 0.0, 1.0, R, keys)
    for x, g in zip(keys, got):
        F = exact_forward(p, x)
        assert F == float(np.float32(float(F)))  # exactly representable in fp32
        Fc = min(max(float(F), 0.0), 1.0)
        want = min(int(np.floor(np.float32(Fc) * np.float32(R))), R - 1)
        assert g == want, (x, float(F), g, want)
    assert np.all(np.diff(got.astype(np.int64)) >= 0) and got.max() < R


@pytest.mark.parametrize("R", [1, 7, 1000])
def test_mlp_bucket_clamps_at_the_ends(R):
    """An output clamped to F = 1 maps to the last bucket R - 1 (not R), F = 0
    to bucket 0; non-finite keys go to 0 / R - 1 by sign."""
    keys = np.array([0.0, 0.25, 0.5, 1.0, 3.0], dtype=np.float64)
    hi = oracle.mlp_buckets(oracle.effective(dyadic_mlp(b3=2.0)), 0.0, 1.0, R, keys)
    assert np.all(hi == R - 1)
    lo = oracle.mlp_buckets(oracle.effective(dyadic_mlp(b3=-4.0)), 0.0, 1.0, R, keys)
    assert np.all(lo == 0)
    nf = np.array([-np.inf, np.nan, -np.nan, np.inf], dtype=np.float64)
    nf[2] = -abs(nf[2])
    g = oracle.mlp_buckets(oracle.effective(dyadic_mlp()), 0.0, 1.0, R, nf)
    assert list(g) == [0, R - 1, 0, R - 1]


def test_mlp_bucket_monotone_random_weights():
    """Random weights: ids are below R and non-decreasing along sorted keys."""
    w = oracle.effective(rand_params(5))
    keys = np.sort(np.random.default_rng(3).normal(0, 2, 20_000))
    for R in (3, 1000, 65536):
        g = oracle.mlp_buckets(w, -6.0, 1 / 12, R, keys).astype(np.int64)
        assert np.all(np.diff(g) >= 0) and g.max() < R and g.min() >= 0


# -- pivot quality, exact values -----------------------------------------------------------------

@pytest.mark.parametrize("data,pivots,B,want", [
    ([1, 2, 2, 3, 5, 8, 8, 8], [2, 5, 8], 4, 0.5),      # 3/8-1/4 + 5/8-2/4 + 8/8-3/4
    ([1, 2, 3, 4, 5, 6, 7, 8], [2, 4, 6], 4, 0.0),      # perfect splitters
    ([1, 2, 3, 4, 5, 6, 7, 8], [0, 0, 0], 4, 1.5),      # nothing below: 1/4 + 2/4 + 3/4
    ([5, 5, 5, 5], [5], 2, 0.5),                         # all keys <= the pivot: |1 - 1/2|
    ([1, 3], [2], 2, 0.0),
])
def test_pivot_quality_hand_counted(data, pivots, B, want):
    """Sec. 3.4 metric sum_i |P(A <= p_i) - (i+1)/B|, counted by hand."""
    s = oracle.ord_keys(np.array(data, dtype=np.uint64))
    p = oracle.ord_keys(np.array(pivots, dtype=np.uint64))
    assert oracle.pivot_quality(s, p, B) == pytest.approx(want, abs=1e-15)


# -- MLP training rule ---------------------------------------------------------------------------

def test_mlp_step_scale_closed_form():
    """s = 1 / max(1, |V1_k| + |b1_k|) on every layer-2 weight of input unit
    k (row-major V2: entry 32 + 16 i + k), 1 elsewhere."""
    p = np.zeros(oracle.MLP_NP)
    p[0:16] = np.arange(16) - 5.0
    p[16:32] = 0.25
    s = oracle.mlp_step_scale(p)
    bound = np.maximum(1.0, np.abs(np.arange(16) - 5.0) + 0.25)
    for i in range(16):
        for k in range(16):
            assert s[32 + 16 * i + k] == 1.0 / bound[k]
    assert np.all(s[:32] == 1.0) and np.all(s[288:] == 1.0)


def test_mlp_train_zero_steps_is_start_point():
    t = np.linspace(0, 1, 100)
    p0 = dyadic_mlp()
    p, losses = oracle.mlp_train(t, t, p0, 0, 1e-2)
    assert np.array_equal(p, p0) and losses.size == 0


def test_mlp_train_unit_scale_is_plain_adam():
    """With every first-layer bound at most 1 the scale is 1 and training is
    the pinned Adam step (orc_adam_step, closed form) applied to the pinned
    gradient (finite differences) step after step; the returned parameters
    are those of the lowest loss, the final ones on request."""
    rng = np.random.default_rng(4)
    t = np.sort(rng.random(300))
    y = np.arange(300) / 300
    p0 = rng.normal(0, 0.3, oracle.MLP_NP)
    p0[0:16] = rng.uniform(-0.5, 0.5, 16)
    p0[16:32] = rng.uniform(-0.4, 0.4, 16)
    assert np.all(oracle.mlp_step_scale(p0) == 1.0)
    steps, lr = 25, 5e-2
    p, m, v = p0.copy(), np.zeros(oracle.MLP_NP), np.zeros(oracle.MLP_NP)
    hist, losses = [], []
    for k in range(1, steps + 1):
        loss, g = oracle.mlp_loss_grad(p, t, y)
        hist.append(p.copy())
        losses.append(loss)
        p, m, v = oracle.adam_step(p, m, v, g, k, lr=lr)
    final, fl = oracle.mlp_train(t, y, p0, steps, lr, final=True)
    best, bl = oracle.mlp_train(t, y, p0, steps, lr)
    assert np.array_equal(fl, np.array(losses)) and np.array_equal(bl, fl)
    assert np.array_equal(final, p)
    assert np.array_equal(best, hist[int(np.argmin(losses))])
