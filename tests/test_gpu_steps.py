"""GPU parity of the individual steps of one learned partition level.

Each step runs in the library's HIP kernels through the C ABI and is compared
with the CPU oracle on the same seeded input: sampling and all integer work
bit-exact; the least-squares fit within a relative 1e-9 (the GPU sums in
double with its own reduction order, the oracle in long double).  Bucket ids
are compared bit-exact with both sides evaluating the GPU-fitted parameters,
since the evaluation is the same fma/floor/min/max sequence on both.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2307_08637_amd import inputs, lsort
from tests.gpu_helpers import to_dev, to_host

pytestmark = pytest.mark.gpu

FIT_RTOL = 1e-9


def sorted_sample(keys, seed, S):
    smp = oracle.sample(keys, seed, S)
    return oracle.sort(smp)[0]


@pytest.mark.parametrize("law", ["uniform", "u64", "normal"])
@pytest.mark.parametrize("S", [1, 1000, 123_457])
def test_sample(dev, law, S):
    keys = inputs.generate(law, 300_001, seed=3)
    got = to_host(lsort.sample(to_dev(keys, dev), seed=12345, S=S))
    want = oracle.sample(keys, 12345, S)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def check_fit(gp, s, L, R):
    x = oracle.model_x(s)
    # root: compare both lines' leaf coordinate at the ends of the sample
    _, orc, counts = oracle.rmi_fit(x, L, R)
    for xv in (x[0], x[-1]):
        a = gp[0] * xv + gp[1]
        b = orc[0] * xv + orc[1]
        assert abs(a - b) <= FIT_RTOL * (L + abs(b)), (a, b)
    # leaves: the oracle refits with the GPU's root so both see the same leaves
    _, orc, counts = oracle.rmi_fit(x, L, R, root=gp[:2])
    assert counts.sum() == x.size
    lo = 0
    for j in range(L):
        c = int(counts[j])
        g = gp[2 + 4 * j: 6 + 4 * j]
        o = orc[2 + 4 * j: 6 + 4 * j]
        assert g[0] >= 0
        assert abs(g[2] - o[2]) <= FIT_RTOL * R and abs(g[3] - o[3]) <= FIT_RTOL * R, (j, g, o)
        if c:
            for xv in (x[lo], x[lo + c - 1]):
                gv, ov = g[0] * xv + g[1], o[0] * xv + o[1]
                assert abs(gv - ov) <= FIT_RTOL * (R + abs(ov) + abs(o[0] * xv)), (j, gv, ov)
        lo += c
    # monotone clamp chain gamma_0 <= delta_0 <= gamma_1 <= ... (Sec. 4)
    cd = np.stack([gp[4::4][:L], gp[5::4][:L]], axis=1).ravel()
    assert np.all(np.diff(cd) >= 0)
    assert cd[0] >= 0 and cd[-1] <= R


@pytest.mark.parametrize("law,L,S", [("uniform", 1000, 10_000), ("lognormal", 1000, 1_000_000), ("normal", 64, 5000),
                                     ("u64", 1000, 200_000), ("mixgauss", 513, 77_777), ("exponential", 2, 1000),
                                     # leaves of more than one piece (summed by several workgroups)
                                     ("piecewise", 1000, 1_000_000), ("normal", 3, 400_000)])
def test_rmi_fit(dev, law, L, S):
    keys = inputs.generate(law, max(S * 10, 100_000), seed=5)
    s = sorted_sample(keys, 99, S)
    R = 1000.0 * 16
    gp = lsort.rmi_fit(to_dev(s, dev), L, R).cpu().numpy()
    check_fit(gp, s, L, R)


@pytest.mark.parametrize("law", ["uniform", "lognormal", "u64", "piecewise"])
def test_rmi_buckets_bitexact(dev, law):
    n, L, R = 400_000, 1000, 64_000.0
    keys = inputs.generate(law, n, seed=8)
    s = sorted_sample(keys, 7, 4000)
    gpar = lsort.rmi_fit(to_dev(s, dev), L, R)
    got = lsort.rmi_buckets(to_dev(keys, dev), gpar, L, R).view(torch.int32).cpu().numpy().view(np.uint32)
    want = oracle.rmi_buckets(gpar.cpu().numpy(), L, R, keys)
    assert np.array_equal(got, want)
    # monotone along the sorted order (Sec. 3.1 property; Sec. 4 constraint)
    srt = oracle.sort(keys)[0]
    b = lsort.rmi_buckets(to_dev(srt, dev), gpar, L, R).view(torch.int32).cpu().numpy()
    assert np.all(np.diff(b) >= 0)


def test_rmi_buckets_nonfinite(dev):
    keys = inputs.adversarial("with_nan", 50_000, seed=2)
    finite = keys[np.isfinite(keys)]
    s = sorted_sample(finite, 1, 2000)
    L, R = 100, 1000.0
    gpar = lsort.rmi_fit(to_dev(s, dev), L, R)
    got = lsort.rmi_buckets(to_dev(keys, dev), gpar, L, R).view(torch.int32).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle.rmi_buckets(gpar.cpu().numpy(), L, R, keys))


@pytest.mark.parametrize("law,B,S", [("uniform", 256, 10_000), ("rootdups", 256, 50_000), ("zipf", 512, 30_000),
                                     ("twodups", 2, 100), ("u64", 1024, 1023)])
def test_splitters(dev, law, B, S):
    keys = inputs.generate(law, 200_000, seed=9)
    s = sorted_sample(keys, 3, S)
    u, eq = lsort.splitters(to_dev(s, dev), B)
    ou, oeq = oracle.splitters(s, B)
    assert np.array_equal(to_host(u), ou)
    assert np.array_equal(eq.cpu().numpy(), oeq)
    got = lsort.splitter_buckets(to_dev(keys, dev), u, eq).view(torch.int32).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle.splitter_buckets(ou, oeq, keys))


@pytest.mark.parametrize("law,nb,log2b2", [("uniform", 1000, 0), ("lognormal", 1000, 4), ("u64", 37, 3),
                                           ("normal", 1024, 0)])
@pytest.mark.parametrize("n", [1, 8191, 8192, 100_003])
def test_partition_rmi(dev, law, nb, log2b2, n):
    keys = inputs.generate(law, n, seed=10)
    big = inputs.generate(law, 100_000, seed=10)
    s = sorted_sample(big, 5, 5000)
    L = 500
    R = float(nb << log2b2)
    gpar = lsort.rmi_fit(to_dev(s, dev), L, R)
    pay = np.arange(n, dtype=np.uint32)
    tk = to_dev(keys, dev)
    tp = torch.from_numpy(pay.view(np.int32).copy()).to(dev).view(torch.uint32)
    ok, op, counts = lsort.partition_rmi(tk, gpar, L, R, nb, payload=tp)
    torch.cuda.synchronize()
    ids = oracle.rmi_buckets(gpar.cpu().numpy(), L, R, keys) >> log2b2
    wk, wp, wc, _ = oracle.partition(keys, ids, nb, pay)
    assert np.array_equal(to_host(counts).astype(np.uint64), wc)
    assert np.array_equal(to_host(ok).view(np.uint64), wk.view(np.uint64))
    assert np.array_equal(op.view(torch.int32).cpu().numpy().view(np.uint32), wp)


@pytest.mark.parametrize("law", ["uniform", "rootdups", "zipf"])
def test_partition_splitters(dev, law):
    n = 250_001
    keys = inputs.generate(law, n, seed=11)
    s = sorted_sample(keys, 4, 20_000)
    ou, oeq = oracle.splitters(s, 256)
    pay = np.arange(n, dtype=np.uint32)
    tp = torch.from_numpy(pay.view(np.int32).copy()).to(dev).view(torch.uint32)
    ok, op, counts = lsort.partition_splitters(to_dev(keys, dev), to_dev(ou, dev), torch.from_numpy(oeq).to(dev),
                                               payload=tp)
    torch.cuda.synchronize()
    nb = ou.size + 1 + int(oeq.sum())
    ids = oracle.splitter_buckets(ou, oeq, keys)
    wk, wp, wc, _ = oracle.partition(keys, ids, nb, pay)
    assert np.array_equal(to_host(counts).astype(np.uint64), wc)
    assert np.array_equal(to_host(ok).view(np.uint64), wk.view(np.uint64))
    assert np.array_equal(op.view(torch.int32).cpu().numpy().view(np.uint32), wp)


@pytest.mark.parametrize("law,L,S", [("uniform", 1000, 1000), ("normal", 1000, 10_000), ("lognormal", 1000, 16384),
                                     ("u64", 512, 16384), ("mixgauss", 64, 4097), ("exponential", 2, 2),
                                     # leaves of more than 128 points (summed by a whole wavefront)
                                     ("piecewise", 1000, 2048), ("piecewise", 1000, 16384), ("normal", 4, 16384)])
def test_rmi_fit_block(dev, law, L, S):
    """The one-workgroup fit (the model of every segment whose sample fits in
    LDS, and of every batched array) against the oracle's long-double fit,
    within the same relative 1e-9 as the multi-workgroup fit."""
    keys = inputs.generate(law, max(S * 10, 100_000), seed=6)
    s = sorted_sample(keys, 17, S)
    R = 1000 * 8
    print(f"[case] fit_block {law} L={L} S={S}", flush=True)
    gp = lsort.rmi_fit_block(to_dev(s, dev), L, R).cpu().numpy()
    check_fit(gp, s, L, float(R))
