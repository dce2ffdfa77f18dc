"""Seeded sweep of random configurations against the oracle (bit-exact):
sizes from 1 to 3e6, every law and adversarial input, single arrays and
batched calls, with and without a uint32 payload, and random options
(first-level buckets, cutoff, tree fan-out, fallback ratio, balance judge,
model).  Each case draws everything from its own seed, so a case is
reproduced by its id alone."""
import numpy as np
import pytest
import torch

import oracle
from paper_2307_08637_amd import inputs, lsort
from tests.gpu_helpers import to_dev, to_host

pytestmark = pytest.mark.gpu

LAWS = inputs.ALL_LAWS + inputs.ADVERSARIAL_F64 + inputs.ADVERSARIAL_U64


def draw_case(seed: int):
    r = np.random.default_rng([7001, seed])
    law = LAWS[int(r.integers(len(LAWS)))]
    n = int(np.exp(r.uniform(0 if r.random() < 0.5 else np.log(1e4), np.log(3e6))))
    opts = {}
    if r.random() < 0.5:
        opts["buckets"] = int(r.choice([2, 16, 64, 256, 1000, 1024]))
    if r.random() < 0.4:
        opts["cutoff"] = int(r.choice([64, 256, 512, 2048, 4096]))
    if r.random() < 0.3:
        opts["tree_buckets"] = int(r.choice([2, 8, 64, 256, 512]))
    if r.random() < 0.3:
        opts["fallback_ratio"] = float(r.choice([1.2, 1.5, 3.0]))
    if r.random() < 0.3:
        opts["balance_pct"] = int(r.choice([1, 50, 100]))
    if r.random() < 0.2:
        opts["model"] = "splitter"
    pay = bool(r.random() < 0.4)
    segs = int(r.choice([1, 1, 1, 3, 40])) if n > 100 else 1
    return law, n, opts, pay, segs, int(r.integers(1 << 30))


def gen(law, n, seed):
    return inputs.generate(law, n, seed=seed) if law in inputs.ALL_LAWS else inputs.adversarial(law, n, seed=seed)


@pytest.mark.parametrize("case", range(160))
def test_random_case(dev, case):
    law, n, opts, pay, segs, seed = draw_case(case)
    keys = gen(law, n, seed)
    payload = np.arange(n, dtype=np.uint32) if pay else None
    print(f"[case] {case}: law={law} n={n} segs={segs} pay={pay} opts={opts}", flush=True)
    t = to_dev(keys, dev)
    p = None if payload is None else torch.from_numpy(payload.view(np.int32).copy()).to(dev).view(torch.uint32)
    if segs == 1:
        lsort.sort(t, p, **opts)
        want, wp = oracle.sort(keys, payload)
    else:
        cuts = np.sort(np.random.default_rng(seed).integers(0, n + 1, segs - 1)).astype(np.uint64)
        off = np.concatenate([[0], cuts, [n]]).astype(np.uint64)
        o = torch.from_numpy(off.view(np.int64)).to(dev).view(torch.uint64)
        lsort.sort_segmented(t, o, p, **opts)
        want, wp = oracle.sort_segmented(keys, off, payload)
    torch.cuda.synchronize()
    got = to_host(t)
    g = np.ascontiguousarray(got).view(np.uint64)
    w = np.ascontiguousarray(want).view(np.uint64)
    bad = np.flatnonzero(g != w)
    assert bad.size == 0, f"case {case}: {bad.size} key mismatches, first at {bad[:5]}"
    if pay:
        gp = p.view(torch.int32).cpu().numpy().view(np.uint32)
        assert np.array_equal(gp, wp), f"case {case}: payload differs"
