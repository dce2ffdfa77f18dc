"""GPU parity of the monotone MLP CDF: training kernels, the MLP-rooted
two-level model, and sorting with it.

- Gradients and loss of the FP32 GPU forward/backward against the oracle's
  fp64 chain rule on the same parameters and inputs: relative error of the
  whole gradient vector below 1e-3 (fp32 sums of up to 1e5 terms) and the
  loss within a relative 1e-4.
- The start point and lo/inv: bit-exact (both sides compute the same fp64
  values; the GPU rounds them once to fp32).
- Training: loss trajectory within a relative 2e-3 of the oracle's fp64
  Adam run from the same start point.
- Bucket ids (network alone, and the MLP-rooted model): bit-exact with both
  sides evaluating the same fp32 weights, since the evaluation is the same
  fmaf / floor / min / max sequence on both.
- Leaf fit under the MLP root: within a relative 1e-9 of the oracle (the
  leaf runs are identical; only the least-squares summation order differs).
- Sorting with the MLP model: bit-exact against the oracle's sort.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2307_08637_amd import inputs, lsort
from tests.gpu_helpers import to_dev, to_host

pytestmark = pytest.mark.gpu

WEIGHTS = np.r_[0:16, 32:288, 304:320]


def f32(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def model_inputs(keys):
    s = oracle.sort(keys)[0]
    lo, inv = oracle.mlp_lo_inv(s)
    return s, lo, inv, oracle.mlp_inputs(s, lo, inv)


@pytest.mark.parametrize("S", [1, 255, 257, 5000, 70_001])
def test_loss_grad_vs_oracle(dev, S):
    rng = np.random.default_rng(S)
    t = np.sort(rng.random(S)).astype(np.float32)
    y = (np.arange(S) / S).astype(np.float32)
    for seed in range(3):
        p = np.random.default_rng(100 + seed).normal(0, 0.5, 321).astype(np.float32)
        print(f"[case] loss_grad S={S} seed={seed}", flush=True)
        loss, g = lsort.mlp_loss_grad(f32(p, dev), f32(t, dev), f32(y, dev))
        g = g.cpu().numpy().astype(np.float64)
        want_loss, want = oracle.mlp_loss_grad(p.astype(np.float64), t.astype(np.float64), y.astype(np.float64))
        assert float(loss.item()) == pytest.approx(want_loss, rel=1e-4)
        err = np.linalg.norm(g - want) / max(np.linalg.norm(want), 1e-30)
        assert err < 1e-3, err
        loss2, g2 = lsort.mlp_loss_grad(f32(p, dev), f32(t, dev), f32(y, dev))
        assert np.array_equal(g2.cpu().numpy().view(np.uint32), g.astype(np.float32).view(np.uint32))


@pytest.mark.parametrize("S,ties", [(1, False), (2, False), (255, False), (5000, False), (70_001, False),
                                    (1_000_000, False), (40_000, True)])
def test_region_grad_vs_oracle(dev, S, ties):
    """The gradient by activation regions (how training computes it) against
    the oracle's per-sample fp64 chain rule on the same fp32 parameters and
    sorted inputs (with many equal inputs too): the whole vector within a
    relative 1e-4 (only rounding order and units switching within rounding
    of zero differ), the loss within 1e-5, and bit-identical on a repeat."""
    rng = np.random.default_rng(S + 7)
    t = np.sort(rng.integers(0, 40, S) / 40.0 if ties else rng.random(S)).astype(np.float32)
    y = (np.arange(S) / S).astype(np.float32)
    for seed in range(3):
        p = np.random.default_rng(200 + seed).normal(0, 0.5, 321).astype(np.float32)
        if seed == 2:  # the octile start point: ramps switching inside the data
            p = oracle.mlp_init(t.astype(np.float64)).astype(np.float32)
        print(f"[case] region grad S={S} ties={ties} seed={seed}", flush=True)
        loss, g = lsort.mlp_loss_grad(f32(p, dev), f32(t, dev), f32(y, dev), regions=True)
        g = g.cpu().numpy().astype(np.float64)
        want_loss, want = oracle.mlp_loss_grad(p.astype(np.float64), t.astype(np.float64), y.astype(np.float64))
        assert float(loss.item()) == pytest.approx(want_loss, rel=1e-5, abs=1e-30)
        err = np.linalg.norm(g - want) / max(np.linalg.norm(want), 1e-30)
        assert err < 1e-4, err
        loss2, g2 = lsort.mlp_loss_grad(f32(p, dev), f32(t, dev), f32(y, dev), regions=True)
        assert np.array_equal(g2.cpu().numpy().view(np.uint32), g.astype(np.float32).view(np.uint32))


@pytest.mark.parametrize("law", ["uniform", "normal", "lognormal", "piecewise", "u64"])
def test_start_point_and_inputs_bit_exact(dev, law):
    keys = inputs.generate(law, 20_000, seed=17)
    s, lo, inv, t = model_inputs(keys)
    params, lo_inv, _ = lsort.mlp_train(to_dev(s, dev), steps=0, lr=1e-3)
    li = lo_inv.cpu().numpy()
    assert li[0] == lo and li[1] == inv
    want = oracle.mlp_init(t.astype(np.float64)).astype(np.float32)
    got = params.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("law", ["normal", "lognormal"])
def test_training_trajectory_vs_oracle(dev, law):
    S, steps, lr = 4096, 25, 3e-3
    keys = inputs.generate(law, S, seed=19)
    s, lo, inv, t = model_inputs(keys)
    p0 = oracle.mlp_init(t.astype(np.float64)).astype(np.float32)
    params, _, losses = lsort.mlp_train(to_dev(s, dev), steps=steps, lr=lr, params_init=f32(p0, dev))
    y = (np.arange(S) / S).astype(np.float32).astype(np.float64)
    _, want_losses = oracle.mlp_train(t.astype(np.float64), y, p0.astype(np.float64), steps, lr)
    got = losses.cpu().numpy().astype(np.float64)
    assert np.allclose(got, want_losses, rtol=2e-3, atol=0), (got[:5], want_losses[:5])
    # the returned parameters are the best seen: their loss (fp64, oracle) is the trajectory's minimum
    best_loss, _ = oracle.mlp_loss_grad(params.cpu().numpy().astype(np.float64), t.astype(np.float64), y)
    assert best_loss == pytest.approx(want_losses.min(), rel=2e-3)
    assert best_loss <= want_losses[0]


def trained(dev, law, S=20_000, steps=60):
    keys = inputs.generate(law, S, seed=23)
    s = oracle.sort(keys)[0]
    params, lo_inv, losses = lsort.mlp_train(to_dev(s, dev), steps=steps, lr=3e-3)
    return s, params, lo_inv, losses


@pytest.mark.parametrize("n", [1, 1000, 300_001])
@pytest.mark.parametrize("law", ["normal", "piecewise"])
def test_mlp_buckets_bit_exact(dev, n, law):
    s, params, lo_inv, _ = trained(dev, law)
    keys = inputs.generate(law, n, seed=29)
    if n > 10:
        keys[:4] = [np.inf, -np.inf, np.nan, -0.0]
    R = 1000
    got = to_host(lsort.mlp_buckets(to_dev(keys, dev), params, lo_inv, R).view(torch.int32)).view(np.uint32)
    li = lo_inv.cpu().numpy()
    w = oracle.effective(params.cpu().numpy())
    want = oracle.mlp_buckets(w, float(li[0]), float(li[1]), R, keys)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("law", ["uniform", "lognormal", "piecewise", "mixgauss"])
@pytest.mark.parametrize("L", [2, 100, 1000])
def test_mlp_rmi_fit_and_buckets(dev, law, L):
    s, params, lo_inv, _ = trained(dev, law)
    R = 1000.0 * 16
    leaves = lsort.mlp_rmi_fit(to_dev(s, dev), params, lo_inv, L, R).cpu().numpy()
    li = lo_inv.cpu().numpy()
    w = oracle.effective(params.cpu().numpy())
    x = oracle.model_x(s)
    _, want, counts = oracle.mlp_rmi_fit(x, w, float(li[0]), float(li[1]), L, R)
    assert counts.sum() == s.size
    g, o = leaves.reshape(L, 4), want.reshape(L, 4)
    assert np.all(np.abs(g[:, 2:] - o[:, 2:]) <= 1e-9 * R)
    lo = 0
    for j in range(L):
        c = int(counts[j])
        if c:
            for xv in (x[lo], x[lo + c - 1]):
                gv, ov = g[j, 0] * xv + g[j, 1], o[j, 0] * xv + o[j, 1]
                assert abs(gv - ov) <= 1e-9 * (R + abs(ov) + abs(o[j, 0] * xv)), (j, gv, ov)
        lo += c
    # bucket ids under the oracle's leaves, both sides evaluating the same model
    keys = inputs.generate(law, 200_003, seed=31)
    keys[:3] = [np.inf, -np.inf, np.nan]
    got = to_host(lsort.mlp_rmi_buckets(to_dev(keys, dev), params, lo_inv,
                                        torch.from_numpy(want).to(dev), L, R).view(torch.int32)).view(np.uint32)
    ref = oracle.mlp_rmi_buckets(w, float(li[0]), float(li[1]), want, L, R, keys)
    assert np.array_equal(got, ref)
    # monotone along the sorted keys (Sec. 3.1)
    order = np.argsort(oracle.ord_keys(keys), kind="stable")
    assert np.all(np.diff(got[order].astype(np.int64)) >= 0)


@pytest.mark.parametrize("law", ["uniform", "normal", "lognormal", "piecewise", "mixgauss", "u64"])
@pytest.mark.parametrize("n", [100_000, 1_000_000])
def test_sort_with_mlp_model(dev, law, n):
    keys = inputs.generate(law, n, seed=37)
    t = to_dev(keys, dev)
    print(f"[case] mlp sort {law} n={n}", flush=True)
    lsort.sort(t, model="mlp", mlp_steps=50)
    torch.cuda.synchronize()
    want, _ = oracle.sort(keys)
    assert np.array_equal(to_host(t).view(np.uint64), want.view(np.uint64))
    st = lsort.stats()
    if st["levels"][0]["learned"]:
        assert st["first_model"] == 2
        # the model keeps the best parameters seen: never worse than the start point
        assert st["mlp_loss_last"] <= st["mlp_loss_first"]


def test_sort_with_mlp_model_payload_stable(dev):
    n = 400_000
    keys = inputs.generate("rootdups", n, seed=41).astype(np.float64)
    pay = np.arange(n, dtype=np.uint32)
    t = to_dev(keys, dev)
    p = torch.from_numpy(pay.view(np.int32).copy()).to(dev).view(torch.uint32)
    lsort.sort(t, p, model="mlp", mlp_steps=20)
    torch.cuda.synchronize()
    want, wp = oracle.sort(keys, pay)
    assert np.array_equal(to_host(t).view(np.uint64), want.view(np.uint64))
    assert np.array_equal(p.view(torch.int32).cpu().numpy().view(np.uint32), wp)


def test_mlp_gain_over_linear_root(dev):
    """What the trained network buys inside the sort: on the 70/20/10
    piecewise law the first level's largest bucket (x expected) under the
    MLP-rooted model is several times smaller than under the RMI's linear
    root (the balance judge off: by default it gives this law's first level
    to the splitter tree); and 200 Adam steps improve on the untrained start
    point."""
    n = 4_000_000
    keys = inputs.generate("piecewise", n, seed=43)
    ratios = {}
    for model in ("rmi", "mlp"):
        t = to_dev(keys, dev)
        lsort.sort(t, model=model, balance_pct=100)
        torch.cuda.synchronize()
        st = lsort.stats()
        assert st["levels"][0]["learned"] == 1
        ratios[model] = st["levels"][0]["max_bucket_x1000_over_mean"] / 1000.0
        del t
    print(f"[gain] first-level max/mean: rmi {ratios['rmi']:.2f} mlp {ratios['mlp']:.2f}", flush=True)
    assert ratios["mlp"] * 2 < ratios["rmi"], ratios
    # trained vs start point, same sample, same leaves fit
    smp = oracle.sort(oracle.sample(keys, 5, 40_000))[0]
    sd = to_dev(smp, dev)
    kd = to_dev(keys[:1_000_000], dev)
    bal = {}
    for steps in (0, 200):
        params, lo_inv, _ = lsort.mlp_train(sd, steps=steps, lr=3e-3)
        leaves = lsort.mlp_rmi_fit(sd, params, lo_inv, 1000, 1000.0)
        b = lsort.mlp_rmi_buckets(kd, params, lo_inv, leaves, 1000, 1000.0).to(torch.int64)
        bal[steps] = float(torch.bincount(b, minlength=1000).max().item()) / (kd.numel() / 1000)
    print(f"[gain] MLP-rooted max/mean: start {bal[0]:.2f} trained {bal[200]:.2f}", flush=True)
    assert bal[200] < bal[0], bal
