"""Benchmark: Gkeys/s sorting 1e8 float64 keys on one MI355X, learned (RMI)
partitioning vs the splitter-tree form, with the roofline of the dominant
kernel and the CPU oracle's rate on the host.

A step is one complete sort of the 1e8-key array (sampling, sample sort,
model fit, every partition level and the base case).  The keys of every
timed step are already in HBM: K unsorted copies are made before the timed
region and step k sorts copy k in place.

Besides the headline line it reports, in extra fields of the same JSON
object:
  * the output check: sorted, the same multiset as the input (two 64-bit
    hashes), and -- with the CPU baseline -- equal word for word to the
    oracle's sort of the same keys;
  * the pivot quality of Table 1 (Sec. 3.4) at 1e8: the RMI's implicit
    pivots (Alg. 4) vs the splitter tree's sample quantiles vs random keys;
  * the same sort per input law, the duplicate-heavy laws included;
  * the batched form: sort_segmented over the whole 10,000-array workload
    (sizes log-uniform in [1e3, 1e6], five float64 laws, uint32 payload) and
    over its first 2e8 keys, learned vs splitter, plus the fixed-level form
    eager and replayed from a captured HIP graph;
  * the learned parts on the 70/20/10 piecewise law at 1e8 and at 1e9 keys:
    RMI root vs MLP root vs splitter tree (first-level max/mean bucket ratio,
    fallbacks, Gkeys/s).

  * the sample-once / model-reuse question and the sample size (refit per
    bucket vs reuse; samples of 0.1% .. 4%), with the pivot quality;
  * the other key types and payload widths at 1e8: float32 and int64 keys,
    float64 keys with a 64-bit payload;
  * the base case as comparison sorts vs the model-placed counting sort.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--law normal]
                       [--n 100000000] [--no-cpu-baseline] [--no-laws]
                       [--no-batched] [--no-mlp] [--no-c5] [--no-splitter]
                       [--no-study] [--no-types]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
# Algorithmic bytes each kernel must move per key it processes (keys only,
# float64): k_hist reads each key once (8 B); the scatter and the base-case
# sorts read it and write it once (16 B).
BYTES_PER_KEY = {"k_hist": 8.0, "k_scatter": 16.0, "k_base_small": 16.0, "k_base_big": 16.0}
STREAM_OF = {"k_hist": "read", "k_scatter": "copy", "k_base_small": "copy", "k_base_big": "copy"}
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2307_08637_amd", "csrc", f)
                  for f in ("lsort_kernels.hip", "lsort_dev.hpp", "lsort_internal.hpp")]
SIGN = -(1 << 63)
PAY_MUL = 0x2545F4914F6CDD1D                    # odd: index * PAY_MUL (mod 2^64) is a bijection
PAY_MUL_INV = pow(PAY_MUL, -1, 1 << 64) - (1 << 64) if pow(PAY_MUL, -1, 1 << 64) >= 1 << 63 else pow(PAY_MUL, -1, 1 << 64)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--n", type=int, default=100_000_000)
    p.add_argument("--law", default="normal")
    p.add_argument("--seed", type=int, default=21)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-laws", action="store_true", help="skip the per-law table")
    p.add_argument("--no-batched", action="store_true", help="skip the batched-form measurement")
    p.add_argument("--batched-arrays", type=int, default=10_000, help="arrays of the batched workload")
    p.add_argument("--no-mlp", action="store_true", help="skip the learned-parts comparison")
    p.add_argument("--no-c5", action="store_true", help="skip the learned-parts comparison at 1e9 keys")
    p.add_argument("--no-splitter", action="store_true", help="time the learned sort only (for profiling)")
    p.add_argument("--no-pivots", action="store_true", help="skip the pivot-quality metric")
    p.add_argument("--no-study", action="store_true", help="skip the sampling / refit study")
    p.add_argument("--no-types", action="store_true", help="skip the other key types and payload widths")
    p.add_argument("--mlp-n", type=int, default=100_000_000, help="keys of the piecewise-law comparison")
    p.add_argument("--c5-n", type=int, default=1_000_000_000, help="keys of the large piecewise-law comparison")
    return p.parse_args()


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def log(*x):
    print("[bench]", *x, file=sys.stderr, flush=True)


# -- properties of an output (GPU, any size) ----------------------------------------------

def order_key(t, torch):
    """int64 whose signed order is the keys' order (totalOrder for float64)."""
    b = t.view(torch.int64)
    if t.dtype == torch.uint64:
        return b ^ SIGN
    return torch.where(b < 0, b ^ 0x7FFFFFFFFFFFFFFF, b)


def mix_hash(x, torch, salt=0):
    """Wrapping sum of a 64-bit mix of every element (equal for any
    permutation of the same multiset); x: int64 tensor."""
    def lsr(z, s):
        return (z >> s) & ((1 << (64 - s)) - 1)
    z = x ^ salt
    z = (z ^ lsr(z, 30)) * -4658895280553007687   # 0xBF58476D1CE4E5B9
    z = (z ^ lsr(z, 27)) * -7723592293110705685   # 0x94D049BB133111EB
    z = z ^ lsr(z, 31)
    return int(z.sum().item())


def multiset(t, torch):
    x = t.view(torch.int64)
    return (t.numel(), mix_hash(x, torch), mix_hash(x, torch, 0x5A5A5A5A5A5A5A5))


def is_sorted(t, torch):
    k = order_key(t, torch)
    return t.numel() < 2 or bool((k[:-1] <= k[1:]).all().item())


# -- the headline sort -------------------------------------------------------------------------

def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2307_08637_amd import inputs, lsort

    dev = torch.device("cuda:0")
    lsort.lib()  # fail loudly if the HIP library is missing

    log("generating", a.n, a.law)
    host = inputs.generate(a.law, a.n, seed=a.seed)
    dtype = torch.uint64 if host.dtype == np.uint64 else torch.float64
    base = torch.from_numpy(host.view(np.int64) if host.dtype == np.uint64 else host).to(dev).view(dtype)
    base_ms = multiset(base, torch)
    bufs = [torch.empty_like(base) for _ in range(a.steps)]
    warm = torch.empty_like(base)

    def run(model, steps, timed_bufs):
        for _ in range(a.warmup):
            warm.copy_(base)
            lsort.sort(warm, model=model, stats=False)
        for b in timed_bufs[:steps]:
            b.copy_(base)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        for b in timed_bufs[:steps]:
            lsort.sort(b, model=model, stats=False)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # the same sorts again with a HIP event pair around every kernel
        # launch (the per-kernel durations of the roofline); kept out of the
        # step time above, which the events would lengthen
        for b in timed_bufs[:steps]:
            b.copy_(base)
        torch.cuda.synchronize()
        lsort.timing(True)
        for b in timed_bufs[:steps]:
            lsort.sort(b, model=model, stats=False)
        torch.cuda.synchronize()
        kern = lsort.timing_read()
        recs = lsort.timing_records()
        lsort.timing(False)
        warm.copy_(base)  # one more (untimed) sort for the per-level statistics
        lsort.sort(warm, model=model)
        st = lsort.stats()
        # every timed output is a sorted permutation of the input
        for b in timed_bufs[:steps]:
            if not is_sorted(b, torch) or multiset(b, torch) != base_ms:
                raise SystemExit(f"bench: output of model={model} is not a sorted permutation of the input")
        ms = e0.elapsed_time(e1) / steps
        return {"ms_per_step": ms, "wall_ms_per_step": 1e3 * wall / steps, "kernels": kern, "records": recs,
                "stats": st}

    log("learned", a.steps, "steps")
    L = run("auto", a.steps, bufs)
    log("reference streams")
    cal = calibrate(base, warm, lsort, torch, a.steps)
    S = None
    if not a.no_splitter:
        log("splitter", a.steps, "steps")
        S = run("splitter", a.steps, bufs)
    gpu_out = bufs[0].clone() if not a.no_splitter else None  # a sorted copy (the splitter's, same bytes)
    if gpu_out is None:
        bufs[0].copy_(base)
        lsort.sort(bufs[0], stats=False)
        gpu_out = bufs[0].clone()

    gk = lambda r: a.n / (r["ms_per_step"] * 1e-3) / 1e9  # noqa: E731
    kern = L["kernels"]
    dom = max((k for k in kern if k in BYTES_PER_KEY), key=lambda k: kern[k]["ms"])
    dk = kern[dom]
    avg_ms = dk["ms"] / dk["launches"]
    avg_bytes = dk["keys"] * BYTES_PER_KEY[dom] / dk["launches"]
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        with open(PROFILE_TRAFFIC) as f:
            tr = json.load(f)
        if tr.get("kernel") == dom and tr.get("source_sha") == kernel_source_sha() and tr.get("workload") == \
                f"{a.n} {a.law} learned":
            traffic = tr.get("bytes_per_launch")

    def level_summary(st):
        return [{"segments": lv["segments"], "keys": lv["keys"], "learned": lv["learned"], "tree": lv["tree"],
                 "radix": lv["radix"], "max_over_mean": lv["max_bucket_x1000_over_mean"] / 1000.0,
                 "fallback": lv["fallback"]} for lv in st["levels"]]

    pivots = None
    if not a.no_pivots:
        log("pivot quality")
        pivots = pivot_quality(base, gpu_out, lsort, torch, seed=a.seed)

    laws = {}
    if not a.no_laws and S is not None:
        for law in ("uniform", "normal", "lognormal", "exponential", "chisquared", "mixgauss", "u64",
                    "rootdups", "twodups", "zipf"):
            if law == a.law:
                laws[law] = {"learned": round(gk(L), 3), "splitter": round(gk(S), 3)}
                continue
            log("law", law)
            h = inputs.generate(law, a.n, seed=a.seed)
            dt = torch.uint64 if h.dtype == np.uint64 else torch.float64
            src = torch.from_numpy(h.view(np.int64) if h.dtype == np.uint64 else h).to(dev).view(dt)
            bb = [b.view(dt) for b in bufs[:3]]
            rl, stl = run_on(src, bb, "auto", lsort, torch)
            rs, _ = run_on(src, bb, "splitter", lsort, torch)
            laws[law] = {"learned": round(a.n / (rl * 1e-3) / 1e9, 3), "splitter": round(a.n / (rs * 1e-3) / 1e9, 3),
                         "first_level": "learned" if stl["levels"][0]["learned"] else "tree"}
            del src, h

    # the CPU oracle on the same keys (rank 0, one GPU): its rate, and the GPU
    # output compared with its output word for word
    cpu = None
    oracle_equal = None
    if not a.no_cpu_baseline:
        import oracle
        model, avail = host_cpu()
        log("oracle on", a.n, "keys")
        t0 = time.perf_counter()
        want, _ = oracle.sort(host)
        dt = time.perf_counter() - t0
        got = gpu_out.view(torch.int64).cpu().numpy()
        oracle_equal = bool(np.array_equal(got, want.view(np.int64)))
        if not oracle_equal:
            raise SystemExit("bench: GPU output differs from the oracle's")
        cpu = {"value": round(a.n / dt / 1e9, 6), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
               "sample": f"the same {a.n} {a.law} keys, one single-threaded oracle sort (stable bottom-up merge "
                         f"sort) in {dt:.1f} s; 1 core used of nproc = {avail}, {model}"}
        del want, got
    del gpu_out

    bufs = warm = None
    batched = None
    if not a.no_batched:
        torch.cuda.empty_cache()
        batched = run_batched(inputs, lsort, torch, np, dev, a.batched_arrays)
    mlp = None
    if not a.no_mlp:
        torch.cuda.empty_cache()
        mlp = {"n_1e8": run_learned_parts(inputs, lsort, torch, np, dev, a.mlp_n, a.seed, reps=3)}
        if not a.no_c5:
            torch.cuda.empty_cache()
            mlp["n_1e9"] = run_learned_parts(inputs, lsort, torch, np, dev, a.c5_n, a.seed, reps=2)

    study = None
    if not a.no_study:
        torch.cuda.empty_cache()
        study = run_sampling_study(inputs, lsort, torch, np, dev, a.n, a.seed)

    base_case = None
    if not a.no_study:
        torch.cuda.empty_cache()
        base_case = run_base_case(inputs, lsort, torch, np, dev, a.n, a.seed)

    types = None
    if not a.no_types:
        torch.cuda.empty_cache()
        types = run_types(inputs, lsort, torch, np, dev, a.n, a.seed)

    per_level = per_level_rates(L["records"], a.n, a.steps)
    out = {
        "metric": "Gkeys/s sorting 1e8 f64 keys, learned vs splitter buckets; % HBM peak",
        "value": round(gk(L), 4),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(L["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if dtype == torch.float64 else "u64",
        "data": "synthetic",
        "config": {"workload": f"sort {a.n} {'float64' if dtype == torch.float64 else 'uint64'} keys, law {a.law}, "
                               f"learned RMI partitioning (1% sample, 1000 leaves, 1000 buckets), stable, in place",
                   "n": a.n, "law": a.law, "seed": a.seed, "model": "auto"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_key": BYTES_PER_KEY[dom], "avg_launch_ms": round(avg_ms, 4),
                     "launches": dk["launches"],
                     # against the reference stream of the same access pattern
                     "frac_of_stream": round(achieved / cal[STREAM_OF[dom]]["GB/s"], 4)},
        "partition_passes": per_level,
        "streams": cal,
        "cpu_baseline": cpu,
        "output_check": {"sorted": True, "multiset_equal": True, "oracle_equal": oracle_equal},
        "pivot_quality": pivots,
        "splitter": None if S is None else {"value": round(gk(S), 4), "ms_per_step": round(S["ms_per_step"], 4),
                                            "levels": level_summary(S["stats"])},
        "learned_over_splitter": None if S is None else round(gk(L) / gk(S), 4),
        "levels": level_summary(L["stats"]),
        "kernels": {k: {"launches": v["launches"], "ms_per_step": round(v["ms"] / a.steps, 4),
                        "keys_per_step": v["keys"] / a.steps} for k, v in kern.items()},
        "wall_ms_per_step": round(L["wall_ms_per_step"], 4),
        "laws": laws,
        "batched": batched,
        "learned_parts": mlp,
        "sampling_study": study,
        "key_types": types,
        "base_case": base_case,
    }
    print(json.dumps(out), flush=True)


def per_level_rates(recs, n, steps):
    """Achieved HBM rate of each partition pass of the array (launches that
    processed all n keys, in launch order: level 0, then level 1), apart from
    the launches that sort the first level's sample."""
    res = {}
    for name in ("k_hist", "k_scatter"):
        rs = [(ms, keys) for nm, ms, keys in recs if nm == name]
        full = [ms for ms, keys in rs if keys == n]
        per = len(full) // max(steps, 1)
        for lv in range(per):
            sel = full[lv::per]
            ms = sum(sel) / len(sel)
            gbs = n * BYTES_PER_KEY[name] / (ms * 1e-3) / 1e9
            res[f"{name}_level{lv}"] = {"avg_ms": round(ms, 4), "GB/s": round(gbs, 1),
                                        "frac": round(gbs / HBM_PEAK_GBS, 4)}
        other = [ms for ms, keys in rs if keys != n]
        if other:
            res[f"{name}_sample_sort"] = {"launches_per_step": len(other) // max(steps, 1),
                                          "avg_ms": round(sum(other) / len(other), 4)}
    return res


def pivot_quality(src, out, lsort, torch, seed, B=256, L=1000, sample_frac=0.01):
    """Table 1 metric (Sec. 3.4): sum over B-1 pivots p_i of
    |P(A <= p_i) - (i + 1) / B|, P taken over the sorted keys `out`.
      learned:  the RMI's implicit pivots (Alg. 4: the largest key of each of
                B buckets), the RMI fitted on a 1% sample with L leaves; as
                the buckets do not decrease along sorted keys, P(A <= p_b) is
                the fraction of keys in buckets 0..b (an empty bucket repeats
                the previous pivot);
      splitter: the sample quantiles sample[floor((i + 1) S / B)] a splitter
                tree takes from the same 1% sample (Sec. 2.4);
      random:   B - 1 keys drawn at random from the input (the pivots of the
                paper's random-sample column)."""
    n = src.numel()
    dev = src.device
    S = max(int(n * sample_frac), B)
    smp = lsort.sample(src, seed, S)
    lsort.sort(smp, stats=False)
    tgt = torch.arange(1, B, dtype=torch.float64, device=dev) / B
    par = lsort.rmi_fit(smp, L, float(B))
    ids = lsort.rmi_buckets(out, par, L, float(B)).view(torch.int32).to(torch.int64)
    cum = torch.cumsum(torch.bincount(ids, minlength=B), 0)[:B - 1].to(torch.float64) / n
    learned = float((cum - tgt).abs().sum().item())
    okey = order_key(out, torch)

    def quality(piv):
        pos = torch.searchsorted(okey, order_key(piv, torch).contiguous(), right=True).to(torch.float64) / n
        return float((pos - tgt).abs().sum().item())
    q = (torch.arange(1, B, device=dev, dtype=torch.int64) * S) // B
    splitter = quality(smp[q])
    g = torch.Generator(device="cpu").manual_seed(seed)
    ridx = torch.randint(0, n, (B - 1,), generator=g).to(dev)
    rnd = src[ridx].clone()
    rk = order_key(rnd, torch)
    rnd = rnd[torch.argsort(rk)]
    random_q = quality(rnd)
    return {"buckets": B, "sample": S, "leaves": L, "learned_rmi": round(learned, 4),
            "splitter_quantiles": round(splitter, 4), "random": round(random_q, 4),
            "paper_table1_uniform": {"random": 1.1016, "rmi": 0.4388}}


def calibrate(src, dst, lsort, torch, reps):
    """The library's reference streams over the benchmark's key buffer: a
    copy (read + write of every word) and a read-only sum, timed with HIP
    events on the stream they run on; the practical ceilings of a scatter /
    base-case pass and of a histogram pass."""
    nbytes = src.numel() * 8
    out = torch.empty(2, dtype=torch.uint64, device=src.device)
    for _ in range(2):
        lsort.stream_copy(src, dst)
        lsort.stream_read(src, out)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(reps):
        lsort.stream_copy(src, dst)
    e[1].record()
    for _ in range(reps):
        lsort.stream_read(src, out)
    e[2].record()
    torch.cuda.synchronize()
    copy_ms, read_ms = e[0].elapsed_time(e[1]) / reps, e[1].elapsed_time(e[2]) / reps
    copy_gbs, read_gbs = 2 * nbytes / copy_ms / 1e6, nbytes / read_ms / 1e6
    return {"bytes": nbytes,
            "copy": {"ms": round(copy_ms, 4), "GB/s": round(copy_gbs, 1), "frac": round(copy_gbs / HBM_PEAK_GBS, 4)},
            "read": {"ms": round(read_ms, 4), "GB/s": round(read_gbs, 1), "frac": round(read_gbs / HBM_PEAK_GBS, 4)}}


def time_call(fn, reps, before, torch):
    """Mean ms of fn() over reps calls after one untimed call; before() runs
    (untimed) ahead of each call."""
    tot = 0.0
    for r in range(reps + 1):
        before()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        if r:
            tot += e0.elapsed_time(e1)
    return tot / reps


def run_batched(inputs, lsort, torch, np, dev, arrays):
    """sort_segmented over the batched workload (sizes log-uniform in
    [1e3, 1e6], five float64 laws, uint32 payload = index in its array):
    all `arrays` arrays, and its leading arrays up to 2e8 keys; learned vs
    splitter with a host read-back per level; the fixed-level form eager and
    replayed from a captured graph (caller-owned workspace).  Restore copies
    are outside the timed region."""
    log("batched: generating", arrays, "arrays")
    keys, off, pay, _ = inputs.segmented(arrays, seed=41)
    n, m = keys.size, off.size - 1
    cut = int(np.searchsorted(off[1:], 200_000_000)) + 1  # arrays of the 2e8 prefix
    k0 = torch.from_numpy(keys).to(dev)
    p0 = torch.from_numpy(pay.view(np.int32)).to(dev)
    o = torch.from_numpy(off.view(np.int64)).to(dev).view(torch.uint64)
    del keys, pay
    k = torch.empty_like(k0)
    p = torch.empty_like(p0)
    pu = p.view(torch.uint32)

    def restore(nk=n):
        k[:nk].copy_(k0[:nk])
        p[:nk].copy_(p0[:nk])

    res = {"workload": f"{m} arrays (sizes log-uniform in [1e3, 1e6], five float64 laws) = {n} keys + uint32 "
                       f"payload, stable", "arrays": m, "keys": n}
    for name, opts in (("learned", {}), ("splitter", {"model": "splitter"})):
        log("batched:", name)
        ms = time_call(lambda: lsort.sort_segmented(k, o, pu, stats=False, **opts), 3, restore, torch)
        res[name] = {"ms": round(ms, 3), "Gkeys/s": round(n / (ms * 1e-3) / 1e9, 3)}
    # the output: every array sorted, payload stable, (key, payload, array) pairs the same multiset
    restore()
    seg = torch.repeat_interleave(torch.arange(m, device=dev), torch.from_numpy(np.diff(off).astype(np.int64)).to(dev))

    def pair_hash(kk, pp):
        return mix_hash(kk.view(torch.int64) ^ ((pp.to(torch.int64) & 0xFFFFFFFF) << 17) ^ (seg << 45), torch)
    h0 = pair_hash(k, p)
    lsort.sort_segmented(k, o, pu, stats=False)
    kk = order_key(k, torch)
    same = seg[:-1] == seg[1:]
    ok = bool(((kk[:-1] <= kk[1:]) | ~same).all().item())
    tie = same & (kk[:-1] == kk[1:])
    pi = p.to(torch.int64) & 0xFFFFFFFF
    ok = ok and bool(((pi[:-1] < pi[1:]) | ~tie).all().item()) and pair_hash(k, p) == h0
    del kk, same, tie, pi
    if not ok:
        raise SystemExit("bench: batched output is not a stable per-array sort of the input")
    ref_k, ref_p = k.clone(), p.clone()
    res["output_check"] = {"sorted_per_array": True, "stable": True, "pair_multiset_equal": True}
    # the 2e8-key prefix
    npre = int(off[cut])
    opre = o[:cut + 1]
    for name, opts in (("learned", {}), ("splitter", {"model": "splitter"})):
        ms = time_call(lambda: lsort.sort_segmented(k[:npre], opre, pu[:npre], stats=False, **opts), 3,
                       lambda: restore(npre), torch)
        res.setdefault("prefix_2e8", {"arrays": cut, "keys": npre})[name] = {
            "ms": round(ms, 3), "Gkeys/s": round(npre / (ms * 1e-3) / 1e9, 3)}
    # fixed levels (no host read-back): eager, then a captured graph replayed
    log("batched: fixed levels and graph replay")
    nbytes = lsort.workspace_bytes(n, m, payload=True, fixed_levels=True)
    ws = torch.empty((nbytes + 7) // 8, dtype=torch.int64, device=dev)
    lsort.set_workspace(ws)
    try:
        fixed = dict(fixed_levels=True, stats=False)
        ms = time_call(lambda: lsort.sort_segmented(k, o, pu, **fixed), 3, restore, torch)
        res["fixed_levels_eager"] = {"ms": round(ms, 3), "Gkeys/s": round(n / (ms * 1e-3) / 1e9, 3)}
        restore()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            lsort.sort_segmented(k, o, pu, **fixed)
        ms = time_call(g.replay, 3, restore, torch)
        equal = bool(torch.equal(k, ref_k) and torch.equal(p, ref_p))
        ovf = lsort.stats()["overflow"]
        res["graph_replay"] = {"ms": round(ms, 3), "Gkeys/s": round(n / (ms * 1e-3) / 1e9, 3),
                               "output_equal_to_readback_path": equal, "overflow": ovf}
        if not equal or ovf:
            raise SystemExit("bench: graph replay output differs from the read-back path")
        del g
    finally:
        torch.cuda.synchronize()
        lsort.set_workspace(None)
    del ws, k0, p0, k, p, ref_k, ref_p, seg
    return res


def run_learned_parts(inputs, lsort, torch, np, dev, n, seed, reps):
    """The piecewise law (70% LogNormal(0, 2), 20% 1e6 + U[0, 1), 10% N(-5e3, 1)):
    the RMI, the MLP-rooted model (200 Adam steps on a 1e6-key training set)
    and the splitter tree as the first level; first-level max/mean bucket
    ratio, fallbacks and Gkeys/s; every output checked sorted and the same
    multiset as the input."""
    log("learned parts: generating", n)
    h = inputs.generate("piecewise", n, seed=seed + 30)
    src = torch.from_numpy(h).to(dev)
    del h
    ms0 = multiset(src, torch)
    buf = torch.empty_like(src)
    res = {"workload": f"sort {n} float64 keys, piecewise law 70/20/10, out-of-place copy restored per run"}
    for name, model, opts in (("rmi", "auto", {}), ("rmi_no_judge", "auto", {"balance_pct": 100}), ("mlp", "mlp", {}),
                              ("splitter", "splitter", {})):
        log("learned parts:", name, n)
        ms = time_call(lambda: lsort.sort(buf, model=model, stats=False, **opts), reps, lambda: buf.copy_(src), torch)
        buf.copy_(src)  # one more (untimed) sort for the statistics and the check
        lsort.sort(buf, model=model, **opts)
        st = lsort.stats()
        if not is_sorted(buf, torch) or multiset(buf, torch) != ms0:
            raise SystemExit(f"bench: learned-parts output of {name} is not a sorted permutation")
        lv0 = st["levels"][0]
        res[name] = {"ms": round(ms, 3), "Gkeys/s": round(n / (ms * 1e-3) / 1e9, 3),
                     "first_level_model": {1: "rmi", 2: "mlp", 3: "splitter"}.get(st["first_model"], "auto"),
                     "first_level_max_over_mean": lv0["max_bucket_x1000_over_mean"] / 1000.0,
                     "first_level_fallbacks": lv0["fallback"], "levels": len(st["levels"])}
        if name == "mlp":
            res[name]["loss_first"] = st["mlp_loss_first"]
            res[name]["loss_best"] = st["mlp_loss_last"]
    del src, buf
    return res


def run_on(src, bufs, model, lsort, torch, **opts):
    """ms per sort of `src` (K = len(bufs) copies, after one warm-up), and
    the statistics of one more sort."""
    tmp = bufs[0]
    tmp.copy_(src)
    lsort.sort(tmp, model=model, stats=False, **opts)
    for b in bufs:
        b.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for b in bufs:
        lsort.sort(b, model=model, stats=False, **opts)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / len(bufs)
    tmp.copy_(src)
    lsort.sort(tmp, model=model, **opts)
    return ms, lsort.stats()


def run_base_case(inputs, lsort, torch, np, dev, n, seed, reps=3):
    """The base case two ways on the same first-level buckets: the
    comparison sorts (register bitonic networks, the default) against the
    model-placed counting sort (LS_FLAG_MODEL_BASE: the RMI's fine position
    places each key, its rank inside its bin finishes it), per law at n
    keys: whole-sort time and each base-case kernel's time per sort."""
    res = {"n": n}
    for law in ("normal", "lognormal"):
        h = inputs.generate(law, n, seed=seed)
        src = torch.from_numpy(h).to(dev)
        del h
        ms0 = multiset(src, torch)
        buf = torch.empty_like(src)
        row = {}
        for name, mb in (("comparison_sort", False), ("model_placed", True)):
            log("base case:", law, name)
            ms = time_call(lambda: lsort.sort(buf, stats=False, model_base=mb), reps, lambda: buf.copy_(src), torch)
            if not is_sorted(buf, torch) or multiset(buf, torch) != ms0:
                raise SystemExit(f"bench: base-case output ({law}, {name}) is not a sorted permutation")
            buf.copy_(src)
            torch.cuda.synchronize()
            lsort.timing(True)
            lsort.sort(buf, stats=False, model_base=mb)
            torch.cuda.synchronize()
            kern = lsort.timing_read()
            lsort.timing(False)
            row[name] = {"ms": round(ms, 4), "Gkeys/s": round(n / (ms * 1e-3) / 1e9, 3),
                         "base_kernels": {k: {"ms": round(v["ms"], 4), "keys": v["keys"]} for k, v in kern.items()
                                          if k.startswith("k_base")}}
        res[law] = row
        del src, buf
    return res


def run_types(inputs, lsort, torch, np, dev, n, seed, reps=3):
    """float32 keys (the normal law rounded to float32), int64 keys (the
    uniform 64-bit law read as signed) and float64 keys with a 64-bit
    payload: Gkeys/s of the whole call (the maps around the engine
    included), each output checked sorted and the same multiset."""
    res = {"n": n}
    h = inputs.generate("normal", n, seed=seed)
    cases = [("float32", torch.from_numpy(h.astype(np.float32)).to(dev), None),
             ("int64", torch.from_numpy(inputs.generate("u64", n, seed=seed).view(np.int64)).to(dev), None),
             ("float64_payload64", torch.from_numpy(h).to(dev),
              torch.arange(n, dtype=torch.int64, device=dev).mul_(PAY_MUL))]
    del h
    for name, src, pay in cases:
        log("key types:", name)
        buf = torch.empty_like(src)
        pbuf = None if pay is None else torch.empty_like(pay)

        def before():
            buf.copy_(src)
            if pay is not None:
                pbuf.copy_(pay)
        ms = time_call(lambda: lsort.sort(buf, pbuf, stats=False), reps, before, torch)
        before()
        lsort.sort(buf, pbuf, stats=False)
        k = buf.view(torch.int32).to(torch.int64) if src.dtype == torch.float32 else buf.view(torch.int64)
        if src.dtype == torch.float32:
            kk = torch.where(k < 0, k ^ 0x7FFFFFFF, k)
        else:
            kk = k if src.dtype == torch.int64 else torch.where(k < 0, k ^ 0x7FFFFFFF_FFFFFFFF, k)
        ok = bool((kk[:-1] <= kk[1:]).all().item())
        s0 = src.view(torch.int32).to(torch.int64) if src.dtype == torch.float32 else src.view(torch.int64)
        ok = ok and mix_hash(k, torch) == mix_hash(s0, torch)
        if pay is not None:  # payload: the key's original index times an odd constant, so it names the key
            idx = pbuf * PAY_MUL_INV  # (wrapping) the original index back
            ok = ok and bool(((idx >= 0) & (idx < n)).all().item()) and torch.equal(src[idx], buf)
            del idx
        if not ok:
            raise SystemExit(f"bench: output for key type {name} is not a sorted permutation")
        res[name] = {"ms": round(ms, 3), "Gkeys/s": round(n / (ms * 1e-3) / 1e9, 3)}
        del buf, pbuf, k, kk, s0
    return res


def run_sampling_study(inputs, lsort, torch, np, dev, n, seed, laws=("normal", "lognormal")):
    """The sample-once vs sample-per-call question (Sec. 3.3: LearnedSort
    samples once and reuses its model; Sec. 5.1: AIPS2o trains a model per
    recursive call) and the sample size (Sec. 6 future work on sampling):
    per law at n keys, the reused model (default) against a fresh model per
    bucket (refit), and the 1% sample against smaller and larger ones --
    Gkeys/s, max/mean bucket ratio per level, fallbacks, and the Table 1
    pivot quality of the RMI fitted on that sample.  Every output is checked
    sorted and the same multiset as the input."""
    res = {"n": n, "workload": f"sort {n} float64 keys per law, 3 timed sorts per configuration"}
    bufs = None
    for law in laws:
        log("sampling study:", law)
        h = inputs.generate(law, n, seed=seed)
        src = torch.from_numpy(h).to(dev)
        del h
        ms0 = multiset(src, torch)
        if bufs is None:
            bufs = [torch.empty_like(src) for _ in range(3)]
        ref = bufs[0]
        ref.copy_(src)
        lsort.sort(ref, stats=False)
        out = ref.clone()
        row = {}
        configs = [("reuse", {}), ("refit", {"refit": True})] + [
            (f"sample_{f:g}", {"sample_frac": f}) for f in (0.001, 0.0025, 0.04)]
        for name, opts in configs:
            ms, st = run_on(src, bufs, "auto", lsort, torch, **opts)
            for b in bufs:
                if not is_sorted(b, torch) or multiset(b, torch) != ms0:
                    raise SystemExit(f"bench: sampling-study output ({law}, {name}) is not a sorted permutation")
            lv = st["levels"]
            row[name] = {"Gkeys/s": round(n / (ms * 1e-3) / 1e9, 3), "ms": round(ms, 4),
                         "max_over_mean": [x["max_bucket_x1000_over_mean"] / 1000.0 for x in lv],
                         "fallback": [x["fallback"] for x in lv],
                         "learned_segments": [x["learned"] for x in lv], "tree_segments": [x["tree"] for x in lv]}
        for f in (0.001, 0.0025, 0.01, 0.04):
            q = pivot_quality(src, out, lsort, torch, seed, sample_frac=f)
            key = "reuse" if f == 0.01 else f"sample_{f:g}"
            row[key]["pivot_quality_rmi"] = q["learned_rmi"]
            row[key]["pivot_quality_splitter"] = q["splitter_quantiles"]
        res[law] = row
        del src, out
    del bufs
    return res


if __name__ == "__main__":
    main()
