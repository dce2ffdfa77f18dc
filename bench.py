"""Benchmark: Gkeys/s sorting 1e8 float64 keys on one MI355X, learned (RMI)
partitioning vs the splitter-tree form, with the roofline of the dominant
kernel and the CPU oracle's rate on the host.

A step is one complete sort of the 1e8-key array (sampling, sample sort,
model fit, every partition level and the base case).  The keys of every
timed step are already in HBM: K unsorted copies are made before the timed
region and step k sorts copy k in place.

Besides the headline line it reports, in extra fields of the same JSON
object: the same sort per input law, the batched form (sort_segmented over
the 10,000-array workload's first 2e8 keys, with payload), and the learned
parts on the 70/20/10 piecewise law (RMI root vs MLP root vs splitter
tree: first-level max/mean bucket ratio and Gkeys/s).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--law normal]
                       [--n 100000000] [--no-cpu-baseline] [--no-laws]
                       [--no-batched] [--no-mlp] [--no-splitter]
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
    p.add_argument("--cpu-keys", type=int, default=50_000_000, help="keys in the oracle's timed sample")
    p.add_argument("--no-batched", action="store_true", help="skip the batched-form measurement")
    p.add_argument("--no-mlp", action="store_true", help="skip the learned-parts comparison")
    p.add_argument("--no-splitter", action="store_true", help="time the learned sort only (for profiling)")
    p.add_argument("--mlp-n", type=int, default=100_000_000, help="keys of the piecewise-law comparison")
    return p.parse_args()


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

    def log(*x):
        print("[bench]", *x, file=sys.stderr, flush=True)

    log("generating", a.n, a.law)
    host = inputs.generate(a.law, a.n, seed=a.seed)
    dtype = torch.uint64 if host.dtype == np.uint64 else torch.float64
    base = torch.from_numpy(host.view(np.int64) if host.dtype == np.uint64 else host).to(dev).view(dtype)
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
        lsort.timing(False)
        warm.copy_(base)  # one more (untimed) sort for the per-level statistics
        lsort.sort(warm, model=model)
        st = lsort.stats()
        # the result must be a sorted permutation (cheap properties on the GPU)
        k = timed_bufs[0].view(torch.int64)
        key = k ^ (-(1 << 63)) if dtype == torch.uint64 else torch.where(k < 0, k ^ 0x7FFFFFFFFFFFFFFF, k)
        if not bool((key[:-1] <= key[1:]).all().item()):
            raise SystemExit(f"bench: output of model={model} is not sorted")
        ms = e0.elapsed_time(e1) / steps
        return {"ms_per_step": ms, "wall_ms_per_step": 1e3 * wall / steps, "kernels": kern, "stats": st}

    log("learned", a.steps, "steps")
    L = run("auto", a.steps, bufs)
    log("reference streams")
    cal = calibrate(base, warm, lsort, torch, a.steps)
    S = None
    if not a.no_splitter:
        log("splitter", a.steps, "steps")
        S = run("splitter", a.steps, bufs)

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

    laws = {}
    if not a.no_laws and S is not None:
        for law in ("uniform", "normal", "lognormal", "exponential", "chisquared", "mixgauss", "u64"):
            if law == a.law:
                laws[law] = {"learned": round(gk(L), 3), "splitter": round(gk(S), 3)}
                continue
            log("law", law)
            h = inputs.generate(law, a.n, seed=a.seed)
            dt = torch.uint64 if h.dtype == np.uint64 else torch.float64
            src = torch.from_numpy(h.view(np.int64) if h.dtype == np.uint64 else h).to(dev).view(dt)
            bb = [b.view(dt) for b in bufs[:3]]
            rl = run_on(src, bb, "auto", lsort, torch)
            rs = run_on(src, bb, "splitter", lsort, torch)
            laws[law] = {"learned": round(a.n / (rl * 1e-3) / 1e9, 3), "splitter": round(a.n / (rs * 1e-3) / 1e9, 3)}
            del src, h

    batched = None
    if not a.no_batched:
        bufs = warm = None
        torch.cuda.empty_cache()
        batched = run_batched(inputs, lsort, torch, np, dev, log)
    mlp = None
    if not a.no_mlp:
        torch.cuda.empty_cache()
        mlp = run_learned_parts(inputs, lsort, torch, np, dev, log, a.mlp_n, a.seed)

    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        m = min(a.cpu_keys, a.n)
        log("oracle on", m, "keys")
        t0 = time.perf_counter()
        oracle.sort(host[:m])
        dt = time.perf_counter() - t0
        cpu = {"value": round(m / dt / 1e9, 6), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
               "sample": f"first {m} of the same {a.n} {a.law} keys, one single-threaded oracle sort "
                         f"({dt:.1f} s) on {os.cpu_count()} host CPUs"}

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
        "streams": cal,
        "cpu_baseline": cpu,
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
    }
    print(json.dumps(out), flush=True)


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


def run_batched(inputs, lsort, torch, np, dev, log):
    """sort_segmented over the 10,000-array workload (sizes log-uniform in
    [1e3, 1e6], five float64 laws, uint32 payload) up to its first 2e8
    keys; restore copies are outside the timed region."""
    log("batched: generating")
    keys, off, pay, _ = inputs.segmented(10_000, seed=41, max_total=200_000_000)
    k0 = torch.from_numpy(keys).to(dev)
    p0 = torch.from_numpy(pay.view(np.int32)).to(dev).view(torch.uint32)
    o = torch.from_numpy(off.view(np.int64)).to(dev).view(torch.uint64)
    k, p = torch.empty_like(k0), torch.empty_like(p0)
    del keys, pay
    res = {}
    for name, opts in (("learned", {}), ("splitter", {"model": "splitter"})):
        log("batched:", name)
        tot = 0.0
        reps = 3
        for r in range(reps + 1):
            k.copy_(k0)
            p.view(torch.int32).copy_(p0.view(torch.int32))
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            lsort.sort_segmented(k, o, p, stats=False, **opts)
            e1.record()
            torch.cuda.synchronize()
            if r:
                tot += e0.elapsed_time(e1)
        ms = tot / reps
        res[name] = {"ms": round(ms, 3), "Gkeys/s": round(k0.numel() / (ms * 1e-3) / 1e9, 3)}
    return {"workload": f"{off.size - 1} arrays (sizes log-uniform in [1e3, 1e6], five float64 laws) = "
                        f"{int(off[-1])} keys + uint32 payload, stable", **res}


def run_learned_parts(inputs, lsort, torch, np, dev, log, n, seed):
    """The piecewise law (70% LogNormal(0, 2), 20% 1e6 + U[0, 1), 10% N(-5e3, 1)):
    the RMI, the MLP-rooted model (200 Adam steps) and the splitter tree as
    the first level; first-level max/mean bucket ratio and Gkeys/s."""
    log("learned parts: generating", n)
    h = inputs.generate("piecewise", n, seed=seed + 30)
    src = torch.from_numpy(h).to(dev)
    del h
    buf = torch.empty_like(src)
    res = {"workload": f"sort {n} float64 keys, piecewise law 70/20/10"}
    for name, model in (("rmi", "auto"), ("mlp", "mlp"), ("splitter", "splitter")):
        log("learned parts:", name)
        tot = 0.0
        reps = 3
        for r in range(reps + 1):
            buf.copy_(src)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            lsort.sort(buf, model=model, stats=False)
            e1.record()
            torch.cuda.synchronize()
            if r:
                tot += e0.elapsed_time(e1)
        buf.copy_(src)  # one more (untimed) sort for the statistics
        lsort.sort(buf, model=model)
        st = lsort.stats()
        lv0 = st["levels"][0]
        ms = tot / reps
        res[name] = {"ms": round(ms, 3), "Gkeys/s": round(n / (ms * 1e-3) / 1e9, 3),
                     "first_level_max_over_mean": lv0["max_bucket_x1000_over_mean"] / 1000.0,
                     "first_level_fallbacks": lv0["fallback"], "levels": len(st["levels"])}
        if name == "mlp":
            res[name]["loss_first"] = st["mlp_loss_first"]
            res[name]["loss_best"] = st["mlp_loss_last"]
    return res


def run_on(src, bufs, model, lsort, torch):
    """ms per sort of `src` (K = len(bufs) copies, after one warm-up)."""
    tmp = bufs[0]
    tmp.copy_(src)
    lsort.sort(tmp, model=model, stats=False)
    for b in bufs:
        b.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for b in bufs:
        lsort.sort(b, model=model, stats=False)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / len(bufs)


if __name__ == "__main__":
    main()
