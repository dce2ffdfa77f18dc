"""Summaries of rocprofv3 output for the sort's kernels.

  python -m paper_2307_08637_amd.profile_summary kernels STATS_CSV
      text table of a --kernel-trace --stats run (name, calls, total ms,
      average us, share)
  python -m paper_2307_08637_amd.profile_summary traffic FETCH_CSV WRITE_CSV KERNEL OUT_JSON
        [--name NAME] [--command TEXT] [--copy-bytes BYTES]
      HBM bytes per dispatch of KERNEL from two --pmc runs (FETCH_SIZE,
      WRITE_SIZE; KiB per dispatch), each scaled by what the counter reads
      for the runtime's buffer-copy kernel of the same run against the bytes
      that copy moves, written as JSON with the hash of the kernel sources
      (NAME: the kernel's name in the benchmark's timing table, when it
      differs from the rocprofv3 name; TEXT: the profiled command)

The copy used for calibration is the largest __amd_rocclr_copyBuffer
dispatch in each run; its size in bytes is passed as --copy-bytes (default
8e8: the benchmark's 1e8 float64 keys).
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2307_08637_amd", "csrc", f)
                  for f in ("lsort_kernels.hip", "lsort_dev.hpp", "lsort_internal.hpp")]


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    name = name.strip('"')
    for pre in ("void ", "ls::"):
        name = name.replace(pre, "")
    name = name.split("(")[0]
    if name.startswith("at::native::"):  # torch's own kernels (the output check): name and functor
        parts = [x for x in name.replace("<", " ").replace(">", " ").replace(",", " ").split() if "::" in x]
        name = "torch " + " ".join(x.split("::")[-1] for x in parts[:2])
    return name[:34]


def kernels(stats_csv: str) -> str:
    rows = list(csv.DictReader(open(stats_csv)))
    out = [f"{'kernel':34s} {'calls':>6s} {'total ms':>10s} {'avg us':>10s} {'share %':>8s}"]
    for r in rows:
        out.append(f"{short(r['Name']):34s} {int(r['Calls']):6d} {int(r['TotalDurationNs']) / 1e6:10.3f} "
                   f"{float(r['AverageNs']) / 1e3:10.1f} {float(r['Percentage']):8.2f}")
    return "\n".join(out)


def _per_dispatch(path: str, counter: str):
    acc = defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        d = int(r["Dispatch_Id"])
        acc[d] += float(r["Counter_Value"])
        names[d] = short(r["Kernel_Name"])
    return acc, names


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: float):
    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        acc, names = _per_dispatch(path, counter)
        copies = [acc[d] for d in acc if names[d] == "__amd_rocclr_copyBuffer"]
        if not copies:
            raise SystemExit(f"{path}: no copy kernel to calibrate against")
        factor = copy_bytes / (max(copies) * 1024.0)
        vals = [acc[d] * 1024.0 * factor for d in acc if names[d] == kernel]
        if not vals:
            raise SystemExit(f"{path}: no dispatch of {kernel}")
        res[counter] = {"factor": round(factor, 4), "dispatches": len(vals), "bytes_per_launch": sum(vals) / len(vals)}
    return res


def main(argv):
    if len(argv) >= 2 and argv[0] == "kernels":
        print(kernels(argv[1]))
        return
    if len(argv) >= 5 and argv[0] == "traffic":
        copy_bytes = 8e8
        if "--copy-bytes" in argv:
            copy_bytes = float(argv[argv.index("--copy-bytes") + 1])
        name = argv[argv.index("--name") + 1] if "--name" in argv else argv[3]
        t = traffic(argv[1], argv[2], argv[3], copy_bytes)
        out = {"kernel": name, "source_sha": kernel_source_sha(), "workload": os.environ.get("LSORT_WORKLOAD", ""),
               "fetch": t["FETCH_SIZE"], "write": t["WRITE_SIZE"],
               "bytes_per_launch": t["FETCH_SIZE"]["bytes_per_launch"] + t["WRITE_SIZE"]["bytes_per_launch"],
               "rocprof_kernel": argv[3]}
        if "--command" in argv:
            out["command"] = argv[argv.index("--command") + 1]
        with open(argv[4], "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps(out))
        return
    raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
