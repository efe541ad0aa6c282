"""Summaries of rocprofv3 CSV output (kernel statistics and per-kernel PMC
averages) for the profiles/ notes.

  python -m paper_0912_3824_amd.profiling stats  <dir-with-*_kernel_stats.csv>
  python -m paper_0912_3824_amd.profiling pmc    <dir-with-*_counter_collection.csv>
"""
import csv
import glob
import os
import sys
from collections import defaultdict


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits


def kernel_stats(d):
    rows = []
    for f in _find(d, "kernel_stats.csv"):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    out = ["kernel | calls | total_us | avg_us | min_us | max_us | pct"]
    for r in rows:
        ns = float(r["TotalDurationNs"])
        out.append(f"{r['Name']} | {r['Calls']} | {ns / 1e3:.1f} | {float(r['AverageNs']) / 1e3:.3f} | "
                   f"{float(r['MinNs']) / 1e3:.3f} | {float(r['MaxNs']) / 1e3:.3f} | {float(r['Percentage']):.2f}")
    return "\n".join(out)


def pmc(d):
    acc = defaultdict(lambda: defaultdict(list))
    for f in _find(d, "counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                key = (r["Kernel_Name"], r.get("Grid_Size", ""))
                acc[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = ["kernel | grid | counter | dispatches | mean per dispatch"]
    for (k, g), cs in sorted(acc.items()):
        for c, v in sorted(cs.items()):
            out.append(f"{k} | {g} | {c} | {len(v)} | {sum(v) / len(v):.6g}")
    return "\n".join(out)


if __name__ == "__main__":
    mode, d = sys.argv[1], sys.argv[2]
    print(kernel_stats(d) if mode == "stats" else pmc(d))
