"""Summaries of rocprofv3 CSV output (kernel statistics, per-kernel PMC
averages, and calibrated HBM traffic per launch) for the profiles/ notes.

  python -m paper_0912_3824_amd.profiling stats   <dir-with-*_kernel_stats.csv>
  python -m paper_0912_3824_amd.profiling pmc     <dir-with-*_counter_collection.csv>
  python -m paper_0912_3824_amd.profiling traffic <fetch-dir> <write-dir> --kernel REGEX
        [--copy-bytes 268435456] [--json OUT] [--command "..."]

The traffic mode scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the
chosen kernel by what the same counters read for a plain device copy of
--copy-bytes bytes (the largest-grid __amd_rocclr_copyBuffer dispatch in the
same runs), so that the result is in true bytes moved to and from HBM.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def _code_only(text: str) -> str:
    """C++ source without its comments, whitespace runs collapsed: the part
    of a source that the compiler sees (string and character literals kept)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash(read=None) -> str:
    """Hash of the code (comments and layout left out) of the sources the
    fused step kernel is compiled from: counter summaries taken on other
    code are stale.  `read(name)` returns a source's text (default: the
    files under csrc/)."""
    if read is None:
        def read(name):
            with open(os.path.join(CSRC, name), encoding="utf-8") as fh:
                return fh.read()
    h = hashlib.sha256()
    for f in ("step.hip", "dev_common.hpp", "md_dev.hpp", "ds.hpp", "kernels.hpp"):
        h.update(_code_only(read(f)).encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


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


def _counters(d, where=None):
    """Mean inputs per (kernel, grid): counter -> list of per-dispatch values
    (a counter's rows of one dispatch are summed).  `where` = (counter,
    minimum) keeps only the dispatches whose value of that counter reaches
    the minimum (e.g. the launches of a kernel that did work)."""
    per = defaultdict(lambda: defaultdict(float))
    keys = {}
    for f in _find(d, "counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                did = (f, r.get("Dispatch_Id", ""))
                keys[did] = (r["Kernel_Name"], int(r.get("Grid_Size", 0) or 0))
                per[did][r["Counter_Name"]] += float(r["Counter_Value"])
    acc = defaultdict(lambda: defaultdict(list))
    for did, cs in per.items():
        if where and cs.get(where[0], float("-inf")) < where[1]:
            continue
        for c, v in cs.items():
            acc[keys[did]][c].append(v)
    return acc


def pmc(d, where=None):
    out = ["kernel | grid | counter | dispatches | mean per dispatch"]
    for (k, g), cs in sorted(_counters(d, where).items()):
        for c, v in sorted(cs.items()):
            out.append(f"{k} | {g} | {c} | {len(v)} | {sum(v) / len(v):.6g}")
    return "\n".join(out)


def _mean_of(acc, counter, pred):
    vals = []
    for (k, g), cs in acc.items():
        if pred(k, g) and counter in cs:
            vals += cs[counter]
    if not vals:
        raise SystemExit(f"no {counter} samples for the selected kernel")
    return sum(vals) / len(vals), len(vals)


def traffic(fetch_dir, write_dir, kernel_regex, copy_bytes):
    rx = re.compile(kernel_regex)
    fa, wa = _counters(fetch_dir), _counters(write_dir)

    def copy_pred(acc):
        grids = [g for (k, g) in acc if "copyBuffer" in k]
        if not grids:
            raise SystemExit("no copy-kernel dispatch to calibrate against")
        gmax = max(grids)
        return lambda k, g: "copyBuffer" in k and g == gmax

    cf, _ = _mean_of(fa, "FETCH_SIZE", copy_pred(fa))
    cw, _ = _mean_of(wa, "WRITE_SIZE", copy_pred(wa))
    fetch_scale = copy_bytes / (cf * 1024.0)
    write_scale = copy_bytes / (cw * 1024.0)
    # The fused kernel's launches that reuse stored forces (no force loop)
    # read a fifth of what a force launch reads; they are left out of the
    # read average (below half the median).  Both kinds write the same.
    fvals = [v for (k, g), cs in fa.items() if rx.search(k) for v in cs.get("FETCH_SIZE", [])]
    if not fvals:
        raise SystemExit("no FETCH_SIZE samples for the selected kernel")
    med = sorted(fvals)[len(fvals) // 2]
    full = [v for v in fvals if v >= 0.5 * med]
    kf, nf = sum(full) / len(full), len(full)
    kw, nw = _mean_of(wa, "WRITE_SIZE", lambda k, g: bool(rx.search(k)))
    fetched = kf * 1024.0 * fetch_scale
    written = kw * 1024.0 * write_scale
    return {"kernel_regex": kernel_regex, "kernel_hash": kernel_source_hash(),
            "dispatches": [nf, nw], "fetch_dispatches_without_force_loop": len(fvals) - nf,
            "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw,
            "copy_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
            "fetch_scale": fetch_scale, "write_scale": write_scale,
            "hbm_read_bytes_per_launch": fetched, "hbm_write_bytes_per_launch": written,
            "hbm_bytes_per_launch": fetched + written}


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["stats", "pmc", "traffic"])
    ap.add_argument("dirs", nargs="+")
    ap.add_argument("--kernel", default=r"k_step<")
    ap.add_argument("--copy-bytes", type=int, default=256 * 1024 * 1024)
    ap.add_argument("--json", default=None)
    ap.add_argument("--command", default="")
    ap.add_argument("--where", default=None, help="pmc: COUNTER>=VALUE keeps the dispatches that reach it")
    a = ap.parse_args()
    if a.mode == "stats":
        print(kernel_stats(a.dirs[0]))
    elif a.mode == "pmc":
        where = None
        if a.where:
            c, v = a.where.split(">=")
            where = (c.strip(), float(v))
        print(pmc(a.dirs[0], where))
    else:
        t = traffic(a.dirs[0], a.dirs[1], a.kernel, a.copy_bytes)
        t["command"] = a.command
        if a.json:
            with open(a.json, "w") as fh:
                json.dump(t, fh, indent=1)
        print(json.dumps(t, indent=1))
