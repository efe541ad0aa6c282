"""Host-side pieces of bench.py (no GPU): the oracle timing children of the
CPU-baseline leg run and report a rate."""
import json
import subprocess
import sys

import bench


def test_oracle_timing_child_reports_rates():
    for cfg, route, steps in [("lj4000", "cells", 3), ("lj4000", "brute", 1), ("ka64k", "sample", 16)]:
        r = subprocess.run([sys.executable, "-c", bench._CPU_CFG_CHILD, bench.ROOT, cfg, route, str(steps)],
                           capture_output=True, text=True, check=True)
        d = json.loads(r.stdout.strip().splitlines()[-1])
        assert d["n"] == (4000 if cfg == "lj4000" else 64000)
        assert d["rate"] > 0 and d["seconds"] > 0, d


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr
