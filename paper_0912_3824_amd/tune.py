"""Autotuner of libmdx launch shapes.

The knobs (md_launch: block size of the fused step kernel, cells per LDS row
segment, block size, lanes per member and segment split of the list build,
the rebuilding-replica count from which a build takes the bulk shape, steps
per captured hipGraph, XCD-aware tile mapping) change no result bit: lists are in a canonical order and
every particle sums its own list sequentially.  The tuner therefore times
candidate shapes on the live pool, from a saved checkpoint so that every
candidate advances the same trajectory, and keeps the fastest.  Results are
cached in a JSON file keyed by (precision, particle-count bucket, replicas).
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time
from typing import Dict, List, Optional

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")

SPACE = {
    "step_block": [256, 512, 1024],
    "build_width": [4, 8, 10],
    "build_block": [256, 320, 512],
    "build_lanes": [0, 16],
    "graph_steps": [32],
    "xcd_remap": [0, 1],
    "build_split": [0, 4],
}

# Pools with aligned rebuilds also try the bulk build (one lane per member
# and unsplit row segments in the steps where many replicas rebuild).
ALIGNED_SPACE = {"build_bulk": [0, 32]}


def bucket(n_total: int) -> int:
    return int(round(math.log2(max(n_total, 1)) * 2))


def key_of(pool) -> str:
    """Cache key: precision, particle-count bucket and replicas, plus the
    aligned-rebuild period when the pool sets one (aligned rebuilds make
    most replicas rebuild in the same steps, which favours other
    list-build shapes)."""
    n = sum(pool.sizes.values())
    k = f"p{pool.cfg.precision}_b{bucket(n)}_r{len(pool.sizes)}"
    every = int(getattr(pool.cfg, "rebuild_every", 0) or 0)
    return f"{k}_a{every}" if every > 0 else k


def space_for(pool) -> Dict[str, List[int]]:
    """The shapes tried for a pool: SPACE, and the bulk-build threshold too
    when the pool has aligned rebuilds."""
    aligned = int(getattr(pool.cfg, "rebuild_every", 0) or 0) > 0
    return dict(SPACE, **ALIGNED_SPACE) if aligned else dict(SPACE)


def _base_key(key: str) -> str:
    return key.split("_a")[0]


def _time_steps(pool, steps: int) -> float:
    import torch
    pool.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pool.step(steps)
    pool.sync()
    return (time.perf_counter() - t0) / steps


def tune(pool, steps: int = 200, space: Optional[Dict[str, List[int]]] = None,
         cache: Optional[str] = CACHE, verbose: bool = False) -> dict:
    """Time every shape in `space` on the live pool and apply the fastest.

    Each candidate starts from the same checkpoint of every attached slot, so
    the timed steps (including their list rebuilds) are identical work.
    """
    space = space or space_for(pool)
    slots = sorted(pool.sizes)
    blobs = {s: pool.save(s) for s in slots}
    sizes = dict(pool.sizes)
    boxes = dict(pool.boxes)

    def restore_all():
        for s in slots:
            pool.detach(s)
        for s in slots:
            pool.restore(s, blobs[s], sizes[s], boxes[s])

    results = []
    names = list(space)
    for combo in itertools.product(*(space[k] for k in names)):
        shape = dict(zip(names, combo))
        restore_all()
        pool.set_launch(**shape)
        pool.step(2)          # graph capture / warm caches
        restore_all()
        dt = _time_steps(pool, steps)
        results.append((dt, shape))
        if verbose:
            print(f"[tune] {shape} -> {dt * 1e6:.1f} us/step", flush=True)
    results.sort(key=lambda r: r[0])
    best = results[0][1]
    restore_all()
    pool.set_launch(**best)
    if cache:
        try:
            data = json.load(open(cache)) if os.path.exists(cache) else {}
        except (OSError, ValueError):
            data = {}
        data[key_of(pool)] = {"shape": best, "us_per_step": results[0][0] * 1e6}
        with open(cache, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
    return {"best": best, "us_per_step": results[0][0] * 1e6,
            "all": [(r[0] * 1e6, r[1]) for r in results]}


def apply_cached(pool, cache: str = CACHE) -> Optional[dict]:
    """Apply a cached shape for this pool's key (for a pool with aligned
    rebuilds, else the key without the period), if one exists."""
    if not os.path.exists(cache):
        return None
    try:
        data = json.load(open(cache))
    except (OSError, ValueError):
        return None
    key = key_of(pool)
    hit = data.get(key) or data.get(_base_key(key))  # an aligned pool falls back to the plain key
    if hit:
        pool.set_launch(**hit["shape"])
        return hit["shape"]
    return None
