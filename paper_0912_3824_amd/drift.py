"""Energy-drift measurement of running replicas (NVE, velocity Verlet).

The drift of a replica is the ordinary-least-squares slope of E_tot/N
against the step number, sampled every `every` steps, reported per 1e5 steps
(in units of eps per particle and relative to |E(0)/N|), with a standard
error corrected for the time correlation of the residuals by block averaging
(statistical inefficiency from 10 blocks).  With the plain truncated-and-
shifted cutoff, the force jumps when a pair crosses rc, and the energy of one
trajectory wanders by more than that error suggests; so the drift of a
precision mode is measured on an ensemble of independent replicas (advanced
together in one pool), and its standard error is the spread of their slopes
over the square root of their number.  Energy conservation over long runs is
the quantity Sec. 4.2 of the paper uses to compare single, double-single and
double precision.

  python -m paper_0912_3824_amd.drift --n 64000 --T 0.7 --steps 100000 --replicas 8
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def slope_with_error(t: np.ndarray, e: np.ndarray, n_blocks: int = 10):
    """OLS slope of e(t) and its standard error, inflated by the statistical
    inefficiency of the residuals measured with n_blocks blocks."""
    t = np.asarray(t, dtype=float)
    e = np.asarray(e, dtype=float)
    n = len(t)
    tm = t.mean()
    sxx = float(np.sum((t - tm) ** 2))
    b = float(np.sum((t - tm) * (e - e.mean())) / sxx)
    a = e.mean() - b * tm
    res = e - (a + b * t)
    var = float(np.sum(res ** 2) / max(n - 2, 1))
    se_white = math.sqrt(var / sxx) if sxx > 0 else float("nan")
    m = n // n_blocks
    g = 1.0
    if m >= 2 and var > 0:
        means = res[: m * n_blocks].reshape(n_blocks, m).mean(axis=1)
        g = max(1.0, m * float(np.var(means, ddof=1)) / var)
    return b, se_white * math.sqrt(g), g


def measure(pool, steps: int, every: int = 100):
    """Advance the pool by `steps` in chunks of `every`, sampling E_tot/N of
    every attached replica; one drift record per replica."""
    slots = sorted(k for k, n in pool.sizes.items() if n)
    obs = pool.observables()
    t = [0]
    e = {k: [obs[k]["etot"] / pool.sizes[k]] for k in slots}
    p = {k: [np.abs(obs[k]["momentum"]).max() / pool.sizes[k]] for k in slots}
    done = 0
    while done < steps:
        k = min(every, steps - done)
        pool.step(k)
        done += k
        obs = pool.observables()
        t.append(done)
        for s in slots:
            if obs[s]["status"]:
                raise RuntimeError(f"replica {s} status {obs[s]['status']}")
            e[s].append(obs[s]["etot"] / pool.sizes[s])
            p[s].append(np.abs(obs[s]["momentum"]).max() / pool.sizes[s])
    t = np.array(t)
    out = []
    for s in slots:
        es = np.array(e[s])
        b, se, g = slope_with_error(t, es)
        e0 = abs(es[0])
        out.append({
            "steps": steps, "every": every, "e0_per_particle": float(es[0]),
            "slope_per_1e5_steps": b * 1e5, "stderr_per_1e5_steps": se * 1e5,
            "relative_slope_per_1e5_steps": b * 1e5 / e0, "relative_stderr": se * 1e5 / e0,
            "rms_dev_from_e0": float(np.sqrt(np.mean((es - es[0]) ** 2))),
            "statistical_inefficiency": g,
            "max_abs_momentum_per_particle": float(max(p[s])),
        })
    return out


def ensemble(records) -> dict:
    """Mean drift of the replicas and its standard error from their spread
    (for a single replica, its own block-averaged error)."""
    sl = np.array([r["slope_per_1e5_steps"] for r in records])
    rel = np.array([r["relative_slope_per_1e5_steps"] for r in records])
    k = len(sl)
    se = float(sl.std(ddof=1) / math.sqrt(k)) if k > 1 else records[0]["stderr_per_1e5_steps"]
    rse = float(rel.std(ddof=1) / math.sqrt(k)) if k > 1 else records[0]["relative_stderr"]
    return {
        "replicas": k,
        "slope_per_1e5_steps": float(sl.mean()), "stderr_per_1e5_steps": se,
        "relative_slope_per_1e5_steps": float(rel.mean()), "relative_stderr": rse,
        "replica_slopes_per_1e5_steps": [float(x) for x in sl],
        "mean_block_stderr_per_1e5_steps": float(np.mean([r["stderr_per_1e5_steps"] for r in records])),
        "rms_dev_from_e0": float(np.mean([r["rms_dev_from_e0"] for r in records])),
        "max_abs_momentum_per_particle": float(max(r["max_abs_momentum_per_particle"] for r in records)),
    }


def run(n: int = 64000, temperature: float = 0.7, steps: int = 100000, every: int = 100,
        equil: int = 2000, precisions=("fp32", "ds", "mixed64", "fp64"), seed: int = 20240101,
        replicas: int = 1, log=None) -> dict:
    """Equilibrate `replicas` independent KA replicas (seeds seed, seed + 1,
    ...) with velocity rescaling in FP64, then run the same states for
    `steps` NVE steps in every precision, all replicas in one pool."""
    sys.path.insert(0, __file__.rsplit("/", 2)[0])
    import md_inputs as I
    from paper_0912_3824_amd import mdx
    systems = [I.make_ka(n, temperature, seed=seed + r) for r in range(replicas)]
    pool = mdx.md_init(systems, "fp64")
    done = 0
    while done < equil:
        pool.step(100)
        done += 100
        obs = pool.observables()
        for r in range(replicas):
            pool.scale_velocities(r, math.sqrt(temperature / obs[r]["temperature"]))
    states = [pool.get_state(r) for r in range(replicas)]
    pool.close()
    out = {"n": n, "temperature": temperature, "equil_steps": equil, "replicas": replicas, "results": {}}
    for prec in precisions:
        p = mdx.md_init([I.System(n, s.box, pos, vel, s.species, s.table, temperature)
                         for s, (pos, vel, img) in zip(systems, states)], prec)
        t0 = time.perf_counter()
        recs = measure(p, steps, every)
        r = ensemble(recs)
        r["wall_s"] = time.perf_counter() - t0
        out["results"][prec] = r
        if log:
            log(f"{prec}: {json.dumps(r)}")
        p.close()
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64000)
    ap.add_argument("--T", type=float, default=0.7)
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--equil", type=int, default=2000)
    ap.add_argument("--precisions", default="fp32,ds,mixed64,fp64")
    ap.add_argument("--replicas", type=int, default=8)
    a = ap.parse_args()
    res = run(a.n, a.T, a.steps, a.every, a.equil, tuple(a.precisions.split(",")),
              replicas=a.replicas, log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(res))
