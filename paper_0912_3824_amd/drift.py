"""Energy-drift measurement of a running replica (NVE, velocity Verlet).

The drift is the ordinary-least-squares slope of E_tot/N against the step
number, sampled every `every` steps, reported per 1e5 steps (in units of eps
per particle and relative to |E(0)/N|), with a standard error corrected for
the time correlation of the residuals by block averaging (statistical
inefficiency from 10 blocks).  Energy conservation over long runs is the
quantity Sec. 4.2 of the paper uses to compare single, double-single and
double precision.

  python -m paper_0912_3824_amd.drift --n 64000 --T 0.7 --steps 100000
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


def measure(pool, slot: int, steps: int, every: int = 100):
    """Advance the pool by `steps` in chunks of `every`, sampling E_tot/N."""
    n = pool.sizes[slot]
    o = pool.observables()[slot]
    t, e, p = [0], [o["etot"] / n], [np.abs(o["momentum"]).max() / n]
    done = 0
    while done < steps:
        k = min(every, steps - done)
        pool.step(k)
        done += k
        o = pool.observables()[slot]
        if o["status"]:
            raise RuntimeError(f"replica status {o['status']}")
        t.append(done)
        e.append(o["etot"] / n)
        p.append(np.abs(o["momentum"]).max() / n)
    t, e = np.array(t), np.array(e)
    b, se, g = slope_with_error(t, e)
    e0 = abs(e[0])
    return {
        "steps": steps, "every": every, "e0_per_particle": float(e[0]),
        "slope_per_1e5_steps": b * 1e5, "stderr_per_1e5_steps": se * 1e5,
        "relative_slope_per_1e5_steps": b * 1e5 / e0, "relative_stderr": se * 1e5 / e0,
        "rms_dev_from_e0": float(np.sqrt(np.mean((e - e[0]) ** 2))),
        "statistical_inefficiency": g,
        "max_abs_momentum_per_particle": float(max(p)),
    }


def run(n: int = 64000, temperature: float = 0.7, steps: int = 100000, every: int = 100,
        equil: int = 2000, precisions=("fp32", "ds", "mixed64", "fp64"), seed: int = 20240101,
        log=None) -> dict:
    """Equilibrate one KA replica with velocity rescaling in FP64, then run
    the same state for `steps` NVE steps in every precision."""
    sys.path.insert(0, __file__.rsplit("/", 2)[0])
    import md_inputs as I
    from paper_0912_3824_amd import mdx
    s = I.make_ka(n, temperature, seed=seed)
    pool = mdx.md_init([s], "fp64")
    done = 0
    while done < equil:
        pool.step(100)
        done += 100
        o = pool.observables()[0]
        pool.scale_velocities(0, math.sqrt(temperature / o["temperature"]))
    pos, vel, img = pool.get_state(0)
    pool.close()
    out = {"n": n, "temperature": temperature, "equil_steps": equil, "results": {}}
    for prec in precisions:
        p = mdx.md_init([I.System(n, s.box, pos, vel, s.species, s.table, temperature)], prec)
        t0 = time.perf_counter()
        r = measure(p, 0, steps, every)
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
    a = ap.parse_args()
    res = run(a.n, a.T, a.steps, a.every, a.equil, tuple(a.precisions.split(",")),
              log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(res))
