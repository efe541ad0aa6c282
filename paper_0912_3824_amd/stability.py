"""Numerical long-time stability of the MD step (Sec. 4 of the paper) on the
GPU path: LJ and WCA fluids with and without the C2 smoothing factor
g(x) = x^4 / (1 + x^4), in single, double-single and double precision.

  collapse: q(t) = [E(t) - E(0)] / dt^2 over steps 200..1000 for dt = 0.001
            .. 0.005 (Sec. 4.3).  Velocity Verlet's energy error is second
            order only for a potential with a continuous second derivative,
            so the curves for different dt share one band ("collapse") when
            the arithmetic is precise enough and the potential is smooth.
            Curves at the same step index are at different physical times
            (k dt), so from an equilibrium start they agree in amplitude, not
            point by point.  Reported per dt: the rms and the mean of q over
            the window; and their collapse measure, the ratio of the largest
            to the smallest rms.
  drift:    OLS slope of E_tot/N per 1e5 steps (Sec. 4.2) and the largest
            centre-of-mass speed |sum v|/N reached (Sec. 4.1).
  long:     (with --long-steps) the drift of the smoothed potentials (h =
            0.005, dt = 0.001) over a longer run, where a slope well below
            the short runs' fluctuation level can be resolved.
  speed:    particle-steps/s of WCA against LJ (Sec. 4: shorter lists).

All runs of one potential start from the same state, prepared as Sec. 4
describes: an fcc lattice equilibrated in the heat bath of the modified
Andersen thermostat (Sec. 2.3, collision rate mu = 1) with dt = 0.001 and
h = 0.005 over 1e5 steps in double-single precision.  System: N = 10,000,
rho = 0.75, T = 1.12.

  python -m paper_0912_3824_amd.stability [--steps 200000] [--n 10000] [--long-steps 2000000]
      [--only-long --potentials lj --precisions ds,fp64]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def log(*a):
    print("[stability]", *a, file=sys.stderr, flush=True)


def equilibrated(n: int, rc: float, rho: float, temperature: float, steps: int, seed: int):
    """Lattice start equilibrated in the Andersen heat bath (mu = 1, dt = 0.001,
    h = 0.005, double-single), as in Sec. 4."""
    import md_inputs as I
    from paper_0912_3824_amd import mdx
    s = I.smoothed(I.make_lj(n, rho=rho, temperature=temperature, seed=seed, jitter=0.05, rc=rc), 0.005)
    s = dataclasses.replace(s, dt=0.001)
    pool = mdx.md_init([s], "ds")
    pool.andersen(0, temperature, mu=1.0, steps=steps, seed=seed)
    pos, vel, _ = pool.get_state(0)
    pool.close()
    return dataclasses.replace(s, pos=pos, vel=vel)


def _energy_series(s, prec: str, h: float, dt: float, steps: int, every: int):
    import md_inputs as I
    from paper_0912_3824_amd import mdx
    r = dataclasses.replace(I.smoothed(s, h), dt=dt)
    pool = mdx.md_init([r], prec)
    o = pool.observables()[0]
    t, e, p = [0], [o["etot"] / r.n], [float(np.abs(o["momentum"]).max()) / r.n]
    done = 0
    tick = max(steps // 10, 1)
    while done < steps:
        k = min(every, steps - done)
        pool.step(k)
        done += k
        o = pool.observables()[0]
        if o["status"]:
            raise RuntimeError(f"replica status {o['status']}")
        if steps >= 10 ** 6 and done % tick < k:
            log(f"  {prec} h={h} dt={dt}: {done} of {steps} steps, E/N {o['etot'] / r.n:.9f}")
        t.append(done)
        e.append(o["etot"] / r.n)
        p.append(float(np.abs(o["momentum"]).max()) / r.n)
    pool.close()
    return np.array(t), np.array(e), np.array(p)


def collapse(s, precs, hs, dts=(0.001, 0.002, 0.003, 0.004, 0.005), steps=1000, every=10,
             window=(200, 1000)) -> dict:
    out = {}
    for prec in precs:
        for h in hs:
            qs = []
            for dt in dts:
                t, e, _ = _energy_series(s, prec, h, dt, steps, every)
                qs.append((e - e[0]) / dt ** 2)
            q = np.array(qs)
            sel = (t >= window[0]) & (t <= window[1])
            qw = q[:, sel]
            rms = [float(np.sqrt(np.mean(x ** 2))) for x in qw]
            key = f"{prec}_h{h}"
            out[key] = {"dt": list(dts), "q_rms_per_dt": rms, "q_mean_per_dt": [float(x.mean()) for x in qw],
                        "rms_ratio": max(rms) / min(rms)}
            log(f"collapse {key}: rms per dt {[round(x, 3) for x in rms]}, ratio {max(rms) / min(rms):.3g}")
    return out


def drift(s, precs, hs, dts, steps, every) -> dict:
    from paper_0912_3824_amd.drift import slope_with_error
    out = {}
    for prec in precs:
        for h in hs:
            for dt in dts:
                t0 = time.perf_counter()
                t, e, p = _energy_series(s, prec, h, dt, steps, every)
                b, se, g = slope_with_error(t, e)
                key = f"{prec}_h{h}_dt{dt}"
                out[key] = {"slope_per_1e5_steps": b * 1e5, "stderr_per_1e5_steps": se * 1e5,
                            "relative_slope_per_1e5_steps": b * 1e5 / abs(e[0]),
                            "rms_dev_from_e0": float(np.sqrt(np.mean((e - e[0]) ** 2))),
                            "max_cm_speed_per_particle": float(p.max()),
                            "wall_s": time.perf_counter() - t0}
                log(f"drift {key}: {json.dumps(out[key])}")
    return out


def speed(s, prec="ds", steps=2000) -> dict:
    import torch
    from paper_0912_3824_amd import mdx
    pool = mdx.md_init([s], prec)
    pool.step(200)
    pool.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pool.step(steps)
    pool.sync()
    dt = time.perf_counter() - t0
    o = pool.observables()[0]
    pool.close()
    return {"particle_steps_per_s": s.n * steps / dt, "us_per_step": dt / steps * 1e6,
            "mean_list_entries": o["list_entries"] / s.n}


def run(n=10000, rho=0.75, temperature=1.12, equil=100000, drift_steps=200000, long_steps=0,
        seed=20240101, only_long=False, potentials=("lj", "wca"), precisions=("fp32", "ds", "fp64")) -> dict:
    import md_inputs as I
    res = {"n": n, "rho": rho, "temperature": temperature, "equil_steps": equil}
    states = {}
    for name, rc in (("lj", 2.5), ("wca", I.WCA_RC)):
        if name not in potentials:
            continue
        t0 = time.perf_counter()
        states[name] = equilibrated(n, rc, rho, temperature, equil, seed)
        log(f"equilibrated {name} in {time.perf_counter() - t0:.1f} s")
    if not only_long:
        res["collapse_lj"] = collapse(states["lj"], precisions, (0.0, 0.01))
        res["drift"] = {}
        for name in states:
            res["drift"][name] = drift(states[name], precisions, (0.0, 0.005), (0.001, 0.003),
                                       drift_steps, max(100, drift_steps // 500))
    if long_steps:
        res["drift_long"] = {name: drift(states[name], precisions, (0.005,), (0.001,),
                                         long_steps, max(100, long_steps // 1000))
                             for name in states}
    if not only_long:
        res["speed"] = {name: speed(states[name]) for name in states}
        log(f"speed {json.dumps(res['speed'])}")
    return res


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--equil", type=int, default=100000)
    ap.add_argument("--steps", type=int, default=200000, help="steps per drift run")
    ap.add_argument("--long-steps", type=int, default=0, help="steps per long drift run (0: none)")
    ap.add_argument("--only-long", action="store_true", help="run only the long drift runs")
    ap.add_argument("--potentials", default="lj,wca")
    ap.add_argument("--precisions", default="fp32,ds,fp64")
    a = ap.parse_args()
    print(json.dumps(run(n=a.n, equil=a.equil, drift_steps=a.steps, long_steps=a.long_steps,
                         only_long=a.only_long, potentials=tuple(a.potentials.split(",")),
                         precisions=tuple(a.precisions.split(",")))))
