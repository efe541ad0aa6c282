"""Measurements of the batching and serving patterns against plain
single-system runs of the same replicas (equal arithmetic, bitwise-equal
results).

  python -m paper_0912_3824_amd.patterns_bench batch [--replicas 256 --steps 2000]
  python -m paper_0912_3824_amd.patterns_bench serve [--jobs 40 --load 0.8]
  python -m paper_0912_3824_amd.patterns_bench tcf   [--steps 3000]
  python -m paper_0912_3824_amd.patterns_bench thermo [--steps 3000]

batch: 256 Kob-Andersen replicas, N log-uniform in [500, 8000], rho = 1.2,
       T from {0.45, 0.5, 0.6, 0.8}, advanced together in one pool (one
       fused launch per step for all replicas, graph-captured); compared with
       a sample of the same replicas advanced one at a time.
tcf:   the N = 1M KA run with on-device time-correlation functions
       (blocking scheme, Sec. 2.5) sampled every 10 steps, against the same
       run without them.
thermo: the N = 1M KA run in the heat bath of the modified Andersen
       thermostat (Sec. 2.3): the cost of one thermostat call, and the same
       run with a call every (mu dt)^-1 steps against the run without.
serve: Poisson arrivals of KA jobs, N log-uniform in [1000, 256000], steps
       uniform in [steps_lo, steps_hi], T uniform in [0.45, 1.0]; admission
       by arena footprint; p50/p99 latency and throughput over the busy
       period, against the same jobs run one after another alone.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# Rebuild policy of the 256-replica ensemble measurement (md_config
# rebuild_every and rebuild_early, and the Verlet skin): a replica also
# rebuilds at multiples of 12 steps once past half of skin/2.  Chosen by
# measurement over K in 4..32, fractions 0.4..0.8 and skins 0.35..0.5.
BATCH_POLICY = dict(rebuild_every=12, rebuild_early=0.5, skin=0.4)
sys.path.insert(0, ROOT)


def log(*a):
    print("[patterns]", *a, file=sys.stderr, flush=True)


def _timed_step(pool, steps):
    import torch
    pool.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pool.step(steps)
    pool.sync()
    return time.perf_counter() - t0


def batch(n_rep=256, steps=2000, warmup=200, alone_sample=16, precision="ds", seed=20240101,
          rebuild_every=0, rebuild_early=0.0, skin=None, shape=None):
    import md_inputs as I
    from paper_0912_3824_amd import mdx, tune
    reps = I.make_ka_ensemble(n_rep, seed=seed)
    total = sum(r.n for r in reps)
    kw = dict(rebuild_every=rebuild_every, rebuild_early=rebuild_early, skin=skin)
    pool = mdx.md_init(reps, precision, **kw)
    tune.apply_cached(pool)
    if shape:
        pool.set_launch(**shape)
    pool.step(warmup)
    t = _timed_step(pool, steps)
    obs = pool.observables()
    assert not any(o["status"] for o in obs if o["n"])
    prof = pool.profile_steps(100)
    pool_shape = pool.get_launch()
    pool.close()
    batched = total * steps / t
    log(f"batch: {n_rep} replicas, {total} particles, {t / steps * 1e6:.1f} us/step, {batched:.4g} p-s/s")
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(n_rep, size=min(alone_sample, n_rep), replace=False)) if alone_sample > 0 else []
    work, wall = 0, 0.0
    for k in idx:
        p = mdx.md_init([reps[k]], precision, **kw)
        p.step(warmup)
        dt = _timed_step(p, steps)
        work += reps[k].n * steps
        wall += dt
        p.close()
    alone = work / wall if wall > 0 else None
    if alone:
        log(f"alone (sample of {len(idx)}): {alone:.4g} p-s/s")
    return {"replicas": n_rep, "particles": total, "steps": steps, "precision": precision,
            "rebuild_every": rebuild_every, "rebuild_early": rebuild_early, "skin": skin,
            "shape": pool_shape,
            "batched_particle_steps_per_s": batched, "batched_us_per_step": t / steps * 1e6,
            "alone_particle_steps_per_s": alone, "alone_sample": int(len(idx)),
            "speedup_vs_alone": batched / alone if alone else None, "step_kernel_ms": prof["step_kernel_ms"],
            "rebuild_group_ms_mean": prof["rebuild_ms_mean"]}


def serve(n_jobs=40, load=0.8, steps_lo=1000, steps_hi=10000, n_lo=1000, n_hi=256000,
          max_slots=32, hbm_budget_gb=4.0, chunk=256, precision="ds", seed=20240101,
          rebuild_every=0, rebuild_early=0.0, skin=0.3, shape=None, tcf_fraction=0.0):
    import md_inputs as I
    from paper_0912_3824_amd import mdx
    from paper_0912_3824_amd.serve import Server
    # capacity estimate: the throughput of a mid-size replica alone
    probe = I.make_ka(64000, 0.7, seed=seed)
    p = mdx.md_init([probe], precision)
    p.step(100)
    cap = probe.n * 1000 / _timed_step(p, 1000)
    p.close()
    mean_job = math.exp((math.log(n_hi) + math.log(n_lo)) / 2) * 1.15 * (steps_lo + steps_hi) / 2
    rate = load * cap / mean_job
    jobs = I.serving_trace(n_jobs, rate, n_lo=n_lo, n_hi=n_hi, steps_lo=steps_lo,
                           steps_hi=steps_hi, seed=seed, tcf_fraction=tcf_fraction)
    max_particles = Server.bytes_for_budget(I.ka_table(), precision, hbm_budget_gb * 1e9, max_slots)
    log(f"serve: {n_jobs} jobs at {rate:.2f}/s (offered load {load}), arena {max_particles} particles")
    kw = dict(rebuild_every=rebuild_every, rebuild_early=rebuild_early)
    srv = Server(I.ka_table(), precision, max_slots=max_slots, max_particles=max_particles, skin=skin,
                 chunk_steps=chunk, make_system=lambda j: I.job_system(j, skin=skin), shape=shape, **kw)
    out = srv.run(jobs)
    srv.close()
    # the same jobs, one after another, each alone
    work, wall = 0, 0.0
    for j in jobs:
        s = I.job_system(j, skin=skin)
        q = mdx.md_init([s], precision, **kw)
        wall += _timed_step(q, j.steps)
        work += s.n * j.steps
        q.close()
    res = {k: v for k, v in out.items() if k != "results"}
    res.update({"jobs": n_jobs, "rate_per_s": rate, "offered_load": load, "max_slots": max_slots,
                "rebuild_every": rebuild_every, "rebuild_early": rebuild_early, "skin": skin,
                "tcf_jobs": sum(1 for j in jobs if j.tcf_every),
                "arena_particles": max_particles, "chunk_steps": chunk, "precision": precision,
                "alone_sequential_particle_steps_per_s": work / wall,
                "served_vs_alone": res["throughput_busy"] / (work / wall),
                "latencies_s": [round(r.latency, 4) for r in out["results"]]})
    log(json.dumps({k: v for k, v in res.items() if k != "latencies_s"}))
    return res


def tcf(n=1_000_000, steps=3000, every=10, levels=4, block=10, precision="ds", seed=20240101):
    """Cost of on-device time-correlation functions (blocking scheme) at the
    N = 1M KA workload: the same run with and without a sample every `every`
    steps, and the MSD / F_s / VACF the scheme produces."""
    import torch
    import md_inputs as I
    from paper_0912_3824_amd import mdx
    s = I.make_ka(n, 0.5, seed=seed)
    pool = mdx.md_init([s], precision)
    for _ in range(10):
        pool.step(100)
        o = pool.observables()[0]
        pool.scale_velocities(0, math.sqrt(0.5 / o["temperature"]))
    blob = pool.save(0)

    def chunks(sample):  # the same launch pattern with and without sampling
        pool.step(200)
        pool.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            if sample:
                sample()
            pool.step(every)
            done += every
        pool.sync()
        return time.perf_counter() - t0

    base = chunks(None)
    pool.detach(0)
    pool.restore(0, blob, s.n, s.box)
    q = 2 * math.pi * round(7.25 * s.box / (2 * math.pi)) / s.box
    t = pool.tcf(0, levels, block, q)
    with_tcf = chunks(t.sample)
    lags, vals, terms = t.read()
    pool.close()
    dt_s = every * s.dt
    curve = [{"t": float(lags[a, j] * dt_s), "terms": int(terms[a, j]),
              "msd_A": vals[a, j, 0, 0], "fs_A": vals[a, j, 0, 2], "vacf_A": vals[a, j, 0, 1]}
             for a in range(levels) for j in range(block - 1) if terms[a, j]]
    res = {"particles": n, "steps": steps, "sample_every": every, "levels": levels, "block": block,
           "q": q, "us_per_step_plain": base / steps * 1e6, "us_per_step_with_tcf": with_tcf / steps * 1e6,
           "overhead": with_tcf / base - 1.0, "curve": curve}
    log(json.dumps({k: v for k, v in res.items() if k != "curve"}))
    return res


def thermo(n=1_000_000, steps=3000, calls=100, mu=1.0, precision="ds", seed=20240101):
    """Cost of the modified Andersen thermostat at the N = 1M KA workload:
    `calls` back-to-back calls, and `steps` steps with and without the bath
    (a call every (mu dt)^-1 steps)."""
    import torch
    import md_inputs as I
    from paper_0912_3824_amd import mdx
    s = I.make_ka(n, 0.5, seed=seed)
    pool = mdx.md_init([s], precision)
    pool.step(200)
    for c in range(5):  # warm-up
        pool.thermostat(0, 0.5, seed, c)
    pool.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(calls):
        pool.thermostat(0, 0.5, seed, 5 + c)
    pool.sync()
    per_call = (time.perf_counter() - t0) / calls
    base = _timed_step(pool, steps)
    pool.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pool.andersen(0, 0.5, mu=mu, steps=steps, seed=seed, first_call=1000)
    pool.sync()
    bath = time.perf_counter() - t0
    o = pool.observables()[0]
    pool.close()
    res = {"particles": n, "precision": precision, "us_per_call": per_call * 1e6,
           "every": int(round(1.0 / (mu * s.dt))), "steps": steps,
           "us_per_step_plain": base / steps * 1e6, "us_per_step_bath": bath / steps * 1e6,
           "overhead": bath / base - 1.0, "temperature_after": o["temperature"]}
    log(json.dumps(res))
    return res


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["batch", "serve", "tcf", "thermo"])
    ap.add_argument("--replicas", type=int, default=256)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--jobs", type=int, default=40)
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--steps-lo", type=int, default=1000)
    ap.add_argument("--steps-hi", type=int, default=10000)
    ap.add_argument("--precision", default="ds")
    ap.add_argument("--rebuild-every", type=int, default=0, help="aligned list rebuilds (md_config)")
    ap.add_argument("--rebuild-early", type=float, default=0.0)
    ap.add_argument("--skin", type=float, default=None)
    ap.add_argument("--alone-sample", type=int, default=16)
    ap.add_argument("--shape", default=None, help="launch shape as JSON (md_launch fields)")
    ap.add_argument("--tcf-fraction", type=float, default=0.0, help="serve: jobs asking for correlations")
    a = ap.parse_args()
    if a.mode == "batch":
        r = batch(a.replicas, a.steps, precision=a.precision, rebuild_every=a.rebuild_every,
                  rebuild_early=a.rebuild_early, skin=a.skin, alone_sample=a.alone_sample,
                  shape=json.loads(a.shape) if a.shape else None)
    elif a.mode == "tcf":
        r = tcf(steps=a.steps, precision=a.precision)
    elif a.mode == "thermo":
        r = thermo(steps=a.steps, precision=a.precision)
    else:
        r = serve(a.jobs, a.load, a.steps_lo, a.steps_hi, precision=a.precision,
                  rebuild_every=a.rebuild_every, rebuild_early=a.rebuild_early,
                  skin=a.skin if a.skin is not None else 0.3,
                  shape=json.loads(a.shape) if a.shape else None, tcf_fraction=a.tcf_fraction)
    print(json.dumps(r))
