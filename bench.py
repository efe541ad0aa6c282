#!/usr/bin/env python3
"""Benchmark of the MD hot path on one MI355X: particle-steps/s of the
Kob-Andersen mixture (N = 1,000,000, rho = 1.2, T = 0.5, dt = 0.001,
double-single integration) through the libmdx C ABI.

One "step" is one pass of the whole hot path over the system: the fused
force + velocity-Verlet kernel and the rebuild kernels (cell sort + Verlet
lists, which do work only when the maximum displacement exceeds skin/2).

Prints ONE JSON line on stdout; diagnostics go to stderr.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ka1m]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X vendor peaks
HBM_PEAK_GBS = 8000.0
# VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64 VALU
# instruction occupies a SIMD for 4 cycles); packed-FP32 dual issue is not used.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic work of one fused step per particle with L list entries.
# Bytes: list count 4 + list 4L + own snapshot + state read/write + new
# snapshot + reference position + cell-count atomic (neighbour snapshots are
# re-reads of data counted once).  VALU lane-ops: per list entry (separation,
# r^2, species select, pair term with a quarter-rate reciprocal counted as 4,
# cutoff mask, accumulation) and per particle (two kicks, drift, snapshot,
# displacement test).
ALGO = {
    "fp32": {"bytes": (4, 120), "ops_entry": 31, "ops_particle": 45},
    "ds": {"bytes": (4, 152), "ops_entry": 52, "ops_particle": 180},
    "mixed64": {"bytes": (4, 152), "ops_entry": 35, "ops_particle": 50},
    "fp64": {"bytes": (4, 200), "ops_entry": 48, "ops_particle": 50},
}

WORKLOADS = {
    "ka1m": ("Kob-Andersen 80/20, N=1,000,000, rho=1.2, T=0.5, dt=0.001, skin=0.3", "ds"),
    "ka64k": ("Kob-Andersen 80/20, N=64,000, rho=1.2, T=0.7, dt=0.001, skin=0.3", "ds"),
    "lj4000": ("LJ fcc start, N=4000, rho=0.8442, T=1.5, rc=2.5, skin=0.3, dt=0.001", "fp64"),
    "batch256": ("256 KA replicas, N log-uniform [500,8000], rho=1.2, T in {0.45,0.5,0.6,0.8}", "ds"),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def read_traffic(workload: str, prec: str, n_particles: int, cell_order: str = "row"):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source and in the
    same cell order."""
    tag = "" if cell_order == "row" else f"_{cell_order}"
    path = os.path.join(ROOT, "profiles", f"k_step_{prec}_{workload}{tag}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    from paper_0912_3824_amd.profiling import kernel_source_hash
    if d.get("kernel_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def build_systems(workload: str, seed: int):
    import md_inputs as I
    if workload == "ka1m":
        return [I.make_ka(1_000_000, 0.5, seed=seed)]
    if workload == "ka64k":
        return [I.make_ka(64_000, 0.7, seed=seed)]
    if workload == "lj4000":
        return [I.make_lj(4000, seed=seed)]
    if workload == "batch256":
        return I.make_ka_ensemble(256, seed=seed)
    raise SystemExit(f"unknown workload {workload}")


def equilibrate(pool, systems, steps: int, every: int = 100):
    """Velocity rescaling to each replica's target T every `every` steps."""
    done = 0
    while done < steps:
        k = min(every, steps - done)
        pool.step(k)
        done += k
        obs = pool.observables()
        for slot, s in enumerate(systems):
            t = obs[slot]["temperature"]
            if t > 0:
                pool.scale_velocities(slot, math.sqrt(s.temperature / t))


def cpu_baseline(system, budget_s: float = 15.0):
    """The FP64 oracle (brute force) timed on a bounded sample of the same
    workload: forces on m randomly chosen particles of the system, m grown
    until one timed call takes about budget_s (bounded to ~2 budgets of CPU
    time in total)."""
    import numpy as np
    from oracle import oracle as O
    O.build(force=False)
    rng = np.random.default_rng(1)
    cores = len(os.sched_getaffinity(0))
    n = system.n
    m = min(n, 256 if n > 100000 else 2048)
    spent = 0.0
    while True:
        sel = rng.choice(n, size=m, replace=False).astype(np.int32)
        t0 = time.perf_counter()
        O.forces(system.pos, system.box, system.species, system.table, sel)
        dt = time.perf_counter() - t0
        spent += dt
        if m >= n or dt >= 0.6 * budget_s or spent + 2 * dt > 2 * budget_s:
            break
        m = int(min(n, m * min(8.0, max(1.5, budget_s / max(dt, 1e-3)))))
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    return {"value": m / dt, "unit": "particle-steps/s", "cores": min(threads, cores),
            "kind": "oracle",
            "sample": f"brute-force FP64 forces (one step's force work) on {m} randomly chosen "
                      f"particles of the N={n} system, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--equil", type=int, default=1000, help="rescaled equilibration steps before warmup")
    ap.add_argument("--workload", default="ka1m", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp32", "ds", "mixed64", "fp64"])
    ap.add_argument("--profile-steps", type=int, default=300)
    ap.add_argument("--graph-steps", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=20240101)
    ap.add_argument("--skin", type=float, default=None, help="Verlet skin (default: the workload's)")
    ap.add_argument("--cell-order", default="row", choices=["row", "morton", "hilbert"],
                    help="order of the cells in the particle sort")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding of this "
              "path is a design note, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0912_3824_amd import mdx

    desc, default_prec = WORKLOADS[args.workload]
    if args.skin is not None:
        desc = desc.replace("skin=0.3", f"skin={args.skin:g}")
    prec = args.precision or default_prec
    systems = build_systems(args.workload, args.seed)
    n_total = sum(s.n for s in systems)
    log(f"workload {args.workload}: {len(systems)} replica(s), {n_total} particles, precision {prec}")

    pool = mdx.md_init(systems, prec, skin=args.skin, cell_order=args.cell_order)
    from paper_0912_3824_amd import tune
    tuned = tune.apply_cached(pool)  # launch shapes from the autotuner, if tuned
    pool.set_launch(graph_steps=args.graph_steps)
    log(f"launch shapes: {pool.get_launch()} ({'autotuned' if tuned else 'defaults'})")
    if args.equil > 0:
        equilibrate(pool, systems, args.equil)
    pool.step(args.warmup)
    pool.sync()
    obs0 = pool.observables()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pool.step(args.steps)
    pool.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    obs1 = pool.observables()
    status = [o["status"] for o in obs1 if o["n"]]
    if any(status):
        raise SystemExit(f"replica status bits set: {status}")
    rebuilds = sum(o1["n_rebuilds"] - o0["n_rebuilds"] for o0, o1 in zip(obs0, obs1))
    entries = sum(o["list_entries"] for o in obs1)
    mean_list = entries / n_total
    value = n_total * args.steps / wall
    ms_per_step = 1e3 * wall / args.steps
    log(f"timed {args.steps} steps: {wall:.4f} s, {ms_per_step * 1e3:.1f} us/step, "
        f"{value:.4g} particle-steps/s, {rebuilds} rebuild(s) (max over replicas per step), "
        f"mean list {mean_list:.2f}")

    # per-kernel timing with hipEvents on the pool's stream (eager launches)
    prof = pool.profile_steps(args.profile_steps)
    log(f"profile: {prof}")
    # force-only kernel (md_forces: force, energy, virial; no integration)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    pool.forces(0, copy=False)
    ev0.record(pool.stream)
    for _ in range(reps):
        pool.forces(0, copy=False)
    ev1.record(pool.stream)
    ev1.synchronize()
    force_ms = ev0.elapsed_time(ev1) / reps

    a = ALGO[prec]
    k_ms = prof["step_kernel_ms"]
    bytes_launch = n_total * (a["bytes"][0] * mean_list + a["bytes"][1])
    ops_launch = n_total * (a["ops_entry"] * mean_list + a["ops_particle"])
    hbm_gbs = bytes_launch / (k_ms * 1e-3) / 1e9
    alu_tops = ops_launch / (k_ms * 1e-3) / 1e12
    t_hbm = bytes_launch / (HBM_PEAK_GBS * 1e9)
    t_alu = ops_launch / (VALU_PEAK_TOPS * 1e12)
    if t_alu >= t_hbm:
        roof = {"bound": "alu", "achieved": round(alu_tops, 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "TOP/s (VALU lane-ops)", "frac": round(alu_tops / VALU_PEAK_TOPS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(hbm_gbs / HBM_PEAK_GBS, 4)}
    roof["kernel"] = f"k_step<{prec}> (fused force + velocity Verlet)"
    roof["kernel_ms"] = round(k_ms, 5)
    roof["algorithmic_bytes_per_launch"] = int(bytes_launch)
    roof["algorithmic_ops_per_launch"] = int(ops_launch)
    roof["hbm_frac"] = round(hbm_gbs / HBM_PEAK_GBS, 4)
    roof["alu_frac"] = round(alu_tops / VALU_PEAK_TOPS, 4)
    traffic = read_traffic(args.workload, prec, n_total, args.cell_order)
    roof["traffic"] = traffic
    log(f"roofline: {roof}")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(systems[0] if len(systems) == 1 else max(systems, key=lambda s: s.n))
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": "particle-steps/s (Kob-Andersen mixture, whole MD step)",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "ds": "f32 pair term, double-single (f32x2) sum and integration",
                  "mixed64": "f32 pair term, f64 sum and integration", "fp64": "f64"}[prec],
        "data": "synthetic (seeded fcc-subset start, Maxwell-Boltzmann velocities, rescaled equilibration)",
        "config": {"workload": args.workload, "description": desc, "particles": n_total,
                   "replicas": len(systems), "precision": prec,
                   "skin": args.skin if args.skin is not None else systems[0].skin,
                   "cell_order": args.cell_order,
                   "graph_steps": args.graph_steps, "equil_steps": args.equil,
                   "launch": pool.get_launch(),
                   "mean_list_entries": round(mean_list, 3), "rebuilds_in_timed_region": int(rebuilds)},
        "breakdown": {"step_kernel_ms": round(k_ms, 5),
                      "rebuild_group_ms_mean": round(prof["rebuild_ms_mean"], 5),
                      "rebuild_group_ms_when_rebuilding": round(prof["rebuild_ms_when_rebuilding"], 5),
                      "eager_ms_per_step": round(prof["total_ms"] / args.profile_steps, 5),
                      "force_only_kernel_ms": round(force_ms, 5)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if args.calib_copy:  # a copy of known size: 256 MiB read + 256 MiB written
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    pool.close()


if __name__ == "__main__":
    main()
