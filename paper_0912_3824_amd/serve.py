"""Continuous-batching serving loop for MD trajectory jobs on one GPU.

A job is a Kob-Andersen replica (N particles, a number of steps).  Jobs
arrive over time; the loop keeps every running job's state resident in one
libmdx pool and advances all of them together with md_advance, in chunks of
graph-captured steps.  Between chunks it

  * retires jobs that reached their step target (md_poll reports the step
    count and that the velocities are back at a full step), copying their
    final state out and releasing their slot and arena ranges (md_detach);
  * admits queued jobs in arrival order while a slot is free and the job's
    HBM footprint (its particle and cell ranges in the pool's arena) fits
    (md_attach refuses with MD_E_CAPACITY otherwise; the job then waits);
  * rejects, with an error result, a job that could never run: one that
    would not fit even an empty pool (md_validate), or one whose attach
    still fails once nothing else is running (e.g. its first Verlet lists
    exceed the pool's capacity);
  * retires with an error result a job whose replica stopped with an error
    bit (a list that outgrew its capacity, non-finite coordinates);
  * for a job that asks for time-correlation functions (Sec. 2.5), binds a
    blocking scheme to its slot at admission, stops the replica at a full
    step every tcf_every steps (its step target), samples it there, and
    returns the MSD / VACF / F_s curves with the job's result.  Stopping
    at a full step and resuming leaves the trajectory bitwise unchanged,
    so the curves are the ones the job computes alone.  Each advance runs
    up to the nearest target of any running job.

A replica's trajectory does not depend on the other replicas in the pool,
so every job's result is bitwise the one it would get alone.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import mdx


@dataclasses.dataclass
class JobResult:
    job_id: int
    n: int
    steps: int
    arrival: float
    admitted: float
    finished: float
    pos: Optional[np.ndarray]
    vel: Optional[np.ndarray]
    image: Optional[np.ndarray]
    error: Optional[str] = None
    tcf: Optional[dict] = None  # lags (samples), values [levels, block-1, species, (MSD, VACF, F_s)], terms

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def footprint_bytes(pool: "mdx.MdSystem", n: int) -> int:
    """Device bytes a job of n particles occupies in the pool's arena."""
    per = pool.ws_bytes / max(1, pool.cfg.max_particles)
    return int(math.ceil(per * n))


class Server:
    """Serve trajectory jobs from a pool of `max_slots` slots whose arena holds
    `max_particles` particles (chosen from an HBM budget by the caller)."""

    def __init__(self, table, precision="ds", dt=0.001, skin=0.3, max_slots=32,
                 max_particles=2_000_000, chunk_steps=256, device="cuda:0",
                 make_system: Optional[Callable] = None, pool=None, shape: Optional[dict] = None,
                 **cfg_kw):
        """cfg_kw: further md_config fields (e.g. rebuild_every, rebuild_early);
        shape: launch shape (md_launch fields) for the pool."""
        if pool is None:
            cfg = mdx.make_config(table, precision, dt, skin, max_slots, max_particles, **cfg_kw)
            pool = mdx.MdSystem(cfg, device=device)
            if shape:
                pool.set_launch(**shape)
        self.pool = pool
        self.chunk = int(chunk_steps)
        self.max_slots = max_slots
        self.make_system = make_system
        self.free = list(range(max_slots))
        self.running: Dict[int, dict] = {}

    @staticmethod
    def bytes_for_budget(table, precision, hbm_budget: float, max_slots: int,
                         dt=0.001, skin=0.3) -> int:
        """Largest arena (particles) whose workspace fits `hbm_budget` bytes."""
        probe = mdx.make_config(table, precision, dt, skin, max_slots, 1 << 20)
        per = mdx.md_workspace_bytes(probe) / (1 << 20)
        return int(hbm_budget / per)

    def _try_admit(self, job, system, now) -> str:
        """'admitted', 'wait' (no slot or arena space now) or an error text
        (the job can never run in this pool)."""
        if not self.free:
            return "wait"
        st = self.pool.validate(system.n, system.box)
        if st != 0:
            return f"{mdx.STATUS_NAMES.get(st, st)}: does not fit an empty pool"
        slot = self.free[0]
        try:
            self.pool.attach(slot, system.n, system.box, system.species, system.pos, system.vel)
        except mdx.MdError as e:
            if e.status != mdx.MD_E_CAPACITY:
                raise
            if self.running:  # arena full: wait for a job to finish
                return "wait"
            return str(e)  # refused by an empty pool: it never fits
        self.free.pop(0)
        r = {"job": job, "admitted": now, "tcf": None}
        every = int(getattr(job, "tcf_every", 0) or 0)
        if every > 0:
            r["tcf"] = self.pool.tcf(slot, job.tcf_levels, job.tcf_block, job.tcf_q)
            r["tcf"].sample()  # the replica starts at a full step
            r["next_sample"] = every
        r["target"] = min(job.steps, r["next_sample"]) if r["tcf"] is not None else job.steps
        self.pool.set_target(slot, r["target"])
        self.running[slot] = r
        return "admitted"

    def _release(self, slot):
        r = self.running.pop(slot)
        if r["tcf"] is not None:
            r["tcf"].close()
        self.pool.detach(slot)
        self.free.append(slot)
        self.free.sort()
        return r

    def run(self, jobs: List, time_scale: float = 1.0, log: Optional[Callable] = None) -> dict:
        """Serve `jobs` (md_inputs.Job, sorted by arrival).  Arrival times are
        in seconds of wall clock, multiplied by `time_scale`."""
        pending = sorted(jobs, key=lambda j: j.arrival)
        queue: List = []
        results: List[JobResult] = []
        t0 = time.perf_counter()
        busy = 0.0
        work = 0
        pi = 0
        while pi < len(pending) or queue or self.running:
            now = time.perf_counter() - t0
            while pi < len(pending) and pending[pi].arrival * time_scale <= now:
                queue.append((pending[pi], self.make_system(pending[pi])))  # built once per job
                pi += 1
            # admission in arrival order (head-of-line: a job that does not fit
            # yet blocks later ones, so large jobs are not starved)
            while queue:
                job, sys_ = queue[0]
                now = time.perf_counter() - t0
                outcome = self._try_admit(job, sys_, now)
                if outcome == "wait":
                    break
                queue.pop(0)
                if outcome != "admitted":
                    results.append(JobResult(job.job_id, sys_.n, job.steps, job.arrival * time_scale,
                                             now, now, None, None, None, error=outcome))
                    if log:
                        log(f"job {job.job_id} n={sys_.n} rejected: {outcome}")
            if not self.running:
                if pi < len(pending):  # idle until the next arrival
                    time.sleep(max(0.0, pending[pi].arrival * time_scale - (time.perf_counter() - t0)))
                continue
            tb = time.perf_counter()
            # up to the nearest target of a running job (a sample point or its
            # last step), plus the launch that finalises it at a full step
            launches = self.chunk
            for slot, r in self.running.items():
                launches = min(launches, max(1, r["target"] - r.get("steps", 0) + 1))
            self.pool.advance(launches)
            steps, status = self.pool.poll()
            busy += time.perf_counter() - tb
            now = time.perf_counter() - t0
            for slot in list(self.running):
                r = self.running[slot]
                job = r["job"]
                r["steps"] = int(steps[slot])
                if status[slot] & 0xFF:  # the replica stopped with an error bit
                    results.append(JobResult(job.job_id, self.pool.sizes[slot], job.steps,
                                             job.arrival * time_scale, r["admitted"], now, None, None,
                                             None, error=f"stopped at step {int(steps[slot])} with "
                                                         f"status bits {int(status[slot]) & 0xFF:#x}"))
                    self._release(slot)
                    if log:
                        log(f"job {job.job_id} failed: {results[-1].error}")
                    continue
                at_target = steps[slot] >= r["target"] and status[slot] & mdx.MD_ST_AT_FULL_STEP
                if at_target and r["tcf"] is not None and steps[slot] == r["next_sample"]:
                    r["tcf"].sample()
                    r["next_sample"] += job.tcf_every
                if at_target and steps[slot] < job.steps:  # a sample point: on to the next target
                    r["target"] = min(job.steps, r["next_sample"])
                    self.pool.set_target(slot, r["target"])
                    continue
                if steps[slot] >= job.steps and status[slot] & mdx.MD_ST_AT_FULL_STEP:
                    pos, vel, img = self.pool.get_state(slot)
                    curves = None
                    if r["tcf"] is not None:
                        lags, vals, terms = r["tcf"].read()
                        curves = {"lags": lags, "values": vals, "terms": terms, "every": job.tcf_every}
                    results.append(JobResult(job.job_id, self.pool.sizes[slot], job.steps,
                                             job.arrival * time_scale, r["admitted"], now,
                                             pos, vel, img, tcf=curves))
                    work += self.pool.sizes[slot] * job.steps
                    self._release(slot)
                    if log:
                        log(f"job {job.job_id} n={results[-1].n} steps={job.steps} "
                            f"latency {results[-1].latency:.3f}s")
        wall = time.perf_counter() - t0
        lat = np.array([r.latency for r in results if r.error is None])
        return {
            "results": sorted(results, key=lambda r: r.job_id),
            "failed": sorted(r.job_id for r in results if r.error is not None),
            "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "particle_steps": int(work),
            "busy_s": busy,
            "wall_s": wall,
            "throughput_busy": work / busy if busy > 0 else None,
            "throughput_wall": work / wall if wall > 0 else None,
        }

    def close(self):
        self.pool.close()
