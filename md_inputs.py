"""Seeded synthetic inputs for the Lennard-Jones / Kob-Andersen MD workloads.

This module is shared by the oracle (test infrastructure) and by the HIP path's
callers (tests, bench).  It holds only input preparation: lattice starts,
species assignment, Maxwell-Boltzmann velocities, pair-parameter tables and
the workload definitions.  It holds none of the method's arithmetic (no forces,
no integrator, no neighbour search).

Workloads follow the paper's stated systems:
  * single-species LJ liquid, fcc start, rc = 2.5 sigma (Sec. 3, "Performance
    measurements", LJ 12-6 potential cut off at 2.5 sigma, dt* = 0.001);
  * Kob-Andersen 80/20 binary mixture at density 1.2 with the pair table of
    Sec. 5 ("Application to glassy dynamics": sigma_AA=1, sigma_BB=0.88,
    sigma_AB=0.8, eps_AA=1, eps_BB=0.5, eps_AB=1.5, equal masses).

Readings where the paper is silent:
  * the cutoff of each KA pair is 2.5 sigma_ab;
  * N that is not 4 n^3 is placed on a random subset of an fcc lattice with
    n = ceil((N/4)^(1/3)) cells per edge;
  * the box edge L = (N/rho)^(1/3) is rounded to the nearest float32 so that
    every precision mode holds exactly the same box;
  * T = 2 E_kin / (3 N) (velocities rescaled to exactly this T, zero momentum).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

MASTER_SEED = 20240101

# Species codes
A, B = 0, 1


@dataclasses.dataclass
class PairTable:
    """Symmetric per-species-pair LJ parameters (absolute cutoffs)."""
    n_species: int
    eps: np.ndarray     # [2,2]
    sigma: np.ndarray   # [2,2]
    rcut: np.ndarray    # [2,2]
    smooth: float = 0.0 # h of the C2 smoothing factor (0 = none)

    def max_rcut(self) -> float:
        k = self.n_species
        return float(self.rcut[:k, :k].max())


def lj_table(rc: float = 2.5, smooth: float = 0.0) -> PairTable:
    """Single-species LJ, eps = sigma = 1, cutoff rc (Sec. 3); rc = 2^(1/6)
    gives the WCA potential of Sec. 4; `smooth` is the width h of its C2
    smoothing."""
    e = np.ones((2, 2))
    s = np.ones((2, 2))
    return PairTable(1, e, s, np.full((2, 2), rc), smooth=smooth)


WCA_RC = 2.0 ** (1.0 / 6.0)


def smoothed(system: "System", h: float) -> "System":
    """The same replica with the pair table's smoothing width set to h."""
    return dataclasses.replace(system, table=dataclasses.replace(system.table, smooth=h))


def ka_table(rc_over_sigma: float = 2.5) -> PairTable:
    """Kob-Andersen pair table of Sec. 5; rc_ab = 2.5 sigma_ab (reading)."""
    eps = np.array([[1.0, 1.5], [1.5, 0.5]])
    sig = np.array([[1.0, 0.8], [0.8, 0.88]])
    return PairTable(2, eps, sig, rc_over_sigma * sig)


def box_length(n: int, rho: float, float32_box: bool = True) -> float:
    """Cubic box edge for density rho, rounded to the nearest float32 unless
    float32_box is False (then the double (n / rho)^(1/3))."""
    L = (n / rho) ** (1.0 / 3.0)
    return float(np.float32(L)) if float32_box else float(L)


def fcc_positions(n: int, box: float, rng: Optional[np.random.Generator],
                  jitter: float = 0.0) -> np.ndarray:
    """N positions on (a random subset of) an fcc lattice filling the box.

    n_c = ceil((n/4)^(1/3)) unit cells per edge, lattice constant box/n_c.
    When 4 n_c^3 > n, a seeded random subset of sites is kept (sorted by site
    index).  `jitter` adds a uniform displacement in [-jitter, jitter) per
    component (used to break lattice-shell degeneracy in list tests).
    Positions are wrapped into [0, box).
    """
    nc = int(math.ceil((n / 4.0) ** (1.0 / 3.0) - 1e-9))
    while 4 * nc ** 3 < n:
        nc += 1
    a = box / nc
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    g = np.arange(nc)
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    sites = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    if len(sites) > n:
        if rng is None:
            raise ValueError("a subset of lattice sites needs an rng")
        keep = np.sort(rng.choice(len(sites), size=n, replace=False))
        sites = sites[keep]
    pos = sites + 0.25 * a  # keep sites off the box faces
    if jitter > 0.0:
        if rng is None:
            raise ValueError("jitter needs an rng")
        pos = pos + rng.uniform(-jitter, jitter, size=pos.shape)
    pos = np.mod(pos, box)
    pos[pos >= box] = 0.0
    return np.ascontiguousarray(pos, dtype=np.float64)


def species_80_20(n: int, rng: np.random.Generator) -> np.ndarray:
    """Exactly round(0.8 n) A particles, placed by a seeded permutation."""
    na = int(round(0.8 * n))
    sp = np.full(n, B, dtype=np.int32)
    sp[rng.permutation(n)[:na]] = A
    return sp


def maxwell_velocities(n: int, temperature: float, rng: np.random.Generator,
                       mass: float = 1.0) -> np.ndarray:
    """Gaussian velocities, zero total momentum, rescaled to exactly T
    with T = m sum v^2 / (3 n)."""
    v = rng.normal(0.0, math.sqrt(temperature / mass), size=(n, 3))
    v -= v.mean(axis=0)
    t_now = mass * float(np.sum(v * v)) / (3.0 * n)
    if t_now > 0:
        v *= math.sqrt(temperature / t_now)
    return np.ascontiguousarray(v, dtype=np.float64)


@dataclasses.dataclass
class System:
    """One replica: positions/velocities in FP64, species, cubic box."""
    n: int
    box: float
    pos: np.ndarray
    vel: np.ndarray
    species: np.ndarray
    table: PairTable
    temperature: float
    dt: float = 0.001
    skin: float = 0.3
    mass: float = 1.0
    label: str = ""


def make_lj(n: int = 4000, rho: float = 0.8442, temperature: float = 1.5,
            seed: int = MASTER_SEED, jitter: float = 0.0,
            rc: float = 2.5, skin: float = 0.3) -> System:
    """Single-species LJ fluid on an fcc start (4000 = 4 * 10^3 sites)."""
    ss = np.random.SeedSequence(seed)
    rng = np.random.Generator(np.random.PCG64(ss))
    box = box_length(n, rho)
    pos = fcc_positions(n, box, rng, jitter)
    vel = maxwell_velocities(n, temperature, rng)
    sp = np.zeros(n, dtype=np.int32)
    return System(n, box, pos, vel, sp, lj_table(rc), temperature, skin=skin,
                  label=f"lj_n{n}_rho{rho}")


def make_ka(n: int, temperature: float, rho: float = 1.2,
            seed: int = MASTER_SEED, jitter: float = 0.0,
            skin: float = 0.3, rng: Optional[np.random.Generator] = None,
            float32_box: bool = True) -> System:
    """Kob-Andersen 80/20 mixture at density rho on an fcc-subset start."""
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    box = box_length(n, rho, float32_box)
    pos = fcc_positions(n, box, rng, jitter)
    sp = species_80_20(n, rng)
    vel = maxwell_velocities(n, temperature, rng)
    return System(n, box, pos, vel, sp, ka_table(), temperature, skin=skin,
                  label=f"ka_n{n}_rho{rho}_T{temperature}")


def make_ka_ensemble(n_rep: int = 256, n_lo: int = 500, n_hi: int = 8000,
                     temps=(0.45, 0.5, 0.6, 0.8), seed: int = MASTER_SEED,
                     jitter: float = 0.0, skin: float = 0.3) -> List[System]:
    """Batched ensemble: N log-uniform in [n_lo, n_hi], T from `temps`,
    each replica drawn from its own spawned stream."""
    root = np.random.SeedSequence(seed)
    top = np.random.Generator(np.random.PCG64(root.spawn(1)[0]))
    ns = np.exp(top.uniform(math.log(n_lo), math.log(n_hi), size=n_rep))
    ns = np.clip(np.round(ns).astype(int), n_lo, n_hi)
    ts = top.choice(np.asarray(temps, dtype=float), size=n_rep)
    out = []
    for k, child in enumerate(root.spawn(n_rep + 1)[1:]):
        rng = np.random.Generator(np.random.PCG64(child))
        s = make_ka(int(ns[k]), float(ts[k]), rng=rng, jitter=jitter, skin=skin)
        s.label = f"rep{k}_n{ns[k]}_T{ts[k]}"
        out.append(s)
    return out


@dataclasses.dataclass
class Job:
    """A trajectory job of the serving trace.  A job with tcf_every > 0 also
    asks for time-correlation functions (Sec. 2.5 blocking scheme: levels of
    tcf_block entries, a sample every tcf_every steps, wave number tcf_q)."""
    job_id: int
    arrival: float      # seconds after trace start
    n: int
    steps: int
    temperature: float
    seed: int
    tcf_every: int = 0
    tcf_levels: int = 4
    tcf_block: int = 10
    tcf_q: float = 7.25


def serving_trace(n_jobs: int, rate_per_s: float, n_lo: int = 1000,
                  n_hi: int = 256000, steps_lo: int = 1000,
                  steps_hi: int = 100000, t_lo: float = 0.45,
                  t_hi: float = 1.0, seed: int = MASTER_SEED,
                  tcf_fraction: float = 0.0, tcf_every: int = 10,
                  tcf_levels: int = 4, tcf_block: int = 10) -> List[Job]:
    """Poisson arrivals (exponential gaps at `rate_per_s`) of KA jobs with
    N log-uniform in [n_lo, n_hi], steps uniform in [steps_lo, steps_hi],
    T uniform in [t_lo, t_hi]; a seeded `tcf_fraction` of them also ask for
    time-correlation functions sampled every `tcf_every` steps (wave number
    q = 7.25, the first peak of the KA structure factor, Sec. 5)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 5])))
    gaps = rng.exponential(1.0 / rate_per_s, size=n_jobs)
    arr = np.cumsum(gaps) - gaps[0]
    ns = np.round(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), n_jobs))).astype(int)
    st = rng.integers(steps_lo, steps_hi + 1, size=n_jobs)
    ts = rng.uniform(t_lo, t_hi, size=n_jobs)
    seeds = rng.integers(1, 2**31 - 1, size=n_jobs)
    wants = rng.uniform(size=n_jobs) < tcf_fraction
    return [Job(i, float(arr[i]), int(ns[i]), int(st[i]), float(ts[i]), int(seeds[i]),
                tcf_every=tcf_every if wants[i] else 0, tcf_levels=tcf_levels, tcf_block=tcf_block)
            for i in range(n_jobs)]


def job_system(job: Job, skin: float = 0.3) -> System:
    """The initial state of a serving job (fcc subset + MB velocities)."""
    s = make_ka(job.n, job.temperature, seed=job.seed, skin=skin)
    s.label = f"job{job.job_id}"
    return s


# Named workloads (sizes of the paper's systems; see module docstring).
def workload(name: str, seed: int = MASTER_SEED) -> System:
    if name == "lj4000":
        return make_lj(4000, seed=seed)
    if name == "ka64k":
        return make_ka(64000, 0.7, seed=seed)
    if name == "ka1m":
        return make_ka(1000000, 0.5, seed=seed)
    raise KeyError(name)
