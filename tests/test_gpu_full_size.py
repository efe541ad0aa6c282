"""Parity at the full workload sizes, in the launch configuration bench.py
times (the autotuner's cached shapes): the N = 1M and N = 64k Kob-Andersen
systems and the 256-replica ensemble.  The oracle computes forces, energies
and list membership for a random sample of particles one by one against all
N (brute force), on the seeded input as the precision mode holds it after
upload (oracle/upload.py; nothing read back from the device is fed to the
oracle).  Whole-system dynamics are checked through properties that hold at
any size (momentum and energy conservation, time reversibility)."""
import math

import numpy as np
import pytest

import md_inputs as I
from oracle import oracle as O
from oracle.upload import state_after_upload
from gpu_helpers import TOL_F, cutoff_jump, pool_for, say

pytestmark = pytest.mark.gpu


def _tuned_pool(systems, prec, **kw):
    from paper_0912_3824_amd import tune
    pool = pool_for(systems, prec, **kw)
    shape = tune.apply_cached(pool)
    say("launch", pool.get_launch(), "(cached)" if shape else "(defaults)")
    return pool


def _band_mask(pos, box, species, table, sel, radius_of, band):
    """Sampled particles with a pair within a relative `band` of radius_of."""
    from scipy.spatial import cKDTree
    p = np.mod(pos, box)
    p[p >= box] = 0.0
    tree = cKDTree(p, boxsize=box)
    rm = max(radius_of(a, b) for a in range(2) for b in range(2)) * (1 + 2 * band)
    out = np.zeros(len(sel), dtype=bool)
    sp = species if table.n_species > 1 else np.zeros(len(pos), dtype=int)
    for k, i in enumerate(sel):
        js = np.array([j for j in tree.query_ball_point(p[i], rm) if j != i], dtype=np.int64)
        if len(js) == 0:
            continue
        d = p[js] - p[i]
        d -= box * np.rint(d / box)
        r = np.sqrt((d * d).sum(axis=1))
        rad = np.array([radius_of(sp[i], sp[j]) for j in js])
        out[k] = bool(np.any(np.abs(r - rad) < band * rad))
    return out


def _sampled_parity(pool, slot, s, prec, m, seed):
    """Forces, energies and lists of a sample of particles at the uploaded
    state (call before any step)."""
    pos, vel, img = state_after_upload(s.pos, s.vel, s.box, prec)
    f, e = pool.forces(slot)
    assert np.isfinite(f).all() and np.isfinite(e).all()
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(s.n, size=min(m, s.n), replace=False)).astype(np.int32)
    fr, er, _ = O.forces(pos, s.box, s.species, s.table, sel)
    frms = math.sqrt(float(np.mean(fr * fr)))  # of the oracle's sampled forces
    # no device force may be wild anywhere (the sample sees only m of them)
    assert float(np.abs(f).max()) < 1e3 * frms
    excl = np.zeros(len(sel), dtype=bool)
    if prec != "fp64":
        excl = _band_mask(pos, s.box, s.species, s.table, sel, lambda a, b: s.table.rcut[a, b], 2e-6)
    d = np.abs(f[sel] - fr)
    # e_F = max component error / F_rms, and the relative error of each
    # sampled particle's force against its own magnitude with F_rms as the
    # floor (a near-zero force has no useful relative error); both held to
    # the tolerance
    rel = np.linalg.norm(f[sel] - fr, axis=1) / np.maximum(np.linalg.norm(fr, axis=1), frms)
    err = float(rel[~excl].max())
    say("  sampled", len(sel), "of", s.n, "per-particle relative error", err, "e_F",
        float(d[~excl].max()) / frms, "F_rms", frms, "excluded", int(excl.sum()))
    assert err < TOL_F[prec]
    assert float(d[~excl].max()) / frms < TOL_F[prec]  # e_F, F_rms of the oracle's forces
    if excl.any():  # one cutoff jump at most
        assert d[excl].max() < 2 * cutoff_jump(s.table) + TOL_F[prec] * frms
    scale = max(1.0, float(np.abs(er).max()))
    assert float(np.abs(e[sel] - er)[~excl].max()) < (1e-10 if prec == "fp64" else 1e-5) * scale
    # lists of the sample (built at upload) against brute-force membership
    cnt, ids = pool.neighbours(slot, cap=160)
    ref = O.neighbours(pos, s.box, s.species, s.table, s.skin, sel)
    amb = _band_mask(pos, s.box, s.species, s.table, sel, lambda a, b: s.table.rcut[a, b] + s.skin, 1e-6)
    bad = 0
    for k, i in enumerate(sel):
        got = ids[i, :cnt[i]]
        assert len(set(got.tolist())) == cnt[i]  # no duplicates
        if set(got.tolist()) != set(ref[k].tolist()):
            assert amb[k], (int(i), sorted(set(got.tolist()) ^ set(ref[k].tolist())))
            bad += 1
    say("  lists of the sample equal the oracle's; band cases", bad)


def test_ka1m_sampled_forces_lists_and_dynamics():
    """N = 1,000,000 KA at T = 0.5 in double-single (the benchmark system,
    from a jittered start so that no lattice shell sits on a cutoff)."""
    s = I.make_ka(1_000_000, 0.5, seed=20240101, jitter=0.08)
    pool = _tuned_pool([s], "ds")
    _sampled_parity(pool, 0, s, "ds", 256, seed=5)
    pool.step(200)
    # dynamics at full size: momentum stays zero, energy is conserved over
    # 100 steps, and 100 steps back with reversed velocities return the start
    o0 = pool.observables()[0]
    p0, v0, i0 = pool.get_state(0)
    pool.step(100)
    o1 = pool.observables()[0]
    pool.scale_velocities(0, -1.0)
    pool.step(100)
    o2 = pool.observables()[0]
    p2, v2, i2 = pool.get_state(0)
    de = abs(o1["etot"] - o0["etot"]) / s.n
    back = np.abs((p2 + i2 * s.box) - (p0 + i0 * s.box)).max()
    say("  |dE|/N over 100 steps", de, "momentum/N", np.abs(o1["momentum"]).max() / s.n,
        "return error after 100 + 100 reversed steps", back, "rebuilds", o2["n_rebuilds"])
    assert o1["status"] == 0 and o2["status"] == 0
    assert de < 1e-4
    assert np.abs(o1["momentum"]).max() / s.n < 1e-12
    assert back < 1e-4
    assert np.abs(v2 + v0).max() < 1e-4
    pool.close()


@pytest.mark.parametrize("prec", ["ds", "mixed64", "fp64", "fp32"])
def test_ka1m_every_particle_against_the_cell_list_oracle(prec):
    """N = 1,000,000 KA in every precision mode (double-single first), every
    particle: forces at the uploaded state against the oracle's cell-list
    forces, then ten steps against the oracle's velocity Verlet over Verlet
    lists (both FP64, both pinned against brute force), max |dr| and max
    |dv| over all particles.  FP32 rounds positions to ~8e-6 at this box
    size, so over ten steps some pairs cross the unsmoothed cutoff at other
    steps than in FP64, each changing a velocity by up to the force jump
    times dt: its velocities are held to that allowance (one such crossing
    per step) instead of 1e-4."""
    s = I.make_ka(1_000_000, 0.5, seed=20240101, jitter=0.08)
    pool = _tuned_pool([s], prec)
    pos, vel, img = state_after_upload(s.pos, s.vel, s.box, prec)
    f, _ = pool.forces(0)
    say("  oracle: cell-list forces of 1M particles")
    fr, _, _ = O.forces_cells(pos, s.box, s.species, s.table)
    frms = math.sqrt(float(np.mean(fr * fr)))
    rel = np.linalg.norm(f - fr, axis=1) / np.maximum(np.linalg.norm(fr, axis=1), frms)
    d = np.abs(f - fr)
    over = np.nonzero(rel >= TOL_F[prec])[0]
    # particles over the bound must each have a pair within rounding of a
    # cutoff (classified either way by an FP32 test; none in FP64) and
    # differ by at most one cutoff jump per such pair
    near = _band_mask(pos, s.box, s.species, s.table, over, lambda a, b: s.table.rcut[a, b], 2e-6)
    keep = np.ones(s.n, dtype=bool)
    keep[over] = False
    say("  all particles:", prec, "per-particle relative error", float(rel[keep].max()), "e_F",
        float(d[keep].max()) / frms, "over the bound", len(over), "(all near a cutoff:", bool(near.all()), ")")
    if prec == "fp64":
        assert len(over) == 0
    assert near.all()
    assert len(over) < 1e-3 * s.n
    assert float(d[keep].max()) / frms < TOL_F[prec]  # e_F over every other particle
    if len(over):
        assert float(d[over].max()) < 2 * cutoff_jump(s.table) + TOL_F[prec] * frms
    pool.step(10)
    p1, v1, i1 = pool.get_state(0)
    obs = pool.observables()[0]
    assert obs["status"] == 0
    say("  oracle: 10 velocity-Verlet steps of 1M particles over Verlet lists")
    pr, vr, ir, _, builds = O.vv_lists(pos, vel, s.box, s.species, s.table, s.dt, 10, s.skin)
    dr = np.abs((p1 + i1 * s.box) - (pr + (ir + img) * s.box))
    dv = np.abs(v1 - vr)
    say("  10 steps:", prec, "max|dr|", float(dr.max()), "max|dv|", float(dv.max()), "oracle builds", builds,
        "device builds", obs["n_rebuilds"])
    assert float(dr.max()) <= 1e-4
    assert float(dv.max()) <= (10 * 2 * cutoff_jump(s.table) * s.dt if prec == "fp32" else 1e-4)
    pool.close()


@pytest.mark.parametrize("prec", ["fp32", "ds", "mixed64", "fp64"])
def test_ka64k_sampled_forces_and_lists(prec):
    """N = 64,000 KA at T = 0.7, every precision mode."""
    s = I.make_ka(64_000, 0.7, seed=20240101, jitter=0.08)
    pool = _tuned_pool([s], prec)
    _sampled_parity(pool, 0, s, prec, 512, seed=6)
    pool.close()


def test_batch256_sampled_forces_and_lists():
    """The 256-replica ensemble (N log-uniform in [500, 8000]) in its tuned
    launch shapes: a sample of replicas, each against the oracle."""
    reps = I.make_ka_ensemble(256, seed=20240101, jitter=0.08)
    pool = _tuned_pool(reps, "ds")
    for k in (0, 37, 101, 170, 255):
        say("replica", k, "N", reps[k].n)
        _sampled_parity(pool, k, reps[k], "ds", 128, seed=k)
    pool.step(100)
    obs = pool.observables()
    assert not any(o["status"] for o in obs if o["n"])
    pool.close()


@pytest.mark.parametrize("aligned", [False, True])
def test_batch256_every_particle_against_the_cell_list_oracle(aligned):
    """Every particle of every replica of the 256-replica ensemble (716k
    particles, double-single), in the tuned launch shapes of the pool with
    and without aligned rebuilds (with: the rebuild policy and skin of the
    ensemble measurement): forces at the uploaded state against the
    oracle's cell-list forces (particles with a pair within rounding of a
    cutoff held to one cutoff jump per such pair), then ten steps against
    its velocity Verlet over Verlet lists, max |dr| and max |dv| over all
    particles."""
    reps = I.make_ka_ensemble(256, seed=20240101, jitter=0.08)
    from paper_0912_3824_amd import patterns_bench as PB
    kw = dict(PB.BATCH_POLICY) if aligned else {}
    pool = _tuned_pool(reps, "ds", **kw)
    starts, worst_rel, worst_ef, n_over = [], 0.0, 0.0, 0
    for k, s in enumerate(reps):
        pos, vel, img = state_after_upload(s.pos, s.vel, s.box, "ds")
        starts.append((pos, vel, img))
        f, _ = pool.forces(k)
        fr, _, _ = O.forces_cells(pos, s.box, s.species, s.table)
        frms = math.sqrt(float(np.mean(fr * fr)))
        rel = np.linalg.norm(f - fr, axis=1) / np.maximum(np.linalg.norm(fr, axis=1), frms)
        d = np.abs(f - fr)
        over = np.nonzero(rel >= TOL_F["ds"])[0]
        keep = np.ones(s.n, dtype=bool)
        keep[over] = False
        if len(over):
            near = _band_mask(pos, s.box, s.species, s.table, over, lambda a, b: s.table.rcut[a, b], 2e-6)
            assert near.all(), k
            assert float(d[over].max()) < 2 * cutoff_jump(s.table) + TOL_F["ds"] * frms, k
        n_over += len(over)
        worst_rel = max(worst_rel, float(rel[keep].max()))
        worst_ef = max(worst_ef, float(d[keep].max()) / frms)
    say("  forces, all replicas: per-particle relative error", worst_rel, "e_F", worst_ef,
        "particles over the bound", n_over)
    assert worst_ef < TOL_F["ds"]
    assert n_over < 1e-3 * sum(s.n for s in reps)
    pool.step(10)
    obs = pool.observables()
    worst_dr = worst_dv = 0.0
    for k, s in enumerate(reps):
        assert obs[k]["status"] == 0, k
        p1, v1, i1 = pool.get_state(k)
        pos, vel, img = starts[k]
        pr, vr, ir, _, _ = O.vv_lists(pos, vel, s.box, s.species, s.table, s.dt, 10, s.skin)
        worst_dr = max(worst_dr, float(np.abs((p1 + i1 * s.box) - (pr + (ir + img) * s.box)).max()))
        worst_dv = max(worst_dv, float(np.abs(v1 - vr).max()))
    say("  10 steps, all replicas: max|dr|", worst_dr, "max|dv|", worst_dv)
    assert worst_dr <= 1e-4 and worst_dv <= 1e-4
    pool.close()


@pytest.mark.parametrize("prec", ["fp32", "ds", "mixed64", "fp64"])
def test_ka64k_every_particle_against_the_cell_list_oracle(prec):
    """N = 64,000 KA at T = 0.7 in every precision mode, every particle:
    forces at the uploaded state against the oracle's cell-list forces, then
    ten steps against its velocity Verlet over Verlet lists.  FP32 rounds
    positions to ~4e-6 at this box size, so some pairs cross the unsmoothed
    cutoff at other steps than in FP64, each changing a velocity by up to
    the force jump times dt: its velocities are held to that allowance (one
    such crossing per step) instead of 1e-4."""
    s = I.make_ka(64_000, 0.7, seed=20240101, jitter=0.08)
    pool = _tuned_pool([s], prec)
    pos, vel, img = state_after_upload(s.pos, s.vel, s.box, prec)
    f, _ = pool.forces(0)
    fr, _, _ = O.forces_cells(pos, s.box, s.species, s.table)
    frms = math.sqrt(float(np.mean(fr * fr)))
    rel = np.linalg.norm(f - fr, axis=1) / np.maximum(np.linalg.norm(fr, axis=1), frms)
    d = np.abs(f - fr)
    over = np.nonzero(rel >= TOL_F[prec])[0]
    keep = np.ones(s.n, dtype=bool)
    keep[over] = False
    say("  all particles:", prec, "per-particle relative error", float(rel[keep].max()), "e_F",
        float(d[keep].max()) / frms, "over the bound", len(over))
    if len(over):
        near = _band_mask(pos, s.box, s.species, s.table, over, lambda a, b: s.table.rcut[a, b], 2e-6)
        assert prec != "fp64" and near.all()
        assert float(d[over].max()) < 2 * cutoff_jump(s.table) + TOL_F[prec] * frms
    assert float(d[keep].max()) / frms < TOL_F[prec]
    pool.step(10)
    p1, v1, i1 = pool.get_state(0)
    assert pool.observables()[0]["status"] == 0
    pr, vr, ir, _, builds = O.vv_lists(pos, vel, s.box, s.species, s.table, s.dt, 10, s.skin)
    dr = float(np.abs((p1 + i1 * s.box) - (pr + (ir + img) * s.box)).max())
    dv = float(np.abs(v1 - vr).max())
    say("  10 steps:", prec, "max|dr|", dr, "max|dv|", dv)
    assert dr <= 1e-4
    assert dv <= (10 * 2 * cutoff_jump(s.table) * s.dt if prec == "fp32" else 1e-4)
    pool.close()
