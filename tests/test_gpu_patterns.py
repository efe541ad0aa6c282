"""GPU tests of the systems patterns around the hot path, through the C ABI:
bitwise independence of replicas in a batch, graph replay vs eager launches,
launch shapes, split md_step calls, checkpoint/resume, the serving loop's
alone-vs-mix results, the autotuner, double-single arithmetic against exact
rational arithmetic, conservation laws, and error paths."""
import math
from fractions import Fraction

import numpy as np
import pytest

import md_inputs as I
from gpu_helpers import pool_for, say

pytestmark = pytest.mark.gpu


def _state(pool, slot=0):
    p, v, i = pool.get_state(slot)
    return p.copy(), v.copy(), i.copy()


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def _reps():
    out = []
    for k, (n, T) in enumerate([(600, 0.8), (1500, 0.5), (3001, 0.6), (5003, 0.45)]):
        out.append(I.make_ka(n, T, jitter=0.05, seed=100 + k))
    return out


@pytest.mark.parametrize("prec,align", [("ds", 0), ("fp32", 0), ("fp64", 0), ("ds", 8), ("fp64", 4)])
def test_batched_replicas_equal_alone(prec, align):
    """Replicas of uneven N advanced together by one pool are bitwise equal to
    the same replicas advanced alone (incl. one in single-cell mode), also
    with aligned rebuilds (a replica's rebuild steps depend on its own state
    only)."""
    reps = _reps()
    kw = dict(rebuild_every=align, rebuild_early=0.6) if align else {}
    say("batched vs alone", prec, "aligned rebuilds every", align)
    pool = pool_for(reps, prec, **kw)
    pool.step(300)
    batched = [_state(pool, k) for k in range(len(reps))]
    obs = pool.observables()
    assert all(o["n_rebuilds"] >= 2 for o in obs[:len(reps)])
    pool.close()
    for k, s in enumerate(reps):
        alone = pool_for([s], prec, **kw)
        alone.step(300)
        assert _same(_state(alone), batched[k]), k
        alone.close()


@pytest.mark.parametrize("prec", ["ds", "fp64"])
def test_bulk_list_build_keeps_trajectories_bitwise(prec):
    """A step's list build takes one lane per member and unsplit row segments
    when at least build_bulk replicas rebuild in it.  With aligned rebuilds
    (most replicas rebuilding in the same steps, a few early) the
    trajectories of every replica, the single-cell one included, are the
    same bit for bit whether no build, every build or only the crowded ones
    take that shape."""
    reps = _reps() + [I.make_ka(n, 0.6, jitter=0.05, seed=200 + k) for k, n in enumerate([2000, 4001, 900, 7000])]
    ref = None
    for shape in [dict(build_lanes=8, build_split=4, build_block=512, build_bulk=0),
                  dict(build_lanes=8, build_split=4, build_block=512, build_bulk=1),
                  dict(build_lanes=0, build_split=0, build_block=320, build_bulk=4),
                  dict(build_lanes=2, build_split=2, build_block=256, build_bulk=6)]:
        say("bulk build", prec, shape)
        pool = pool_for(reps, prec, rebuild_every=8, rebuild_early=0.6)
        pool.set_launch(**shape)
        pool.step(300)
        st = [_state(pool, k) for k in range(len(reps))]
        assert all(o["n_rebuilds"] >= 2 for o in pool.observables()[:len(reps)])
        pool.close()
        if ref is None:
            ref = st
        assert all(_same(a, b) for a, b in zip(st, ref)), shape


def test_aligned_rebuilds_happen_at_multiples_and_follow_the_oracle():
    """With rebuild_every = 8 the rebuilds of a replica (counted per step)
    fall on multiples of 8 unless the skin/2 rule forces one earlier, and the
    trajectory stays within the oracle's tolerance (rebuilding early only
    moves list builds)."""
    from oracle import oracle as O
    from oracle.upload import state_after_upload
    s = I.make_ka(3001, 1.0, jitter=0.1, seed=4)
    pool = pool_for([s], "ds", rebuild_every=8, rebuild_early=0.5)
    steps_at, last = [], pool.observables()[0]["n_rebuilds"]
    for k in range(1, 201):
        pool.step(1)
        nr = pool.observables()[0]["n_rebuilds"]
        if nr != last:
            steps_at.append(k)
            last = nr
    say("aligned rebuild steps", steps_at)
    assert len(steps_at) >= 4
    assert sum(1 for k in steps_at if k % 8 == 0) >= 0.75 * len(steps_at)
    p1, v1, i1 = pool.get_state(0)
    p0, v0, i0 = state_after_upload(s.pos, s.vel, s.box, "ds")
    pr, vr, ir, _ = O.vv(p0, v0, s.box, s.species, s.table, s.dt, 200)
    d = np.abs((p1 + i1 * s.box) - (pr + (ir + i0) * s.box)).max()
    assert d < 1e-4
    pool.close()


def test_graph_eager_shapes_and_split_calls_are_bitwise_equal():
    s = I.make_ka(4001, 0.7, jitter=0.05, seed=8)
    say("graph/eager/shapes")
    ref = None
    for shape, calls in [(dict(graph_steps=32), [400]),
                         (dict(graph_steps=0), [400]),
                         (dict(graph_steps=8, step_block=64, build_width=2, build_block=128), [400]),
                         (dict(graph_steps=32, step_block=1024, xcd_remap=1, build_width=16), [150, 1, 249]),
                         (dict(graph_steps=2), [100, 100, 200]),
                         (dict(build_lanes=1, build_block=512), [400]),
                         (dict(build_lanes=64, build_block=1024, build_width=1), [200, 200]),
                         (dict(build_lanes=4, build_block=128, build_width=3), [400]),
                         # observation launches between calls overwrite the
                         # rows that hold the finalising launch's forces
                         (dict(graph_steps=32), [150, "obs", 1, "forces", 249]),
                         (dict(graph_steps=0), [7, "forces", "obs", 393])]:
        pool = pool_for([s], "ds")
        pool.set_launch(**shape)
        for c in calls:
            if c == "obs":
                pool.observables()
            elif c == "forces":
                pool.forces(0)
            else:
                pool.step(c)
        st = _state(pool)
        if ref is None:
            ref = st
        assert _same(st, ref), shape
        pool.close()


@pytest.mark.parametrize("prec", ["fp32", "mixed64", "fp64"])
def test_observation_between_calls_is_bitwise_in_every_mode(prec):
    """The forces a call's finalising launch keeps are reused by the next
    call; md_forces and md_observables in between (which write the same rows)
    leave the trajectory bitwise unchanged in the other precision modes too."""
    s = I.make_ka(4001, 0.7, jitter=0.05, seed=8)
    runs = []
    for calls in ([400], [150, "obs", 1, "forces", 249], [7, "forces", "obs", 393]):
        pool = pool_for([s], prec)
        for c in calls:
            if c == "obs":
                pool.observables()
            elif c == "forces":
                pool.forces(0)
            else:
                pool.step(c)
        runs.append(_state(pool))
        pool.close()
    assert _same(runs[0], runs[1]) and _same(runs[0], runs[2])


@pytest.mark.parametrize("prec", ["ds", "mixed64", "fp64"])
def test_checkpoint_resume_is_bitwise(prec):
    s = I.make_ka(3001, 0.7, jitter=0.08, seed=9)
    say("resume", prec)
    pool = pool_for([s], prec)
    pool.step(300)
    ref = _state(pool)
    pool.close()
    a = pool_for([s], prec)
    a.step(137)
    blob = a.save(0)
    a.close()
    b = pool_for([I.make_ka(500, 0.5, seed=1)], prec, max_slots=2, extra_particles=s.n)
    b.restore(1, blob, s.n, s.box)
    b.step(163)
    assert _same(_state(b, 1), ref)
    b.close()


def test_serving_results_equal_alone():
    """Jobs served in a continuously batched pool (arrivals while others run,
    slots and arena reused) end bitwise where they end alone."""
    from paper_0912_3824_amd.serve import Server
    jobs = I.serving_trace(7, rate_per_s=40.0, n_lo=500, n_hi=6000, steps_lo=150, steps_hi=700, seed=3)
    say("serving", [(j.n, j.steps) for j in jobs])
    srv = Server(I.ka_table(), "ds", max_slots=3, max_particles=12000, chunk_steps=64,
                 make_system=lambda j: I.job_system(j))
    out = srv.run(jobs)
    srv.close()
    assert len(out["results"]) == len(jobs)
    assert out["p99_latency_s"] >= out["p50_latency_s"] > 0
    for r, j in zip(out["results"], jobs):
        alone = pool_for([I.job_system(j)], "ds")
        alone.step(j.steps)
        p, v, i = alone.get_state(0)
        assert np.array_equal(p, r.pos) and np.array_equal(v, r.vel) and np.array_equal(i, r.image), j
        alone.close()


def test_autotuner_keeps_results():
    from paper_0912_3824_amd import tune
    s = I.make_ka(3001, 0.6, jitter=0.05, seed=12)
    pool = pool_for([s], "ds")
    ref_pool = pool_for([s], "ds")
    res = tune.tune(pool, steps=20, space={"step_block": [128, 512], "build_width": [4, 8],
                                          "build_block": [256], "graph_steps": [16], "xcd_remap": [0]},
                    cache=None)
    say("tuned", res["best"], res["us_per_step"])
    assert len(res["all"]) == 4
    pool.step(200)
    ref_pool.step(200)
    assert _same(_state(pool), _state(ref_pool))
    pool.close()
    ref_pool.close()


def _exact(h, l):
    return Fraction(float(h)) + Fraction(float(l))


def test_double_single_arithmetic_against_exact_rationals():
    """Device double-single add/sub/mul and the compensated sum against
    Fraction arithmetic: relative error below 2^-44 (Sec. 2.4) apart from
    cancellation, where the error is bounded by 2^-44 of the operands."""
    import torch
    from paper_0912_3824_amd import mdx
    rng = np.random.default_rng(5)
    n = 20000

    def ds_of(x):
        hi = x.astype(np.float32)
        lo = (x - hi.astype(np.float64)).astype(np.float32)
        return np.stack([hi, lo], 1)

    x = rng.uniform(-1, 1, n) * 10.0 ** rng.integers(-6, 6, n)
    y = rng.uniform(-1, 1, n) * 10.0 ** rng.integers(-6, 6, n)
    y[: n // 10] = -x[: n // 10] * (1 + rng.uniform(-1e-6, 1e-6, n // 10))  # cancellation
    a, b = ds_of(x), ds_of(y)
    ta = torch.tensor(a, device="cuda")
    tb = torch.tensor(b, device="cuda")
    out = torch.empty_like(ta)
    for op in (0, 1, 2):
        mdx.md_ds_eval(op, ta, tb, out)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        worst = 0.0
        for k in range(0, n, 7):
            A, B = _exact(*a[k]), _exact(*b[k])
            ex = A + B if op == 0 else (A - B if op == 1 else A * B)
            got = _exact(*o[k])
            scale = (abs(A) + abs(B)) if op < 2 else abs(ex)
            if scale == 0:
                continue
            worst = max(worst, float(abs(got - ex) / scale))
            assert abs(o[k, 1]) <= abs(float(np.spacing(o[k, 0]))) / 2 * (1 + 1e-6)  # normalised
        say("op", op, "worst rel err", worst)
        assert worst < 2.0 ** -44
    # compensated sum of a force-like series (128 terms with cancellation):
    # within the Sum2 bound (n u)^2 sum|x| of Ogita, Rump & Oishi, u = 2^-24
    u = Fraction(1, 2 ** 24)
    for trial in range(20):
        vals = rng.normal(0, 10, 64).astype(np.float32)
        vals = np.concatenate([vals, -vals[::-1] * np.float32(1 + 1e-5)]).astype(np.float32)
        rng.shuffle(vals)
        tv = torch.tensor(np.stack([vals, np.zeros_like(vals)], 1), device="cuda")
        o2 = torch.empty(2, dtype=torch.float32, device="cuda")
        mdx.md_ds_eval(3, tv, None, o2)
        torch.cuda.synchronize()
        got = _exact(*o2.cpu().numpy())
        ex = sum(Fraction(float(v)) for v in vals)
        assert abs(got - ex) <= (len(vals) * u) ** 2 * sum(abs(Fraction(float(v))) for v in vals)


@pytest.mark.parametrize("prec", ["fp32", "ds", "mixed64", "fp64"])
def test_momentum_and_energy_conservation(prec):
    s = I.make_ka(6000, 0.7, jitter=0.05, seed=21)
    pool = pool_for([s], prec)
    o0 = pool.observables()[0]
    pool.step(2000)
    o1 = pool.observables()[0]
    dp = np.abs(o1["momentum"] - o0["momentum"]).max()
    de = abs(o1["etot"] - o0["etot"]) / abs(o0["etot"])
    say(prec, "dP", dp, "dE/E", de, "T", o1["temperature"])
    # momentum: an FP32 force sum conserves it to ~1e-7 per particle-force,
    # double-single / double sums far better
    assert dp < (1e-2 if prec == "fp32" else 1e-6)
    assert de < 1e-3
    pool.close()


def test_scale_velocities_sets_temperature():
    s = I.make_ka(2000, 0.7, seed=3)
    pool = pool_for([s], "ds")
    pool.scale_velocities(0, math.sqrt(0.5 / 0.7))
    assert pool.observables()[0]["temperature"] == pytest.approx(0.5, rel=1e-6)
    pool.close()


def test_error_paths():
    from paper_0912_3824_amd import mdx
    s = I.make_ka(2000, 0.7, seed=3)
    # list capacity far too small: the first build overflows at attach
    with pytest.raises(mdx.MdError) as ei:
        pool_for([s], "ds", nbr_capacity=8)
    assert ei.value.status == -4
    # box too small for the list radius
    small = I.make_ka(100, 0.7, seed=3)
    with pytest.raises(mdx.MdError) as ei:
        pool_for([small], "ds")
    assert ei.value.status == -2
    # arena too small for a second replica; slot reuse after detach
    pool = pool_for([s], "ds", max_slots=2)
    with pytest.raises(mdx.MdError) as ei:
        pool.attach_system(1, s)
    assert ei.value.status == -4
    with pytest.raises(mdx.MdError):
        pool.attach_system(0, s)   # slot busy
    pool.detach(0)
    pool.attach_system(1, s)
    # launch shapes out of range are refused and leave the shape unchanged
    before = pool.get_launch()
    for bad in (dict(build_bulk=-1), dict(build_lanes=3), dict(build_split=257), dict(step_block=96)):
        with pytest.raises(mdx.MdError) as ei:
            pool.set_launch(**bad)
        assert ei.value.status == -1, bad
        assert pool.get_launch() == before, bad
    pool.step(10)
    assert pool.observables()[1]["step"] == 10
    pool.close()


def _imploding_ka(n=3001, speed=15.0, seed=41):
    """A KA replica whose inner sphere (radius 0.45 L) is given an inward
    radial velocity of up to `speed` on top of its thermal velocities: the
    local density in the centre rises by ~1.8x within ~60 steps, so its
    Verlet lists outgrow a capacity that equilibrium replicas never reach
    (checked on the CPU with the oracle: the largest count within 2.8 sigma
    goes 124 -> 240 and positions stay finite)."""
    s = I.make_ka(n, 0.6, jitter=0.05, seed=seed)
    d = s.pos - s.box / 2
    r = np.linalg.norm(d, axis=1)
    m = r < 0.45 * s.box
    v = s.vel.copy()
    v[m] -= speed * d[m] / np.maximum(r[m], 1e-9)[:, None] * np.minimum(1.0, r[m] / 2.0)[:, None]
    s.vel = v
    return s


def test_list_overflow_mid_run_stops_the_replica_and_spares_the_others():
    """A replica whose Verlet lists outgrow the pool's capacity mid-run stops
    at the step whose rebuild overflowed (no step runs on a truncated
    list); md_poll and md_observables report MD_E_CAPACITY with the bit in
    its status; launching calls refuse until it is detached; the other
    replicas of the pool are bitwise what they are alone."""
    from paper_0912_3824_amd import mdx
    normal = [I.make_ka(1500, 0.6, jitter=0.05, seed=42), I.make_ka(3001, 0.5, jitter=0.05, seed=43)]
    boom = _imploding_ka()
    cap = 160
    pool = pool_for(normal + [boom], "ds", nbr_capacity=cap)
    pool.step(200)
    steps, status = pool.poll()
    say("overflow run: steps", steps[:3].tolist(), "status", status[:3].tolist())
    assert status[2] & mdx.MD_ST_LIST_OVERFLOW
    assert 0 < steps[2] < 200
    assert steps[0] == 200 and steps[1] == 200
    assert not (status[0] & 0xFF) and not (status[1] & 0xFF)
    with pytest.raises(mdx.MdError) as ei:
        pool.observables()
    assert ei.value.status == mdx.MD_E_CAPACITY
    obs = pool.observables(check=False)
    assert obs[2]["status"] & mdx.MD_ST_LIST_OVERFLOW and obs[2]["step"] == steps[2]
    with pytest.raises(mdx.MdError) as ei:
        pool.step(10)
    assert ei.value.status == mdx.MD_E_CAPACITY
    stopped = _state(pool, 2)
    pool.detach(2)
    pool.step(10)
    mixed = [_state(pool, k) for k in range(2)]
    assert all(o["status"] == 0 for o in pool.observables()[:2])
    pool.close()
    # the stopped state is the state right after the overflowing rebuild:
    # the same replica alone, advanced exactly that many steps, stops there too
    alone = pool_for([boom], "ds", nbr_capacity=cap)
    alone.step(int(steps[2]))
    st, sb = alone.poll()
    assert st[0] == steps[2] and sb[0] & mdx.MD_ST_LIST_OVERFLOW
    assert _same(_state(alone), stopped)
    alone.close()
    for k, s in enumerate(normal):
        ref = pool_for([s], "ds", nbr_capacity=cap)
        ref.step(210)
        assert _same(_state(ref), mixed[k]), k
        ref.close()


@pytest.mark.parametrize("prec", ["fp32", "ds"])
def test_overlapping_particles_stop_the_replica_and_spare_the_others(prec):
    """Two particles placed 1e-4 sigma apart: their first pair force
    overflows FP32, their positions become non-finite, and the replica stops
    with MD_ST_NONFINITE in its status; md_poll and md_observables report
    MD_E_NONFINITE, launching calls refuse until it is detached, and the
    other replica of the pool is bitwise what it is alone."""
    from paper_0912_3824_amd import mdx
    normal = I.make_ka(1500, 0.6, jitter=0.05, seed=52)
    bad = I.make_ka(1500, 0.6, jitter=0.05, seed=53)
    pos = bad.pos.copy()
    pos[0] = pos[1] + np.array([1e-4, 0.0, 0.0])
    bad.pos = pos
    pool = pool_for([normal, bad], prec)
    pool.step(20)
    steps, status = pool.poll()
    say("non-finite run:", prec, "steps", steps[:2].tolist(), "status", status[:2].tolist())
    assert status[1] & mdx.MD_ST_NONFINITE
    assert steps[1] < 20 and steps[0] == 20
    assert not (status[0] & 0xFF)
    with pytest.raises(mdx.MdError) as ei:
        pool.observables()
    assert ei.value.status == mdx.MD_E_NONFINITE
    with pytest.raises(mdx.MdError) as ei:
        pool.step(1)
    assert ei.value.status == mdx.MD_E_NONFINITE
    pool.detach(1)
    pool.step(5)
    mixed = _state(pool, 0)
    assert pool.observables()[0]["status"] == 0
    pool.close()
    ref = pool_for([normal], prec)
    ref.step(25)
    assert _same(_state(ref), mixed)
    ref.close()


def test_served_time_correlations_equal_alone_and_follow_the_oracle():
    """Jobs that ask for time-correlation functions (Sec. 2.5) while served
    in a continuously batched pool: each job's curves are bitwise the ones it
    computes alone, and a small job's curves match the oracle's blocking
    scheme on the oracle's own trajectory."""
    import math
    from oracle import oracle as O
    from oracle import tcf as OT
    from oracle.upload import state_after_upload
    from paper_0912_3824_amd.serve import Server
    jobs = I.serving_trace(6, rate_per_s=60.0, n_lo=500, n_hi=4000, steps_lo=150, steps_hi=400, seed=8,
                           tcf_fraction=1.0, tcf_every=10, tcf_levels=3, tcf_block=4)
    jobs[1].tcf_every = 0          # a job without correlations in the mix
    jobs[2].tcf_every = 7
    jobs[0].n = 500                # the one the oracle follows
    say("served tcf jobs", [(j.n, j.steps, j.tcf_every) for j in jobs])
    srv = Server(I.ka_table(), "ds", max_slots=3, max_particles=9000, chunk_steps=64,
                 make_system=lambda j: I.job_system(j))
    out = srv.run(jobs)
    srv.close()
    res = {r.job_id: r for r in out["results"]}
    assert not out["failed"] and len(res) == len(jobs)
    assert res[1].tcf is None
    for j in jobs:
        r = res[j.job_id]
        alone = pool_for([I.job_system(j)], "ds")
        if j.tcf_every:
            t = alone.tcf(0, j.tcf_levels, j.tcf_block, j.tcf_q)
            t.sample()
            done = 0
            while done + j.tcf_every <= j.steps:
                alone.step(j.tcf_every)
                done += j.tcf_every
                t.sample()
            if done < j.steps:
                alone.step(j.steps - done)
            lags, vals, terms = t.read()
            assert np.array_equal(lags, r.tcf["lags"]) and np.array_equal(terms, r.tcf["terms"])
            assert np.array_equal(vals, r.tcf["values"], equal_nan=True), j
        else:
            alone.step(j.steps)
        p, v, i = alone.get_state(0)
        assert np.array_equal(p, r.pos) and np.array_equal(v, r.vel) and np.array_equal(i, r.image), j
        alone.close()
    # the oracle's scheme on the oracle's trajectory for the smallest job
    j = jobs[0]
    s = I.job_system(j)
    p, v, img = state_after_upload(s.pos, s.vel, s.box, "ds")
    ref = OT.Blocking(j.tcf_levels, j.tcf_block, s.species, j.tcf_q)
    ref.sample(p + img * s.box, v)
    for _ in range(j.steps // j.tcf_every):
        p, v, di, _ = O.vv(p, v, s.box, s.species, s.table, s.dt, j.tcf_every)
        img = img + di
        ref.sample(p + img * s.box, v)
    rl, rv, rt = ref.result()
    got = res[j.job_id].tcf
    assert (got["terms"] == rt).all()
    ok = rt > 0
    err = np.abs(got["values"][ok] - rv[ok]) / (np.abs(rv[ok]) + 1e-3)
    say("served tcf vs oracle: max rel err", float(err.max()))
    assert err.max() < 1e-4
