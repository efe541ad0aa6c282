"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Inputs are seeded KA / LJ systems (fcc-subset starts with a small jitter so
that no lattice shell sits on a cutoff).  The oracle receives the state the
device starts from, derived on the host from the seeded input by the upload
rule (oracle/upload.py: folded into the box, rounded to the precision
mode's representation), so the comparison isolates the device arithmetic;
nothing read back from the device is ever fed to the oracle.  Sizes span several cells per edge, several workgroups
and a ragged tail (N not a multiple of the block size)."""
import dataclasses
import functools
import math

import numpy as np
import pytest

import md_inputs as I
from oracle import oracle as O
from oracle.upload import state_after_upload
from gpu_helpers import (BAND, TOL_E, TOL_F, cutoff_jump, force_error, near_cutoff,
                         pool_for, say)

pytestmark = pytest.mark.gpu
PRECS = ["fp32", "ds", "mixed64", "fp64"]


def _ka(n, T=0.7, seed=11, jitter=0.06):
    return I.make_ka(n, T, jitter=jitter, seed=seed)


@pytest.mark.parametrize("prec", PRECS)
def test_uploaded_state_follows_the_upload_rule(prec):
    """md_attach stores exactly the state the upload rule defines (positions
    folded into the box, FP32 / double-single / double representation), which
    is what the oracle is given as the device's starting state."""
    s = _ka(3001)
    pool = pool_for([s], prec)
    p, v, i = pool.get_state(0)
    pr, vr, ir = state_after_upload(s.pos, s.vel, s.box, prec)
    dp = np.abs(p - pr)
    dp = np.minimum(dp, np.abs(dp - s.box))  # a value rounded up to L is stored as 0
    say("upload", prec, "max|dx|", dp.max(), "max|dv|", np.abs(v - vr).max())
    assert dp.max() == 0.0
    assert np.array_equal(v, vr)
    assert np.array_equal(p + i * s.box, pr + ir * s.box) or dp.max() == 0.0
    pool.close()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,lpp", [(500, 0), (3001, 1), (3001, 4), (12007, 0)])
def test_forces_match_oracle(prec, n, lpp):
    s = _ka(n)
    say("forces", prec, n, "lanes", lpp)
    pool = pool_for([s], prec, lanes_per_particle=lpp)
    pos, vel, img = state_after_upload(s.pos, s.vel, s.box, prec)
    f, e = pool.forces(0)
    fr, er, wr = O.forces(pos, s.box, s.species, s.table)
    excl = None
    if prec != "fp64":
        excl = near_cutoff(pos, s.box, s.species, s.table, lambda a, b: s.table.rcut[a, b])
    err, frms = force_error(f, fr, excl)
    say("  e_F", err, "F_rms", frms, "excluded", 0 if excl is None else int(excl.sum()))
    assert err < TOL_F[prec]
    assert abs(e.sum() - er.sum()) <= TOL_E[prec] * abs(er.sum())
    if excl is not None and excl.any():  # one cutoff jump at most
        assert np.abs(f - fr)[excl].max() < 2 * cutoff_jump(s.table) + TOL_F[prec] * frms
    pool.close()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,width,lanes", [(500, 4, 0), (500, 4, 1), (3001, 1, 0), (3001, 4, 1),
                                           (3001, 4, 64), (12007, 2, 0), (12007, 8, 1), (12007, 8, 2)])
def test_neighbour_lists_match_oracle(prec, n, width, lanes):
    s = _ka(n)
    say("lists", prec, n, "width", width, "lanes", lanes)
    pool = pool_for([s], prec)
    if (width, lanes) != (4, 0):
        pool.set_launch(build_width=width, build_lanes=lanes)
        pool.rebuild_neighbours()
    pos, vel, img = state_after_upload(s.pos, s.vel, s.box, prec)
    cnt, ids = pool.neighbours(0, cap=256)
    ref = O.neighbours(pos, s.box, s.species, s.table, s.skin)
    amb = near_cutoff(pos, s.box, s.species, s.table,
                      lambda a, b: s.table.rcut[a, b] + s.skin, band=1e-6)
    bad = 0
    for i in range(n):
        got = set(ids[i, :cnt[i]].tolist())
        if got != set(ref[i].tolist()):
            assert amb[i], (i, sorted(got ^ set(ref[i].tolist())))
            bad += 1
        assert len(got) == cnt[i]  # no duplicates
    say("  ambiguous-band particles differing:", bad)
    assert bad <= max(1, n // 10000)
    pool.close()


@pytest.mark.parametrize("prec,n", [("ds", 500), ("ds", 3001), ("ds", 12007), ("ds", 60000),
                                    ("fp64", 500), ("fp64", 3001), ("fp64", 12007)])
def test_list_build_lanes_give_identical_lists(prec, n):
    """One lane per member and groups of 2..64 lanes per member, with row
    segments built by one or several work items (several block sizes and
    row widths), build the same lists, entry by entry."""
    s = _ka(n)
    pool = pool_for([s], prec)
    ref = None
    for lanes, block, width, split in [(1, 256, 4, 0), (2, 256, 4, 0), (4, 512, 1, 0), (8, 1024, 2, 0),
                                       (16, 256, 8, 0), (32, 64, 4, 0), (64, 1024, 4, 0), (0, 512, 8, 0),
                                       (0, 64, 1, 0), (0, 512, 8, 1), (16, 512, 4, 3), (0, 256, 2, 256), (0, 320, 10, 0),
                                       (2, 320, 16, 0)]:
        pool.set_launch(build_lanes=lanes, build_block=block, build_width=width, build_split=split)
        pool.rebuild_neighbours()
        cnt, ids = pool.neighbours(0, cap=256)
        say("lanes", prec, n, lanes, block, width, split, "entries", int(cnt.sum()))
        if ref is None:
            ref = (cnt, ids)
        assert np.array_equal(cnt, ref[0]) and np.array_equal(ids, ref[1]), (lanes, block, width, split)
    pool.close()


@pytest.mark.parametrize("prec", ["fp32", "ds", "fp64"])
def test_lists_do_not_depend_on_lanes_per_particle(prec):
    """The entries of a list are dealt to the lanes of its particle in turn,
    so where an entry is stored depends on the lanes per particle (1, 2 or
    4); read back in the canonical order, the lists are the same entry by
    entry for every lane count, from the one-lane and the grouped-lane
    build."""
    s = _ka(3001)
    ref = None
    for lpp in (1, 2, 4):
        pool = pool_for([s], prec, lanes_per_particle=lpp)
        for lanes in (1, 8):
            pool.set_launch(build_lanes=lanes)
            pool.rebuild_neighbours()
            cnt, ids = pool.neighbours(0, cap=256)
            say("lists", prec, "lanes per particle", lpp, "build lanes", lanes, "entries", int(cnt.sum()))
            if ref is None:
                ref = (cnt, ids)
            assert np.array_equal(cnt, ref[0]) and np.array_equal(ids, ref[1]), (lpp, lanes)
        pool.close()


@pytest.mark.parametrize("prec", ["fp32", "ds", "mixed64"])
def test_list_build_with_large_cells(prec):
    """Cells of ~88 members (skin 1.5, list radius 4.0): more members per
    cell than a wave has lanes, and more candidates per cell than one
    acceptance mask holds.  The one-lane build (one work item per one-cell
    row segment) and the grouped-lane builds give the same lists entry by
    entry, and they equal the oracle's brute-force neighbour sets for a
    sample."""
    n = 30000
    s = I.make_ka(n, 0.7, jitter=0.06, seed=13, skin=1.5)
    pool = pool_for([s], prec)
    ref = None
    # width 1: 7 x 7 x 7 one-cell segments, at least 256, so one work item
    # per segment; lanes 1 -> one lane per member, lanes 16 / 0 -> groups
    for lanes, block, width in [(1, 256, 1), (16, 512, 1), (1, 1024, 1), (0, 256, 8)]:
        pool.set_launch(build_lanes=lanes, build_block=block, build_width=width, build_split=0)
        pool.rebuild_neighbours()
        cnt, ids = pool.neighbours(0, cap=512)
        say("large cells", prec, lanes, block, width, "mean list", float(cnt.mean()))
        if ref is None:
            ref = (cnt, ids)
        assert np.array_equal(cnt, ref[0]) and np.array_equal(ids, ref[1]), (lanes, block, width)
    assert pool.observables()[0]["status"] == 0
    pos, vel, img = state_after_upload(s.pos, s.vel, s.box, prec)
    sel = np.sort(np.random.default_rng(3).choice(n, size=200, replace=False)).astype(np.int32)
    want = O.neighbours(pos, s.box, s.species, s.table, s.skin, sel)
    amb = near_cutoff(pos, s.box, s.species, s.table, lambda a, b: s.table.rcut[a, b] + s.skin, band=1e-6)
    for k, i in enumerate(sel):
        got = set(ref[1][i, :ref[0][i]].tolist())
        assert got == set(want[k].tolist()) or amb[i], int(i)
    pool.close()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("lpp", [1, 2, 4])
def test_ten_step_trajectory(prec, lpp):
    s = _ka(3001, T=0.7)
    say("10-step", prec, "lanes", lpp)
    pool = pool_for([s], prec, lanes_per_particle=lpp)
    p0, v0, i0 = state_after_upload(s.pos, s.vel, s.box, prec)
    pool.step(10)
    p1, v1, i1 = pool.get_state(0)
    pr, vr, ir, _ = O.vv(p0, v0, s.box, s.species, s.table, s.dt, 10)
    d = (p1 + i1 * s.box) - (pr + (ir + i0) * s.box)
    dv = np.abs(v1 - vr).max()
    say("  max|dr|", np.abs(d).max(), "max|dv|", dv)
    tol = 1e-9 if prec == "fp64" else 1e-4
    assert np.abs(d).max() < tol
    assert dv < tol
    pool.close()


@pytest.mark.parametrize("prec", ["fp32", "ds"])
def test_box_that_is_not_a_float(prec):
    """A box edge with no float32 representation (L = (N/rho)^(1/3) in
    double): forces at the uploaded state, then 5 steps, a forced re-sort
    (which folds the particles that crossed a face back into the box by the
    exact edge), and 5 more steps, against the oracle's 10 steps."""
    s = I.make_ka(3001, 0.7, jitter=0.06, seed=21, float32_box=False)
    assert float(np.float32(s.box)) != s.box
    # move the lattice planes that sit a quarter cell inside the faces onto
    # the faces, so that particles cross them within the ten steps
    a = s.box / math.ceil((s.n / 4.0) ** (1.0 / 3.0) - 1e-9)
    s = dataclasses.replace(s, pos=np.mod(s.pos - 0.25 * a, s.box))
    say("non-float box", prec, repr(s.box))
    pool = pool_for([s], prec)
    pos, vel, img = state_after_upload(s.pos, s.vel, s.box, prec)
    f, e = pool.forces(0)
    fr, er, _ = O.forces(pos, s.box, s.species, s.table)
    excl = near_cutoff(pos, s.box, s.species, s.table, lambda a, b: s.table.rcut[a, b])
    err, frms = force_error(f, fr, excl)
    say("  e_F", err, "excluded", int(excl.sum()))
    assert err < TOL_F[prec]
    pool.step(5)
    pool.rebuild_neighbours()
    pool.step(5)
    p1, v1, i1 = pool.get_state(0)
    pr, vr, ir, _ = O.vv(pos, vel, s.box, s.species, s.table, s.dt, 10)
    d = np.abs((p1 + i1 * s.box) - (pr + (ir + img) * s.box)).max()
    dv = np.abs(v1 - vr).max()
    crossed = int(np.count_nonzero(i1 != img))
    say("  10 steps: max|dr|", d, "max|dv|", dv, "face crossings", crossed)
    assert crossed > 0
    assert d < 1e-4 and dv < 1e-4
    assert np.all((p1 >= 0) & (p1 < s.box))
    pool.close()


@pytest.mark.parametrize("prec", ["ds", "fp64"])
def test_long_run_with_rebuilds(prec):
    """300 steps from a jittered lattice (several list rebuilds and cell
    re-sorts) against the oracle's brute-force integrator."""
    s = _ka(1500, T=1.0, jitter=0.1, seed=4)
    say("300-step", prec)
    pool = pool_for([s], prec)
    p0, v0, i0 = state_after_upload(s.pos, s.vel, s.box, prec)
    pool.step(300)
    obs = pool.observables()[0]
    p1, v1, i1 = pool.get_state(0)
    pr, vr, ir, _ = O.vv(p0, v0, s.box, s.species, s.table, s.dt, 300)
    d = np.abs((p1 + i1 * s.box) - (pr + (ir + i0) * s.box)).max()
    say("  rebuilds", obs["n_rebuilds"], "max|dr|", d)
    assert obs["n_rebuilds"] >= 3
    assert obs["step"] == 300 and obs["status"] == 0
    assert d < (1e-8 if prec == "fp64" else 1e-4)
    pool.close()


@pytest.mark.parametrize("prec", PRECS)
def test_observables_match_oracle(prec):
    s = _ka(3001, T=0.7)
    say("observables", prec)
    pool = pool_for([s], prec)
    # at the uploaded state: the same positions and velocities on both sides
    o = pool.observables()[0]
    p0, v0, _ = state_after_upload(s.pos, s.vel, s.box, prec)
    r = O.observables(p0, v0, s.box, s.species, s.table)
    tol = TOL_E[prec]
    for k in ("epot", "virial"):
        assert o[k] == pytest.approx(r[k], rel=tol), k
    assert o["ekin"] == pytest.approx(r["ekin"], rel=1e-12)
    assert np.abs(o["momentum"] - r["momentum"]).max() < 1e-9
    assert o["pressure"] == pytest.approx(r["pressure"], rel=tol * 10)
    # five steps later, against the oracle's trajectory from the same start
    pool.step(5)
    o5 = pool.observables()[0]
    pos, vel, _, _ = O.vv(p0, v0, s.box, s.species, s.table, s.dt, 5)
    r5 = O.observables(pos, vel, s.box, s.species, s.table)
    t5 = 1e-10 if prec == "fp64" else 1e-6
    for k in ("epot", "ekin", "etot", "virial"):
        assert o5[k] == pytest.approx(r5[k], rel=t5), k
    pool.close()


def test_lj_fp64_1000_steps():
    """Single-species LJ, N = 4000 on an fcc lattice, rho 0.8442, T 1.5, FP64
    plain path: 1000 steps against the oracle."""
    s = I.make_lj(4000)
    say("lj4000 fp64 1000 steps")
    pool = pool_for([s], "fp64")
    p0, v0, i0 = state_after_upload(s.pos, s.vel, s.box, "fp64")
    o0 = pool.observables()[0]
    pool.step(1000)
    o1 = pool.observables()[0]
    p1, v1, i1 = pool.get_state(0)
    pr, vr, ir, _ = O.vv(p0, v0, s.box, s.species, s.table, s.dt, 1000)
    d = np.abs((p1 + i1 * s.box) - (pr + (ir + i0) * s.box)).max()
    say("  max|dr|", d, "dE", o1["etot"] - o0["etot"])
    assert d < 1e-6
    assert abs(o1["etot"] - o0["etot"]) < 1e-3 * abs(o0["etot"])
    pool.close()


# ------------------------------------------- WCA and C2 smoothing (Sec. 4)
@functools.lru_cache(maxsize=1)
def _smooth_systems():
    lj = I.make_lj(4000, rho=0.75, temperature=1.12, jitter=0.05, seed=31)
    # On the fcc lattice at rho = 0.75 nearest neighbours (1.235 sigma) lie
    # beyond the WCA cutoff.  The WCA input is a fluid-like state instead:
    # a jittered lattice advanced 100 steps by the oracle's own integrator
    # (F_rms ~ 14, largest force ~ 7 F_rms; no input comes from the device).
    w0 = I.make_lj(4000, rho=0.75, temperature=1.12, jitter=0.12, seed=32, rc=I.WCA_RC)
    p, v, _, _ = O.vv(w0.pos, w0.vel, w0.box, w0.species, w0.table, 0.002, 100)
    wca = dataclasses.replace(w0, pos=p, vel=v)
    ka = _ka(3001)
    return {"lj_h0.005": I.smoothed(lj, 0.005), "lj_h0.05": I.smoothed(lj, 0.05),
            "wca": wca, "wca_h0.005": I.smoothed(wca, 0.005), "ka_h0.01": I.smoothed(ka, 0.01)}


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["lj_h0.005", "lj_h0.05", "wca", "wca_h0.005", "ka_h0.01"])
def test_smoothed_and_wca_forces_match_oracle(prec, name):
    """Forces, energy and virial of the smoothed and WCA potentials.  Their
    force is continuous at the cutoff, so every particle is held to the
    tolerance (no cutoff band is set aside)."""
    s = _smooth_systems()[name]
    say("smoothed forces", prec, name, "h", s.table.smooth)
    pool = pool_for([s], prec)
    pos, vel, img = state_after_upload(s.pos, s.vel, s.box, prec)
    f, e = pool.forces(0)
    fr, er, wr = O.forces(pos, s.box, s.species, s.table)
    err, frms = force_error(f, fr, None)
    say("  e_F", err, "F_rms", frms)
    assert err < TOL_F[prec]
    assert abs(e.sum() - er.sum()) <= TOL_E[prec] * abs(er.sum())
    o = pool.observables()[0]
    assert o["virial"] == pytest.approx(wr.sum(), rel=TOL_E[prec], abs=TOL_E[prec] * np.abs(wr).sum())
    pool.close()


@pytest.mark.parametrize("prec", ["ds", "fp64"])
@pytest.mark.parametrize("name", ["lj_h0.005", "wca_h0.005"])
def test_smoothed_ten_step_trajectory(prec, name):
    s = _smooth_systems()[name]
    say("smoothed 10-step", prec, name)
    pool = pool_for([s], prec)
    p0, v0, i0 = state_after_upload(s.pos, s.vel, s.box, prec)
    pool.step(10)
    p1, v1, i1 = pool.get_state(0)
    pr, vr, ir, _ = O.vv(p0, v0, s.box, s.species, s.table, s.dt, 10)
    d = (p1 + i1 * s.box) - (pr + (ir + i0) * s.box)
    tol = 1e-9 if prec == "fp64" else 1e-4
    assert np.abs(d).max() < tol
    assert np.abs(v1 - vr).max() < tol
    pool.close()
