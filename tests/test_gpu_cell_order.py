"""Particle sort along a space-filling cell order (Sec. 2.2 reorders
particles along a Hilbert curve): Morton and Hilbert cell orders give the
same Verlet lists as sets, the same physics within the parity tolerances,
and stay deterministic (launch-shape independent, batched = alone)."""
import numpy as np
import pytest

import md_inputs as I
from oracle import oracle as O
from oracle.upload import state_after_upload
from gpu_helpers import near_cutoff, pool_for, say

pytestmark = pytest.mark.gpu


def _ka(n, T=0.7, seed=11, jitter=0.06):
    return I.make_ka(n, T, jitter=jitter, seed=seed)


@pytest.mark.parametrize("order", ["morton", "hilbert"])
@pytest.mark.parametrize("prec,n", [("fp32", 3001), ("ds", 12007), ("fp64", 3001), ("ds", 60000)])
def test_lists_match_oracle(order, prec, n):
    s = _ka(n)
    say("curve lists", order, prec, n)
    pool = pool_for([s], prec, cell_order=order)
    pos, vel, img = state_after_upload(s.pos, s.vel, s.box, prec)
    cnt, ids = pool.neighbours(0, cap=256)
    ref = O.neighbours(pos, s.box, s.species, s.table, s.skin)
    amb = near_cutoff(pos, s.box, s.species, s.table, lambda a, b: s.table.rcut[a, b] + s.skin, band=1e-6)
    bad = 0
    for i in range(n):
        got = set(ids[i, :cnt[i]].tolist())
        if got != set(ref[i].tolist()):
            assert amb[i], (i, sorted(got ^ set(ref[i].tolist())))
            bad += 1
        assert len(got) == cnt[i]
    assert bad <= max(1, n // 10000)
    pool.close()


@pytest.mark.parametrize("prec", ["ds", "fp64"])
def test_orders_give_the_same_list_sets(prec):
    s = _ka(12007)
    sets = {}
    for order in ("row", "morton", "hilbert"):
        pool = pool_for([s], prec, cell_order=order)
        cnt, ids = pool.neighbours(0, cap=256)
        sets[order] = [frozenset(ids[i, :cnt[i]].tolist()) for i in range(s.n)]
        pool.close()
    assert sets["morton"] == sets["row"]
    assert sets["hilbert"] == sets["row"]


@pytest.mark.parametrize("prec", ["ds", "fp64"])
def test_ten_steps_and_rebuilds_match_oracle(prec):
    s = _ka(1500, T=1.0, jitter=0.1, seed=4)
    pool = pool_for([s], prec, cell_order="hilbert")
    p0, v0, i0 = state_after_upload(s.pos, s.vel, s.box, prec)
    pool.step(300)
    obs = pool.observables()[0]
    p1, v1, i1 = pool.get_state(0)
    pr, vr, ir, _ = O.vv(p0, v0, s.box, s.species, s.table, s.dt, 300)
    d = np.abs((p1 + i1 * s.box) - (pr + (ir + i0) * s.box)).max()
    say("hilbert 300-step", prec, "rebuilds", obs["n_rebuilds"], "max|dr|", d)
    assert obs["n_rebuilds"] >= 3 and obs["status"] == 0
    assert d < (1e-8 if prec == "fp64" else 1e-4)
    pool.close()


def test_curve_order_is_deterministic():
    """Lists entry by entry across list-build shapes, and a replica batched
    with others equals the replica alone, bit for bit."""
    s = _ka(12007)
    pool = pool_for([s], "ds", cell_order="hilbert")
    ref = None
    for lanes, block, width in [(1, 256, 4), (8, 1024, 2), (0, 512, 8), (0, 64, 1)]:
        pool.set_launch(build_lanes=lanes, build_block=block, build_width=width)
        pool.rebuild_neighbours()
        cnt, ids = pool.neighbours(0, cap=256)
        if ref is None:
            ref = (cnt, ids)
        assert np.array_equal(cnt, ref[0]) and np.array_equal(ids, ref[1]), (lanes, block, width)
    pool.close()
    reps = [_ka(n, seed=60 + k) for k, n in enumerate((900, 4001, 12007))]
    batch = pool_for(reps, "ds", cell_order="hilbert")
    batch.step(200)
    got = [batch.get_state(k) for k in range(3)]
    batch.close()
    for k, r in enumerate(reps):
        alone = pool_for([r], "ds", cell_order="hilbert")
        alone.step(200)
        p, v, i = alone.get_state(0)
        alone.close()
        assert np.array_equal(p, got[k][0]) and np.array_equal(v, got[k][1]), k
