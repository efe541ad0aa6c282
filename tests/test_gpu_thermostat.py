"""The modified Andersen thermostat with the leap-frogged rand48 generator
(Sec. 2.3) on the GPU, through the C ABI, against the oracle."""
import numpy as np
import pytest

import md_inputs as I
from gpu_helpers import pool_for, say
from oracle import thermostat as OT

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,rtol", [("fp64", 1e-12), ("ds", 1e-12), ("mixed64", 1e-12), ("fp32", 3e-7)])
def test_thermostat_velocities_match_oracle(prec, rtol):
    s = I.make_ka(3001, 0.9, jitter=0.05, seed=41)
    pool = pool_for([s], prec)
    pool.thermostat(0, 0.45, seed=1234567, call=5)
    _, vel, _ = pool.get_state(0)
    ref = OT.andersen(s.n, 0.45, seed=1234567, call=5)
    err = np.abs(vel - ref).max() / np.abs(ref).max()
    say("thermostat", prec, "max rel err", err)
    assert err < rtol
    o = pool.observables()[0]
    assert o["temperature"] == pytest.approx(0.45, rel=max(rtol, 1e-12) * 10)
    assert np.abs(o["momentum"]).max() < (1e-9 * s.n if prec != "fp32" else 1e-3)
    pool.close()


def test_thermostat_draws_do_not_depend_on_the_pool():
    """The draws depend on (seed, call, particle id) only: a replica in a
    batch of three gets bitwise the velocities it gets alone."""
    reps = [I.make_ka(n, 0.7, jitter=0.05, seed=50 + k) for k, n in enumerate((700, 1501, 2402))]
    pool = pool_for(reps, "ds")
    for k in range(3):
        pool.thermostat(k, 0.6, seed=99, call=k + 1)
    batched = [pool.get_state(k)[1].copy() for k in range(3)]
    pool.close()
    for k, s in enumerate(reps):
        alone = pool_for([s], "ds")
        alone.thermostat(0, 0.6, seed=99, call=k + 1)
        assert np.array_equal(alone.get_state(0)[1], batched[k]), k
        alone.close()


def test_heat_bath_cools_to_its_temperature():
    s = I.make_ka(4000, 1.2, jitter=0.05, seed=43)
    pool = pool_for([s], "ds")
    nxt = pool.andersen(0, 0.5, mu=1.0, steps=3000, seed=7)
    assert nxt == 3
    ts = []
    for _ in range(5):
        pool.step(100)
        ts.append(pool.observables()[0]["temperature"])
    say("after the bath", ts)
    assert abs(np.mean(ts) - 0.5) < 0.1
    pool.close()
