"""md_thermostat_noalloc (the allocation-free form of md_thermostat, whose
chunk partial sums live in the library's static device array) against
md_thermostat through the C ABI: bitwise the same velocities, on two calls
in a row, the second on a smaller replica (so the scratch array holds the
first call's larger contents when the second runs)."""
import numpy as np
import pytest

import md_inputs as I
from gpu_helpers import pool_for, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["ds", "fp64"])
def test_noalloc_thermostat_equals_thermostat(prec):
    cases = [(I.make_ka(20000, 0.7, jitter=0.05, seed=51), 0.5, 7, 3),   # 5 chunks
             (I.make_ka(5003, 0.6, jitter=0.05, seed=52), 0.8, 11, 0)]   # 2 chunks, smaller
    for s, temp, seed, call in cases:
        say("noalloc thermostat", prec, "n", s.n, "T", temp)
        a = pool_for([s], prec)
        b = pool_for([s], prec)
        fa, _ = a.forces(0)          # fills a's scratch rows; the noalloc call must not touch them
        fb, _ = b.forces(0)
        a.thermostat(0, temp, seed, call)
        b.thermostat_noalloc(0, temp, seed, call)
        pa, va, ia = a.get_state(0)
        pb, vb, ib = b.get_state(0)
        assert np.array_equal(va, vb) and np.array_equal(pa, pb) and np.array_equal(ia, ib)
        o = b.observables()[0]
        assert o["temperature"] == pytest.approx(temp, rel=1e-12 if prec == "fp64" else 1e-6)
        # both pools then step identically
        a.step(20)
        b.step(20)
        assert all(np.array_equal(x, y) for x, y in zip(a.get_state(0), b.get_state(0)))
        a.close()
        b.close()


def test_noalloc_thermostat_rejects_what_exceeds_its_scratch():
    from paper_0912_3824_amd import mdx
    s = I.make_ka(3000, 0.7, seed=53)
    pool = pool_for([s], "ds")
    with pytest.raises(mdx.MdError) as ei:
        pool.thermostat_noalloc(0, -1.0, 1, 0)
    assert ei.value.status == -1
    pool.close()
