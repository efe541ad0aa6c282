"""Pins of the oracle's cell-list route (Sec. 2.2: cell binning, Verlet lists
with a skin, rebuild when a particle has moved more than skin/2) against the
brute-force functions, which are themselves pinned in test_oracle_pins.py.

The two routes share the pair term and the minimum image but find the
partners differently (all j, against the 27 cells around i; or a Verlet list
rebuilt on the displacement criterion), so a wrong cell index, a missed
neighbour cell, a wrong list radius or a missing rebuild makes them differ
by far more than the reordering of the FP64 sums (~1e-15).
"""
import numpy as np
import pytest

import md_inputs as I
from oracle import oracle as O

# (label, system): KA at rho = 1.2 and LJ at rho = 0.8442, with 3 and >= 5
# cells per edge, one box below three cells (one cell: all pairs), and the
# smoothed and WCA pair kinds of Sec. 4.
CASES = [
    ("ka875_3cells", lambda: I.make_ka(875, 0.7, jitter=0.05, seed=3)),
    ("ka4000_5cells", lambda: I.make_ka(4000, 0.7, jitter=0.05, seed=4)),
    ("lj615_3cells", lambda: I.make_lj(615, seed=3, jitter=0.05)),
    ("lj4000_6cells", lambda: I.make_lj(4000, seed=5, jitter=0.05)),
    ("ka300_1cell", lambda: I.make_ka(300, 0.7, jitter=0.05, seed=6)),
    ("lj2000_smooth", lambda: I.smoothed(I.make_lj(2000, seed=7, jitter=0.05), 0.005)),
    ("wca2000", lambda: I.System(**{**I.make_lj(2000, rho=0.75, seed=8, jitter=0.05).__dict__,
                                     "table": I.lj_table(I.WCA_RC)})),
]


def _cells_per_edge(s):
    return int(s.box // s.table.max_rcut())


@pytest.mark.parametrize("label,make", CASES, ids=[c[0] for c in CASES])
def test_cell_list_forces_equal_brute_force(label, make):
    s = make()
    f, e, w = O.forces(s.pos, s.box, s.species, s.table)
    fc, ec, wc = O.forces_cells(s.pos, s.box, s.species, s.table)
    frms = float(np.sqrt(np.mean(f * f)))
    assert float(np.abs(fc - f).max()) <= 1e-13 * frms
    assert float(np.abs(ec - e).max()) <= 1e-13 * float(np.abs(e).max())
    assert float(np.abs(wc - w).max()) <= 1e-13 * float(np.abs(w).max())
    if label.endswith("3cells"):
        assert _cells_per_edge(s) == 3
    if label.endswith("1cell"):
        assert _cells_per_edge(s) < 3


def test_cell_list_forces_equal_brute_force_at_64k():
    """The largest size the brute-force route finishes in seconds."""
    s = I.make_ka(64000, 0.7, jitter=0.05, seed=5)
    assert _cells_per_edge(s) >= 5
    rng = np.random.default_rng(11)
    sel = np.sort(rng.choice(s.n, size=4000, replace=False)).astype(np.int32)
    f, e, w = O.forces(s.pos, s.box, s.species, s.table, sel)
    fc, ec, wc = O.forces_cells(s.pos, s.box, s.species, s.table)
    frms = float(np.sqrt(np.mean(f * f)))
    assert float(np.abs(fc[sel] - f).max()) <= 1e-13 * frms
    assert float(np.abs(ec[sel] - e).max()) <= 1e-13 * float(np.abs(e).max())


def test_cell_list_forces_are_translation_invariant():
    """Shifting every particle (and so the cell each lands in) by a fraction
    of a cell leaves every force unchanged."""
    s = I.make_ka(4000, 0.7, jitter=0.05, seed=12)
    f, _, _ = O.forces_cells(s.pos, s.box, s.species, s.table)
    g, _, _ = O.forces_cells(np.mod(s.pos + np.array([1.37, -0.61, 2.9]), s.box), s.box, s.species,
                             s.table)
    assert float(np.abs(f - g).max()) <= 1e-12 * float(np.sqrt(np.mean(f * f)))


@pytest.mark.parametrize("label,make,steps", [
    ("ka1500", lambda: I.make_ka(1500, 0.7, jitter=0.05, seed=3), 300),
    ("lj2000", lambda: I.make_lj(2000, seed=3, jitter=0.05), 200),
])
def test_verlet_list_trajectory_equals_brute_force(label, make, steps):
    """Velocity Verlet over skin-padded Verlet lists, rebuilt on the skin/2
    displacement criterion, follows the brute-force trajectory (differences
    only from the order of the FP64 sums).  Enough steps for several
    rebuilds: a missed rebuild would leave pairs that entered the cutoff
    out of the force."""
    s = make()
    p, v, im, f = O.vv(s.pos, s.vel, s.box, s.species, s.table, s.dt, steps)
    p2, v2, im2, f2, builds = O.vv_lists(s.pos, s.vel, s.box, s.species, s.table, s.dt, steps,
                                         s.skin)
    assert builds >= 3
    dr = float(np.abs((p + im * s.box) - (p2 + im2 * s.box)).max())
    dv = float(np.abs(v - v2).max())
    assert dr <= 1e-11 and dv <= 1e-10
    assert float(np.abs(f - f2).max()) <= 1e-10


def test_skin_changes_rebuilds_but_not_the_trajectory():
    """The skin is a performance knob: a smaller skin rebuilds more often,
    and every skin gives the same trajectory up to the order of the sums."""
    s = I.make_ka(1500, 0.7, jitter=0.05, seed=3)
    runs = [O.vv_lists(s.pos, s.vel, s.box, s.species, s.table, s.dt, 200, skin)
            for skin in (0.5, 0.3, 0.1)]
    builds = [r[4] for r in runs]
    assert builds[0] < builds[1] < builds[2]
    for r in runs[1:]:
        assert float(np.abs((r[0] + r[2] * s.box) - (runs[0][0] + runs[0][2] * s.box)).max()) <= 1e-11
