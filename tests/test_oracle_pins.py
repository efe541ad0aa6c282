"""Pins of the FP64 oracle against facts that do not come from the oracle:
closed forms of the 12-6 potential, symmetry and conservation laws, finite
differences, a lattice sum from an independent integer-lattice enumeration,
and scipy's periodic kd-tree for neighbour-list membership.

Each test names the mistake it is there to catch (dropped term, sign, index,
minimum-image error, wrong factor).
"""
import math
import os

import numpy as np
import pytest

import md_inputs as I
from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RMIN = 2.0 ** (1.0 / 6.0)


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_ka_table_matches_paper_values():
    """The KA pair table (Sec. 5) used by both sides equals the printed one."""
    t = I.ka_table()
    idx = {"AA": (0, 0), "AB": (0, 1), "BB": (1, 1)}
    for name, sig, eps in _read_golden("ka_pair_table.txt"):
        a, b = idx[name]
        assert t.sigma[a, b] == float(sig) and t.sigma[b, a] == float(sig)
        assert t.eps[a, b] == float(eps) and t.eps[b, a] == float(eps)
        assert t.rcut[a, b] == pytest.approx(2.5 * float(sig), rel=0, abs=1e-15)


def test_lj_setup_matches_paper_values():
    kv = {k: float(v) for k, v in _read_golden("lj_benchmark_setup.txt")}
    assert I.lj_table().rcut[0, 0] == kv["rc"]
    s = I.make_lj(500)
    assert s.dt == kv["dt"]


@pytest.mark.parametrize("eps,sig", [(1.0, 1.0), (1.5, 0.8), (0.5, 0.88)])
def test_pair_closed_forms(eps, sig):
    """Zero crossing at sigma, minimum -eps at 2^(1/6) sigma with zero force,
    |F(sigma)| = 24 eps / sigma repulsive; catches a wrong exponent, factor or
    sign in the pair term."""
    rc = 2.5 * sig
    v_sig, f_sig = O.pair(sig, eps, sig, rc)
    v_min, f_min = O.pair(RMIN * sig, eps, sig, rc)
    assert v_sig - v_min == pytest.approx(eps, rel=1e-14)   # shift cancels
    assert f_sig == pytest.approx(24.0 * eps / sig, rel=1e-14)
    assert abs(f_min) < 1e-13 * eps / sig
    # truncation: zero at and beyond rc; the shifted energy is continuous at rc
    assert O.pair(rc, eps, sig, rc) == (0.0, 0.0)
    assert O.pair(rc * 1.3, eps, sig, rc) == (0.0, 0.0)
    v_in, f_in = O.pair(rc * (1 - 1e-10), eps, sig, rc)
    assert abs(v_in) < 1e-9 * eps
    assert f_in < 0.0   # attractive just inside the cutoff (force not shifted)


def test_force_is_minus_dv_dr():
    """F(r) = -dV/dr by 4th-order central differences at random separations."""
    rng = np.random.default_rng(1)
    for eps, sig in [(1.0, 1.0), (1.5, 0.8), (0.5, 0.88)]:
        for r in rng.uniform(0.85 * sig, 2.45 * sig, 20):
            h = 1e-4
            vs = [O.pair(r + k * h, eps, sig, 2.5 * sig)[0] for k in (-2, -1, 1, 2)]
            dv = (vs[0] - 8 * vs[1] + 8 * vs[2] - vs[3]) / (12 * h)
            f = O.pair(r, eps, sig, 2.5 * sig)[1]
            assert f == pytest.approx(-dv, rel=1e-7, abs=1e-9)


def _ka(n, rho=1.2, T=0.7, jitter=0.08, seed=3):
    return I.make_ka(n, T, rho=rho, jitter=jitter, seed=seed)


def test_newton_third_law_and_momentum():
    s = _ka(864)
    f, e, w = O.forces(s.pos, s.box, s.species, s.table)
    frms = math.sqrt(np.mean(f * f))
    assert np.abs(f.sum(axis=0)).max() < 1e-12 * frms * s.n


def test_two_particles_across_the_boundary():
    """A pair at distance sigma across the periodic face repels along the
    boundary-crossing direction; catches minimum-image sign errors."""
    L = 10.0
    pos = np.array([[0.2, 5.0, 5.0], [L - 0.8, 5.0, 5.0]])
    sp = np.zeros(2, dtype=np.int32)
    f, e, w = O.forces(pos, L, sp, I.lj_table())
    assert f[0, 0] == pytest.approx(24.0, rel=1e-13)
    assert f[1, 0] == pytest.approx(-24.0, rel=1e-13)
    assert np.abs(f[:, 1:]).max() == 0.0
    # same in y and z
    for c in (1, 2):
        p = np.full((2, 3), 5.0)
        p[0, c], p[1, c] = L - 0.3, 0.7
        f, _, _ = O.forces(p, L, sp, I.lj_table())
        assert f[0, c] == pytest.approx(-24.0, rel=1e-13)


def test_translation_and_permutation():
    s = _ka(500)
    f0, e0, w0 = O.forces(s.pos, s.box, s.species, s.table)
    shift = np.array([3.7, -11.2, 0.41])
    p = np.mod(s.pos + shift, s.box)
    f1, e1, _ = O.forces(p, s.box, s.species, s.table)
    frms = math.sqrt(np.mean(f0 * f0))
    assert np.abs(f1 - f0).max() < 1e-11 * frms
    assert e1.sum() == pytest.approx(e0.sum(), rel=1e-12)
    perm = np.random.default_rng(7).permutation(s.n)
    f2, e2, _ = O.forces(s.pos[perm], s.box, s.species[perm], s.table)
    assert np.abs(f2 - f0[perm]).max() < 1e-11 * frms


def test_forces_are_minus_energy_gradient():
    """F_i = -dE_pot/dr_i by central differences; catches dropped terms, a
    missing factor 1/2 in the energy or a sign error in the force."""
    s = _ka(300, rho=0.8, jitter=0.1)
    rng = np.random.default_rng(11)
    h = 1e-6
    f, _, _ = O.forces(s.pos, s.box, s.species, s.table)
    for _ in range(12):
        i = int(rng.integers(s.n))
        c = int(rng.integers(3))
        ep = []
        for sgn in (1, -1):
            p = s.pos.copy()
            p[i, c] += sgn * h
            ep.append(O.forces(p, s.box, s.species, s.table)[1].sum())
        g = (ep[0] - ep[1]) / (2 * h)
        assert f[i, c] == pytest.approx(-g, rel=2e-6, abs=2e-6)


def test_virial_is_minus_volume_derivative():
    """W = sum_{i<j} d.F = -dE/dlambda for a uniform dilation r -> lambda r,
    L -> lambda L; catches a wrong virial factor or sign."""
    s = _ka(400, rho=1.0, jitter=0.1)
    _, e, w = O.forces(s.pos, s.box, s.species, s.table)
    h = 1e-7
    ep = O.forces(s.pos * (1 + h), s.box * (1 + h), s.species, s.table)[1].sum()
    em = O.forces(s.pos * (1 - h), s.box * (1 - h), s.species, s.table)[1].sum()
    assert w.sum() == pytest.approx(-(ep - em) / (2 * h), rel=1e-5)


def _fcc_shells(rc, a):
    """Coordination numbers of the fcc lattice by enumerating integer lattice
    vectors (half-integer cube coordinates with even sum), independent of the
    oracle's box and minimum image."""
    kmax = int(math.ceil(2 * rc / a)) + 1
    shells = {}
    rng = range(-2 * kmax, 2 * kmax + 1)
    for x in rng:
        for y in rng:
            for z in rng:
                if (x + y + z) % 2 or (x, y, z) == (0, 0, 0):
                    continue
                r2 = (x * x + y * y + z * z) * (a / 2) ** 2
                if r2 < rc * rc:
                    key = x * x + y * y + z * z
                    shells[key] = shells.get(key, 0) + 1
    return shells


def test_perfect_fcc_lattice():
    """On a perfect fcc lattice every force vanishes by inversion symmetry and
    the energy per particle is the lattice sum over coordination shells."""
    n = 4 * 6 ** 3
    rho = 0.8442
    L = (n / rho) ** (1 / 3)
    pos = I.fcc_positions(n, L, None)
    sp = np.zeros(n, dtype=np.int32)
    t = I.lj_table()
    f, e, w = O.forces(pos, L, sp, t)
    assert np.abs(f).max() < 1e-11
    a = L / 6
    shells = _fcc_shells(2.5, a)
    assert shells[2] == 12 and shells[4] == 6 and shells[6] == 24  # fcc: 12, 6, 24, ...
    e_sum = 0.0
    for k2, z in shells.items():
        v, _ = O.pair(math.sqrt(k2) * a / 2, 1.0, 1.0, 2.5)
        e_sum += 0.5 * z * v
    assert e.mean() == pytest.approx(e_sum, rel=1e-12)
    assert np.ptp(e) < 1e-12


@pytest.mark.parametrize("n,rho,species", [(216, 0.1, 1), (300, 0.5, 1),
                                           (500, 0.8442, 1), (400, 1.2, 2),
                                           (1000, 1.2, 2), (256, 1.2, 2)])
def test_neighbour_lists_match_kdtree(n, rho, species):
    """List membership equals scipy's periodic kd-tree pair search."""
    from scipy.spatial import cKDTree
    skin = 0.3
    if species == 1:
        s = I.make_lj(n, rho=rho, jitter=0.15, seed=n)
    else:
        s = I.make_ka(n, 0.7, rho=rho, jitter=0.15, seed=n)
    rl = s.table.rcut + skin
    rmax = float(rl[: s.table.n_species, : s.table.n_species].max())
    assert s.box >= 2 * rmax
    tree = cKDTree(s.pos, boxsize=s.box)
    dm = tree.sparse_distance_matrix(tree, rmax, output_type="coo_matrix")
    sp = s.species if species == 2 else np.zeros(n, dtype=int)
    expect = [set() for _ in range(n)]
    for i, j, d in zip(dm.row, dm.col, dm.data):
        if i != j and d < rl[sp[i], sp[j]]:
            expect[i].add(int(j))
    got = O.neighbours(s.pos, s.box, s.species, s.table, skin)
    for i in range(n):
        assert set(got[i].tolist()) == expect[i]
        assert np.all(np.diff(got[i]) > 0)


def test_free_particles_move_linearly():
    """Non-interacting particles move on straight lines; wrapping and image
    counts are consistent with the unwrapped motion."""
    L = 20.0
    pos = np.array([[1.0, 1.0, 1.0], [11.0, 11.0, 11.0]])
    vel = np.array([[3.0, -2.0, 0.5], [-1.25, 4.0, -3.0]])
    sp = np.zeros(2, dtype=np.int32)
    dt, steps = 0.01, 1000
    p, v, img, _ = O.vv(pos, vel, L, sp, I.lj_table(), dt, steps)
    unwrapped = p + img * L
    assert np.allclose(unwrapped, pos + steps * dt * vel, rtol=0, atol=1e-10)
    assert np.array_equal(v, vel)
    assert np.all((p >= 0) & (p < L))


def test_time_reversibility():
    """n steps forward, reverse velocities, n steps back: the start returns."""
    s = _ka(256, T=0.7, jitter=0.05)
    n = 100
    p1, v1, img1, _ = O.vv(s.pos, s.vel, s.box, s.species, s.table, s.dt, n)
    p2, v2, img2, _ = O.vv(p1, -v1, s.box, s.species, s.table, s.dt, n)
    d = p2 + img2 * s.box - s.pos
    d -= s.box * np.rint(d / s.box)
    assert np.abs(d).max() < 1e-10
    assert np.abs(v2 + s.vel).max() < 1e-9


def test_momentum_conserved_by_integration():
    s = _ka(256, T=0.7, jitter=0.05)
    p, v, _, _ = O.vv(s.pos, s.vel, s.box, s.species, s.table, s.dt, 200)
    assert np.abs(v.sum(axis=0)).max() < 1e-11


def test_dimer_small_oscillation_period():
    """A dimer near the potential minimum oscillates with the harmonic period
    2 pi sqrt(mu/k), mu = m/2, k = V''(r_min) = 72 * 2^(-1/3) eps/sigma^2."""
    L = 12.0
    r0 = RMIN + 1e-3
    pos = np.array([[4.0, 6.0, 6.0], [4.0 + r0, 6.0, 6.0]])
    vel = np.zeros((2, 3))
    sp = np.zeros(2, dtype=np.int32)
    dt = 2e-4
    k = 72.0 * 2 ** (-1 / 3)
    period = 2 * math.pi * math.sqrt(0.5 / k)
    seps = []
    p, v = pos, vel
    nsteps = int(2.2 * period / dt)
    for _ in range(nsteps):
        p, v, img, _ = O.vv(p, v, L, sp, I.lj_table(), dt, 1)
        seps.append((p[1, 0] - p[0, 0]) - RMIN)
    seps = np.array(seps)
    crossings = np.where((seps[:-1] > 0) & (seps[1:] <= 0))[0]
    assert len(crossings) >= 2
    measured = (crossings[1] - crossings[0]) * dt
    assert measured == pytest.approx(period, rel=5e-3)


def test_energy_fluctuation_scales_with_dt_squared():
    """Velocity Verlet's energy error is second order (Sec. 4.3): halving dt
    quarters the fluctuation of E(t) - E(0) over a fixed time span."""
    s = I.make_lj(256, rho=0.8442, temperature=1.0, jitter=0.05, seed=5)
    span = 0.2
    amp = []
    for dt in (0.004, 0.002):
        p, v = s.pos, s.vel
        e0 = O.observables(p, v, s.box, s.species, s.table)["etot"]
        dev = 0.0
        nchunk = 10
        for _ in range(nchunk):
            p, v, _, _ = O.vv(p, v, s.box, s.species, s.table, dt, int(round(span / dt / nchunk)))
            dev = max(dev, abs(O.observables(p, v, s.box, s.species, s.table)["etot"] - e0))
        amp.append(dev)
    ratio = amp[0] / amp[1]
    assert 3.0 < ratio < 5.5, ratio


def test_generated_velocities_have_exact_temperature():
    s = I.make_ka(1000, 0.55, seed=9)
    T = float(np.sum(s.vel ** 2)) / (3 * s.n)
    assert T == pytest.approx(0.55, rel=1e-13)
    assert np.abs(s.vel.sum(axis=0)).max() < 1e-11
    assert int((s.species == 0).sum()) == 800


# ---------------------------------------------------------------- smoothing
# Sec. 4: the potential times g(x) = x^4 / (1 + x^4), x = (r - rc) / (h sigma).

def _lj_exact(r2, eps, sig):
    """4 eps [(sig^2/r^2)^6 - (sig^2/r^2)^3] in exact rationals."""
    from fractions import Fraction as Fr
    s2 = Fr(sig) ** 2 / r2
    return 4 * Fr(eps) * (s2 ** 6 - s2 ** 3)


@pytest.mark.parametrize("eps,sig,h", [(1.0, 1.0, 0.005), (1.5, 0.8, 0.01), (0.5, 0.88, 0.02)])
def test_smoothing_at_one_width_inside_the_cutoff(eps, sig, h):
    """At r = rc - h sigma, x = -1: g = 1/2 and g' = -1, so V_s = V_ts / 2 and
    -dV_s/dr = F / 2 + V_ts / (h sigma).  Expected values in exact rationals
    from the LJ formula (catches a wrong power, sign or width in g)."""
    from fractions import Fraction as Fr
    rc = 2.5 * sig
    r = rc - h * sig
    R = Fr(r)
    vts = _lj_exact(R * R, eps, sig) - _lj_exact(Fr(rc) ** 2, eps, sig)
    s2 = Fr(sig) ** 2 / (R * R)
    f_lj = 24 * Fr(eps) * (2 * s2 ** 6 - s2 ** 3) / R
    v, f = O.pair(r, eps, sig, rc, h)
    assert v == pytest.approx(float(vts / 2), rel=1e-9)
    assert f == pytest.approx(float(f_lj / 2 + vts / (Fr(h) * Fr(sig))), rel=1e-7)


def test_smoothing_far_inside_and_at_ten_widths():
    """x = -10: g = 10^4 / (1 + 10^4) exactly; deep inside, V_s -> V_ts."""
    rc, h = 2.5, 0.01
    r = rc - 10 * h
    v_s, _ = O.pair(r, 1.0, 1.0, rc, h)
    v_t, _ = O.pair(r, 1.0, 1.0, rc, 0.0)
    assert v_s == pytest.approx(v_t * 1e4 / (1 + 1e4), rel=1e-9)
    v_s, f_s = O.pair(1.1, 1.0, 1.0, rc, h)
    v_t, f_t = O.pair(1.1, 1.0, 1.0, rc, 0.0)
    x = (1.1 - rc) / h
    assert v_s == pytest.approx(v_t, rel=2.0 / x ** 4)
    assert f_s == pytest.approx(f_t, rel=1e-6)


@pytest.mark.parametrize("h", [0.005, 0.01])
def test_smoothed_potential_is_c2_at_the_cutoff(h):
    """C2 at rc (why the paper smooths): approaching rc from inside, V_s
    vanishes like delta^5 and the force like delta^4 (V_ts is linear in delta
    and g like delta^4), whereas the plain truncated force jumps."""
    rc = 2.5
    d1, d2 = 0.02 * h, 0.01 * h
    v1, f1 = O.pair(rc - d1, 1.0, 1.0, rc, h)
    v2, f2 = O.pair(rc - d2, 1.0, 1.0, rc, h)
    assert v1 / v2 == pytest.approx(32.0, rel=0.02)
    assert f1 / f2 == pytest.approx(16.0, rel=0.02)
    assert abs(f2) < 1e-6
    assert O.pair(rc - d2, 1.0, 1.0, rc, 0.0)[1] == pytest.approx(-0.0389994774528, rel=5e-4)
    assert O.pair(rc, 1.0, 1.0, rc, h) == (0.0, 0.0)


def test_smoothed_force_is_minus_dv_dr():
    """-dV_s/dr by 4th-order central differences, including the smoothing
    region (catches a dropped product-rule term)."""
    rng = np.random.default_rng(2)
    for eps, sig, h in [(1.0, 1.0, 0.005), (1.5, 0.8, 0.01), (0.5, 0.88, 0.05)]:
        rc = 2.5 * sig
        rs = np.concatenate([rng.uniform(0.9 * sig, rc - 5 * h * sig, 10),
                             rc - h * sig * rng.uniform(0.2, 4.0, 10)])
        for r in rs:
            dr = 1e-3 * h * sig
            vs = [O.pair(r + k * dr, eps, sig, rc, h)[0] for k in (-2, -1, 1, 2)]
            dv = (vs[0] - 8 * vs[1] + 8 * vs[2] - vs[3]) / (12 * dr)
            f = O.pair(r, eps, sig, rc, h)[1]
            assert f == pytest.approx(-dv, rel=1e-5, abs=1e-9 / (h * sig))


@pytest.mark.parametrize("h", [0.0, 0.005])
def test_wca_closed_forms(h):
    """WCA (Sec. 4): LJ cut at 2^(1/6) sigma, shifted by +eps, so V(sigma) = eps,
    V and F vanish at the cutoff, and the force is repulsive everywhere."""
    rc = RMIN
    v, f = O.pair(1.0, 1.0, 1.0, rc, h)
    x = (1.0 - rc) / h if h else -np.inf
    g = x ** 4 / (1 + x ** 4) if h else 1.0
    assert v == pytest.approx(1.0 * g, rel=1e-12)
    assert f == pytest.approx(24.0 * g, rel=1e-4)
    v, f = O.pair(rc * (1 - 1e-9), 1.0, 1.0, rc, h)
    assert abs(v) < 1e-12 and abs(f) < 1e-6
    for r in np.linspace(0.85, rc * (1 - 1e-6), 40):
        assert O.pair(r, 1.0, 1.0, rc, h)[1] > 0.0


def test_smoothing_makes_energy_error_second_order():
    """Sec. 4.3: velocity Verlet's energy error is O(dt^2) only for a
    potential with a continuous second derivative.  With a short cutoff
    (rc = 1.5 sigma, a large force jump) the plain truncation breaks the
    dt^2 scaling of E(t) - E(0); the C2-smoothed potential restores a ratio
    of 4 when dt is halved."""
    base = I.make_lj(256, rho=0.75, temperature=1.12, jitter=0.05, seed=6)
    span = 1.0
    ratios = {}
    for h in (0.0, 0.05):
        t = I.PairTable(1, base.table.eps, base.table.sigma, np.full((2, 2), 1.5), smooth=h)
        amp = []
        for dt in (0.004, 0.002):
            p, v = base.pos, base.vel
            e0 = O.observables(p, v, base.box, base.species, t)["etot"]
            dev = 0.0
            for _ in range(20):
                p, v, _, _ = O.vv(p, v, base.box, base.species, t, dt, int(round(span / dt / 20)))
                dev = max(dev, abs(O.observables(p, v, base.box, base.species, t)["etot"] - e0))
            amp.append(dev)
        ratios[h] = amp[0] / amp[1]
    assert 3.8 < ratios[0.05] < 4.2, ratios
    assert abs(ratios[0.0] - 4.0) > 1.0, ratios


# ------------------------------------------------ upload rule (host side)
def test_upload_rule_folds_and_rounds_as_defined():
    """Folding keeps x = x_folded + image L exactly for in-range values and
    lands in [0, L); FP32 rounding is numpy's float32; the double-single
    value hi + lo is within 2^-48 of x, with hi = fl32(x) (Sec. 2.4)."""
    from oracle import upload as U
    rng = np.random.default_rng(3)
    L = 17.25
    x = rng.uniform(-2 * L, 3 * L, size=(2000, 3))
    xf, img = U.fold(x.copy(), L)
    assert (xf >= 0).all() and (xf < L).all()
    assert np.abs(xf + img * L - x).max() < 1e-12 * L
    v = rng.normal(size=(2000, 3))
    p32, v32, _ = U.state_after_upload(x, v, L, "fp32")
    assert np.array_equal(v32, v.astype(np.float32).astype(np.float64))
    assert np.array_equal(p32, xf.astype(np.float32).astype(np.float64))
    pds, vds, _ = U.state_after_upload(x, v, L, "ds")
    assert np.abs(pds - xf).max() <= 2.0 ** -48 * L
    assert np.abs(vds - v).max() <= 2.0 ** -48 * np.abs(v).max()
    assert np.array_equal(pds.astype(np.float32), xf.astype(np.float32))  # hi = fl32(x)
    p64, v64, i64 = U.state_after_upload(x, v, L, "fp64")
    assert np.array_equal(p64, xf) and np.array_equal(v64, v) and np.array_equal(i64, img)


# ------------------------------------------------------- observables
def test_pressure_of_an_ideal_gas():
    """No pair inside the cutoff: W = 0 and E_pot = 0, so the pressure is the
    ideal-gas value P = N T / V with T = m sum v^2 / (3 N) computed here;
    catches a wrong volume (L^2, L^3 / 3), a dropped factor 2 on E_kin or a
    non-zero virial from pairs beyond the cutoff."""
    L = 40.0
    g = np.arange(4) * 10.0 + 1.0  # spacing 10 > rc = 2.5, also across the faces
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    n = len(pos)
    vel = np.random.default_rng(2).normal(size=(n, 3))
    t = I.lj_table()
    o = O.observables(pos, vel, L, np.zeros(n, dtype=np.int32), t, mass=1.7)
    temp = 1.7 * float(np.sum(vel * vel)) / (3 * n)
    assert o["virial"] == 0.0 and o["epot"] == 0.0
    assert o["temperature"] == pytest.approx(temp, rel=1e-14)
    assert o["pressure"] == pytest.approx(n * temp / L ** 3, rel=1e-14)


@pytest.mark.parametrize("r,species", [(1.1, (0, 0)), (1.3, (0, 1)), (0.95, (1, 1))])
def test_pressure_of_two_particles_by_hand(r, species):
    """Two particles of the KA table at separation r along x: E_pot = V_ts(r),
    W = r F(r) with F = -dV/dr = (24 eps / r) [2 (sigma/r)^12 - (sigma/r)^6],
    P = (2 E_kin + W) / (3 L^3), all written out here in exact rationals
    (fractions), independent of the oracle's pair routine."""
    from fractions import Fraction as Fr
    t = I.ka_table()
    a, b = species
    eps, sig, rc = (Fr(float(t.eps[a, b])), Fr(float(t.sigma[a, b])), Fr(float(t.rcut[a, b])))
    L = 12.0
    pos = np.array([[3.0, 5.0, 5.0], [3.0 + r, 5.0, 5.0]])
    vel = np.array([[0.3, -0.2, 0.1], [-0.3, 0.2, -0.1]])
    o = O.observables(pos, vel, L, np.array([a, b], dtype=np.int32), t)
    rr = Fr(pos[1, 0]) - Fr(pos[0, 0])  # the separation as the doubles hold it

    def v(x):
        s6 = (sig / x) ** 6
        return 4 * eps * (s6 * s6 - s6)

    s6 = (sig / rr) ** 6
    force = 24 * eps / rr * (2 * s6 * s6 - s6)
    ekin = Fr(1, 2) * sum(Fr(float(c)) ** 2 for c in vel.ravel())
    epot = v(rr) - v(rc)
    w = rr * force
    p = (2 * ekin + w) / (3 * Fr(L) ** 3)
    assert o["epot"] == pytest.approx(float(epot), rel=1e-13)
    assert o["virial"] == pytest.approx(float(w), rel=1e-13)
    assert o["pressure"] == pytest.approx(float(p), rel=1e-13)
