"""Pins of the blocking-scheme oracle for time-correlation functions
(Sec. 2.5) against facts that do not come from it: closed forms for
ballistic motion, the number of correlation terms each block level must
produce, and the plain estimator over the time origins the scheme uses."""
import math

import numpy as np
import pytest

from oracle import tcf


def _ballistic(n=300, M=130, seed=1):
    rng = np.random.default_rng(seed)
    r0 = rng.uniform(0, 10, (n, 3))
    v = rng.normal(0, 1, (n, 3))
    sp = (rng.uniform(size=n) < 0.2).astype(int)
    samples = [(r0 + v * m * 0.05, v.copy()) for m in range(M)]
    return samples, v, sp


def test_ballistic_closed_forms():
    """Free flight r(t) = r0 + v t: MSD = <v^2> t^2, VACF = <v^2>,
    F_s = <cos(q v_c t)> over particles and axes, per species and lag."""
    samples, v, sp = _ballistic()
    q = 7.25
    b = tcf.Blocking(levels=3, block=5, species=sp, q=q)
    for p, vel in samples:
        b.sample(p, vel)
    lags, means, terms = b.result()
    for n in range(3):
        for j in range(4):
            if terms[n, j] == 0:
                continue
            t = lags[n, j] * 0.05
            for a in (0, 1):
                m = sp == a
                v2 = np.sum(v[m] ** 2, axis=1).mean()
                fs = np.cos(q * v[m] * t).mean()
                assert means[n, j, a, 0] == pytest.approx(v2 * t * t, rel=1e-12)
                assert means[n, j, a, 1] == pytest.approx(v2, rel=1e-12)
                assert means[n, j, a, 2] == pytest.approx(fs, rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("M", [1, 4, 5, 6, 24, 25, 26, 124, 125, 126, 400])
def test_term_counts_per_level(M):
    """Block n receives samples m = 0, l^n, 2 l^n, ... (floor((M-1)/l^n) + 1
    of them); each insertion into a full block gives one term per lag."""
    l, k = 5, 4
    b = tcf.Blocking(levels=k, block=l, species=np.zeros(2, dtype=int), q=1.0)
    for m in range(M):
        b.sample(np.zeros((2, 3)) + m, np.ones((2, 3)))
    _, _, terms = b.result()
    for n in range(k):
        inserted = (M - 1) // l ** n + 1 if M > 0 else 0
        assert (terms[n] == max(0, inserted - l + 1)).all(), (n, terms[n])


def test_blocking_equals_direct_estimator_over_its_origins():
    """Level n correlates origins a l^n (a = 0 .. inserted - l) with lags
    j l^n: the plain estimator over exactly those origins gives the same
    means (a random-walk trajectory, so every lag differs)."""
    rng = np.random.default_rng(3)
    n, M, l, k = 64, 160, 4, 3
    sp = (rng.uniform(size=n) < 0.3).astype(int)
    pos = np.cumsum(rng.normal(0, 0.3, (M, n, 3)), axis=0)
    vel = rng.normal(0, 1, (M, n, 3))
    samples = [(pos[m], vel[m]) for m in range(M)]
    q = 2 * math.pi / 3.0
    b = tcf.Blocking(levels=k, block=l, species=sp, q=q)
    for p, v in samples:
        b.sample(p, v)
    lags, means, terms = b.result()
    for lev in range(k):
        step = l ** lev
        inserted = (M - 1) // step + 1
        origins = [a * step for a in range(inserted - l + 1)]
        for j in range(1, l):
            ref, cnt = tcf.direct(samples, j * step, sp, q, origins=origins)
            assert cnt == terms[lev, j - 1]
            np.testing.assert_allclose(means[lev, j - 1], ref, rtol=1e-12, atol=1e-14)
