"""Blocking scheme for time-correlation functions (Sec. 2.5), plain NumPy.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and nothing on
the product path.  It shares no code with the HIP library.

The scheme, as the paper describes it: samples A_m = A(m dt_s), m = 0, 1, ...
fill k blocks of l entries; block n receives every l^n-th sample (time
resolution l^n dt_s).  Whenever a block holds l entries its first (oldest)
entry is correlated with the l - 1 others -- time lags j l^n dt_s,
j = 1 .. l-1 -- and then discarded.  Each correlation adds one term per lag;
the estimate is the mean of the terms.

Tagged-particle correlations of a sample pair (origin s, later sample t),
averaged over the particles of each species:
  MSD   <|r_i(t) - r_i(s)|^2>      (unwrapped positions)
  VACF  <v_i(t) . v_i(s)>
  F_s   <cos(q (x_i(t) - x_i(s)))> averaged over the three axis directions,
        q = 2 pi n_q / L (the caller picks n_q).
"""
from __future__ import annotations

from collections import deque

import numpy as np


def pair_terms(pos_s, vel_s, pos_t, vel_t, species, q, n_species=2):
    """[n_species, 3] array of (MSD, VACF, F_s) species means, and counts."""
    d = pos_t - pos_s
    msd = np.sum(d * d, axis=1)
    vacf = np.sum(vel_t * vel_s, axis=1)
    fs = np.mean(np.cos(q * d), axis=1)
    out = np.zeros((n_species, 3))
    cnt = np.zeros(n_species, dtype=np.int64)
    for a in range(n_species):
        m = species == a
        cnt[a] = int(m.sum())
        if cnt[a]:
            out[a] = [msd[m].mean(), vacf[m].mean(), fs[m].mean()]
    return out, cnt


class Blocking:
    """The blocking scheme over samples (unwrapped positions, velocities)."""

    def __init__(self, levels: int, block: int, species, q: float, n_species: int = 2):
        self.k, self.l = levels, block
        self.species = np.asarray(species)
        self.q = q
        self.ns = n_species
        self.blocks = [deque() for _ in range(levels)]
        self.sums = np.zeros((levels, block - 1, n_species, 3))
        self.terms = np.zeros((levels, block - 1), dtype=np.int64)
        self.m = 0

    def sample(self, pos, vel):
        """Insert sample m into every block whose resolution divides m."""
        for n in range(self.k):
            if self.m % (self.l ** n):
                break
            b = self.blocks[n]
            b.append((np.array(pos, dtype=np.float64), np.array(vel, dtype=np.float64)))
            if len(b) == self.l:
                p0, v0 = b[0]
                for j in range(1, self.l):
                    t, _ = pair_terms(p0, v0, b[j][0], b[j][1], self.species, self.q, self.ns)
                    self.sums[n, j - 1] += t
                    self.terms[n, j - 1] += 1
                b.popleft()
        self.m += 1

    def result(self):
        """(lags in units of the sample interval [k, l-1], means
        [k, l-1, n_species, 3] (NaN where no term), term counts [k, l-1])."""
        lags = np.array([[j * self.l ** n for j in range(1, self.l)] for n in range(self.k)],
                        dtype=np.int64)
        with np.errstate(invalid="ignore"):
            means = self.sums / self.terms[:, :, None, None]
        return lags, means, self.terms.copy()


def direct(samples, lag: int, species, q, n_species=2, origins=None):
    """The plain estimator of Sec. 2.5 for one lag: the mean over origins s
    (every s with s + lag < M unless `origins` is given) of the terms."""
    M = len(samples)
    if origins is None:
        origins = range(M - lag)
    acc = np.zeros((n_species, 3))
    k = 0
    for s in origins:
        t, _ = pair_terms(samples[s][0], samples[s][1], samples[s + lag][0], samples[s + lag][1],
                          species, q, n_species)
        acc += t
        k += 1
    return acc / k, k
