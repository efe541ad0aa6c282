"""Shared helpers of the GPU parity tests (test infrastructure)."""
import math
import sys

import numpy as np

import md_inputs as I
from oracle import oracle as O

# Tolerances (stated for the force parity):  e_F = max_{i,c} |F - F_ref| / F_rms
TOL_F = {"fp32": 1e-5, "ds": 1e-5, "mixed64": 1e-5, "fp64": 1e-10}
TOL_E = {"fp32": 1e-6, "ds": 1e-6, "mixed64": 1e-6, "fp64": 1e-12}
# pairs closer than this (relative) to a cutoff may be classified either way
# by an FP32 pair test; their particles are checked against the looser bound
BAND = 2e-6


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def pool_for(systems, prec, **kw):
    from paper_0912_3824_amd import mdx
    return mdx.md_init(systems, prec, **kw)


def pair_distances(pos, box, rmax):
    """All pairs within rmax: (i, j, r) with i != j, both orders (scipy kd-tree)."""
    from scipy.spatial import cKDTree
    p = np.mod(pos, box)
    p[p >= box] = 0.0
    t = cKDTree(p, boxsize=box)
    m = t.sparse_distance_matrix(t, rmax, output_type="coo_matrix")
    keep = m.row != m.col
    return m.row[keep], m.col[keep], m.data[keep]


def near_cutoff(pos, box, species, table, radius_of, band=BAND):
    """Boolean mask of particles with a pair whose distance lies within a
    relative `band` of radius_of(si, sj)."""
    sp = species if table.n_species > 1 else np.zeros(len(pos), dtype=int)
    rm = max(radius_of(a, b) for a in range(2) for b in range(2)) * (1 + 2 * band)
    i, j, r = pair_distances(pos, box, rm)
    rad = np.array([[radius_of(a, b) for b in range(2)] for a in range(2)])[sp[i], sp[j]]
    hit = np.abs(r - rad) < band * rad
    mask = np.zeros(len(pos), dtype=bool)
    mask[i[hit]] = True
    mask[j[hit]] = True
    return mask


def cutoff_jump(table):
    """Largest jump of the truncated pair force at a cutoff: |F_ab| just
    inside rc_ab, over the species pairs of the table (KA: the AB pair,
    0.073; single-species LJ at rc = 2.5: 0.039).  A pair within rounding of
    a cutoff can be classified either way by an FP32 test, so its particle's
    force may differ from the oracle's by this much."""
    k = table.n_species
    return max(abs(O.pair(table.rcut[a, b] * (1 - 1e-12), table.eps[a, b], table.sigma[a, b],
                          table.rcut[a, b], table.smooth)[1])
               for a in range(k) for b in range(k))


def force_error(f, ref, exclude=None):
    frms = math.sqrt(float(np.mean(ref * ref)))
    d = np.abs(f - ref)
    if exclude is not None and exclude.any():
        d = d[~exclude]
    return float(d.max()) / frms, frms
