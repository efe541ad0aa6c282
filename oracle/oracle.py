"""Python face of the FP64 CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It wraps `md_oracle.c` (compiled with gcc, no fast-math,
no FP contraction) through ctypes.

What it computes is the plain definition of the paper's MD step (Sec. 2.2,
velocity Verlet with short-ranged pair forces; Sec. 3 LJ 12-6 cut at
rc = 2.5 sigma; Sec. 5 Kob-Andersen pair table; Sec. 4 WCA and the C2
smoothing factor g): brute-force forces, energies
and virials, brute-force neighbour-list membership, and a naive
velocity-Verlet integrator; and, as a second independent route for large N,
cell-list forces and velocity Verlet over skin-padded Verlet lists.  Every function here is pinned by a test
against a fact that does not come from this module (closed forms,
invariants, library routines).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "md_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile md_oracle.c into liboracle.so (gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-std=c99", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_forces.argtypes = [ctypes.c_int, ctypes.c_double, ip, dp, ctypes.c_int,
                                   dp, dp, dp, ctypes.c_double, ip, ctypes.c_int, dp, dp, dp]
        lib.orc_forces.restype = None
        lib.orc_neighbours.argtypes = [ctypes.c_int, ctypes.c_double, ip, dp, ctypes.c_int,
                                       dp, ip, ctypes.c_int, ctypes.c_int, ip, ip]
        lib.orc_neighbours.restype = None
        lib.orc_vv.argtypes = [ctypes.c_int, ctypes.c_double, ip, dp, dp, ip, ctypes.c_int,
                               dp, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_int, dp]
        lib.orc_vv.restype = None
        lib.orc_pair.argtypes = [ctypes.c_double] * 5 + [dp, dp]
        lib.orc_pair.restype = None
        lib.orc_forces_cells.argtypes = [ctypes.c_int, ctypes.c_double, ip, dp, ctypes.c_int,
                                         dp, dp, dp, ctypes.c_double, dp, dp, dp]
        lib.orc_forces_cells.restype = None
        lib.orc_vv_lists.argtypes = [ctypes.c_int, ctypes.c_double, ip, dp, dp, ip, ctypes.c_int,
                                     dp, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, dp]
        lib.orc_vv_lists.restype = ctypes.c_int
        _lib = lib
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _tab(table):
    eps = np.ascontiguousarray(table.eps, dtype=np.float64).reshape(4)
    sig = np.ascontiguousarray(table.sigma, dtype=np.float64).reshape(4)
    rc = np.ascontiguousarray(table.rcut, dtype=np.float64).reshape(4)
    return eps, sig, rc


def pair(r: float, eps: float = 1.0, sigma: float = 1.0, rc: float = 2.5,
         h: float = 0.0) -> Tuple[float, float]:
    """(V(r), F(r)) for one pair at distance r: truncated-and-shifted energy
    (times the smoothing factor g when h > 0) and the radial force -dV/dr
    (positive = repulsive)."""
    lib = _load()
    v = ctypes.c_double()
    ff = ctypes.c_double()
    lib.orc_pair(r * r, eps, sigma, rc, h, ctypes.byref(v), ctypes.byref(ff))
    return v.value, ff.value * r


def forces(pos: np.ndarray, box: float, species: np.ndarray, table,
           sel: Optional[np.ndarray] = None):
    """Brute-force FP64 forces F[m,3], per-particle energy e[m] and per-particle
    virial w[m] for the particles in `sel` (all when None)."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    sp = np.ascontiguousarray(species, dtype=np.int32)
    eps, sig, rc = _tab(table)
    if sel is None:
        m = n
        selp = None
    else:
        sel = np.ascontiguousarray(sel, dtype=np.int32)
        m = len(sel)
        selp = _i(sel)
    f = np.zeros((m, 3))
    e = np.zeros(m)
    w = np.zeros(m)
    lib.orc_forces(n, box, _i(sp), _d(pos), table.n_species, _d(eps), _d(sig), _d(rc),
                   float(table.smooth), selp, m, _d(f), _d(e), _d(w))
    return f, e, w


def neighbours(pos: np.ndarray, box: float, species: np.ndarray, table, skin: float,
               sel: Optional[np.ndarray] = None, cap: int = 512):
    """Neighbour-list membership per particle: ascending ids j != i with
    |d_ij| < rc_{s_i s_j} + skin.  Returns a list of int arrays."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    sp = np.ascontiguousarray(species, dtype=np.int32)
    rl = np.ascontiguousarray(np.asarray(table.rcut, dtype=np.float64) + skin).reshape(4)
    if sel is None:
        sel = np.arange(n, dtype=np.int32)
    sel = np.ascontiguousarray(sel, dtype=np.int32)
    m = len(sel)
    counts = np.zeros(m, dtype=np.int32)
    ids = np.zeros((m, cap), dtype=np.int32)
    lib.orc_neighbours(n, box, _i(sp), _d(pos), table.n_species, _d(rl), _i(sel), m, cap,
                       _i(counts), _i(ids))
    if counts.max(initial=0) > cap:
        return neighbours(pos, box, species, table, skin, sel, int(counts.max()) + 16)
    return [ids[k, :counts[k]].copy() for k in range(m)]


def vv(pos: np.ndarray, vel: np.ndarray, box: float, species: np.ndarray, table,
       dt: float, steps: int, mass: float = 1.0):
    """Naive velocity Verlet for `steps` steps.  Returns (pos, vel, image, f):
    wrapped positions, velocities, box crossings per component and the forces
    at the final positions."""
    lib = _load()
    p = np.array(pos, dtype=np.float64, order="C", copy=True)
    v = np.array(vel, dtype=np.float64, order="C", copy=True)
    n = p.shape[0]
    img = np.zeros((n, 3), dtype=np.int32)
    sp = np.ascontiguousarray(species, dtype=np.int32)
    eps, sig, rc = _tab(table)
    f = np.zeros((n, 3))
    lib.orc_vv(n, box, _i(sp), _d(p), _d(v), _i(img), table.n_species, _d(eps), _d(sig),
               _d(rc), float(table.smooth), mass, dt, steps, _d(f))
    return p, v, img, f


def observables(pos, vel, box, species, table, mass: float = 1.0) -> dict:
    """E_pot, E_kin, E_tot, T = 2E_kin/(3N), momentum, virial W and
    pressure P = (2 E_kin + W) / (3 V), all in FP64 with exact (fsum) sums."""
    f, e, w = forces(pos, box, species, table)
    n = len(pos)
    ekin = 0.5 * mass * math.fsum((np.asarray(vel) ** 2).ravel())
    epot = math.fsum(e)
    wv = math.fsum(w)
    vol = box ** 3
    return {
        "epot": epot, "ekin": ekin, "etot": epot + ekin,
        "temperature": 2.0 * ekin / (3.0 * n),
        "momentum": mass * np.array([math.fsum(vel[:, c]) for c in range(3)]),
        "virial": wv, "pressure": (2.0 * ekin + wv) / (3.0 * vol),
        "forces": f,
    }


def forces_cells(pos: np.ndarray, box: float, species: np.ndarray, table):
    """Forces F[n,3], per-particle energies e[n] and virials w[n] of every
    particle through cell lists (Sec. 2.2 cell binning): the same definition
    as forces(), each particle's partners searched in its own and the 26
    adjacent cells of edge >= the largest cutoff."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    sp = np.ascontiguousarray(species, dtype=np.int32)
    eps, sig, rc = _tab(table)
    f = np.zeros((n, 3))
    e = np.zeros(n)
    w = np.zeros(n)
    lib.orc_forces_cells(n, box, _i(sp), _d(pos), table.n_species, _d(eps), _d(sig), _d(rc),
                         float(table.smooth), _d(f), _d(e), _d(w))
    return f, e, w


def vv_lists(pos: np.ndarray, vel: np.ndarray, box: float, species: np.ndarray, table,
             dt: float, steps: int, skin: float, mass: float = 1.0):
    """Velocity Verlet like vv(), with forces over Verlet lists of radius
    max cutoff + skin built through cell lists and rebuilt whenever a
    particle has moved more than skin/2 since the last build (Sec. 2.2).
    Returns (pos, vel, image, f, builds)."""
    lib = _load()
    p = np.array(pos, dtype=np.float64, order="C", copy=True)
    v = np.array(vel, dtype=np.float64, order="C", copy=True)
    n = p.shape[0]
    img = np.zeros((n, 3), dtype=np.int32)
    sp = np.ascontiguousarray(species, dtype=np.int32)
    eps, sig, rc = _tab(table)
    f = np.zeros((n, 3))
    builds = lib.orc_vv_lists(n, box, _i(sp), _d(p), _d(v), _i(img), table.n_species, _d(eps),
                              _d(sig), _d(rc), float(table.smooth), mass, dt, skin, steps, _d(f))
    return p, v, img, f, int(builds)
