"""rand48 generator with leap-frog streams and the modified Andersen
thermostat of Sec. 2.3, written plainly (exact Python integers, NumPy FP64).

TEST INFRASTRUCTURE ONLY: imported by tests and nothing on the product path.
It shares no code with the HIP library.

rand48: x_{k+1} = (a x_k + c) mod 2^48, a = 0x5DEECE66D, c = 0xB, uniform
u_k = x_k / 2^48 in [0, 1).  Jumping j elements ahead is the affine map
x -> A_j x + C_j with A_j = a^j, C_j = c (1 + a + ... + a^(j-1)) (mod 2^48),
as in the paper's leap-frog; here it is computed by repeated squaring.

Thermostat call k on a replica of n particles, particle id i: the four
stream elements i + n (4k + r), r = 0..3 (a leap-frog of stride n over the
particles) give uniforms u0..u3; Box-Muller gives three standard normals
  g0 = sqrt(-2 ln(1 - u0)) cos(2 pi u1),  g1 = sqrt(-2 ln(1 - u0)) sin(2 pi u1),
  g2 = sqrt(-2 ln(1 - u2)) cos(2 pi u3);
v_i = sqrt(T / m) g.  Optionally the mean velocity is subtracted; then all
velocities are scaled so that 2 E_kin / (3 N) = T exactly.
"""
from __future__ import annotations

import math

import numpy as np

A48 = 0x5DEECE66D
C48 = 0xB
M48 = (1 << 48) - 1


def step(x: int) -> int:
    return (A48 * x + C48) & M48


def jump(j: int):
    """(A_j, C_j) of the j-fold composition of x -> a x + c, mod 2^48."""
    A, C = 1, 0          # accumulated map
    a, c = A48, C48      # the map applied 2^bit times
    while j:
        if j & 1:
            A, C = (a * A) & M48, (a * C + c) & M48
        a, c = (a * a) & M48, (a * c + c) & M48
        j >>= 1
    return A, C


def element(seed_state: int, j: int) -> int:
    """Stream element j counted from the state seed_state (element 0)."""
    A, C = jump(j)
    return (A * seed_state + C) & M48


def seed_state(seed: int) -> int:
    """State of srand48(seed): the seed's low 32 bits above 0x330E."""
    return ((seed & 0xFFFFFFFF) << 16) | 0x330E


def uniforms(seed: int, n: int, call: int):
    """[n, 4] uniforms of thermostat call `call` (by particle id)."""
    x0 = seed_state(seed)
    out = np.zeros((n, 4))
    for i in range(n):
        for r in range(4):
            out[i, r] = element(x0, i + n * (4 * call + r)) / float(1 << 48)
    return out


def andersen(n: int, temperature: float, seed: int, call: int, mass: float = 1.0,
             remove_mean: bool = True):
    """Velocities [n, 3] (by particle id) assigned by thermostat call `call`."""
    u = uniforms(seed, n, call)
    ra = np.sqrt(-2.0 * np.log(1.0 - u[:, 0]))
    rb = np.sqrt(-2.0 * np.log(1.0 - u[:, 2]))
    g = np.stack([ra * np.cos(2 * math.pi * u[:, 1]), ra * np.sin(2 * math.pi * u[:, 1]),
                  rb * np.cos(2 * math.pi * u[:, 3])], axis=1)
    v = math.sqrt(temperature / mass) * g
    if remove_mean:
        v = v - v.mean(axis=0)
    t_now = mass * math.fsum((v * v).ravel()) / (3 * n)
    return v * math.sqrt(temperature / t_now)
