"""Pins of the rand48 / Andersen-thermostat oracle (Sec. 2.3) against an
independent implementation (the C library's erand48), the plain recurrence,
and the statistics and exact temperature the thermostat must produce."""
import ctypes
import math

import numpy as np
import pytest

from oracle import thermostat as T


def _erand48_stream(state48: int, k: int):
    libc = ctypes.CDLL("libc.so.6")
    libc.erand48.restype = ctypes.c_double
    libc.erand48.argtypes = [ctypes.POINTER(ctypes.c_ushort)]
    xs = (ctypes.c_ushort * 3)(state48 & 0xFFFF, (state48 >> 16) & 0xFFFF, (state48 >> 32) & 0xFFFF)
    return [libc.erand48(xs) for _ in range(k)]


@pytest.mark.parametrize("seed", [0, 1, 0x1234ABCD, 20240101])
def test_rand48_matches_the_c_library(seed):
    """erand48 returns x_{k+1} / 2^48 from the state x_k: the oracle's
    recurrence and constants give the same numbers (catches a wrong
    multiplier, addend or modulus)."""
    x = T.seed_state(seed)
    lib = _erand48_stream(x, 50)
    ours = []
    for _ in range(50):
        x = T.step(x)
        ours.append(x / float(1 << 48))
    assert ours == lib


def test_jump_ahead_equals_the_recurrence():
    """A_j x + C_j (repeated squaring) equals j single steps, for j up to a
    few thousand and for the leap-frog strides of a replica."""
    x0 = T.seed_state(7)
    xs = [x0]
    for _ in range(3000):
        xs.append(T.step(xs[-1]))
    for j in [0, 1, 2, 3, 5, 64, 1000, 2047, 2999, 3000]:
        assert T.element(x0, j) == xs[j]
    n = 37  # stride of a replica of 37 particles
    for i in range(n):
        for r in range(4):
            assert T.element(x0, i + n * r) == xs[i + n * r]


def test_thermostat_statistics_and_exact_temperature():
    n, temp = 20000, 0.7
    v = T.andersen(n, temp, seed=11, call=3)
    assert 2 * 0.5 * np.sum(v * v) / (3 * n) == pytest.approx(temp, rel=1e-13)
    assert np.abs(v.sum(axis=0)).max() < 1e-9
    g = v / math.sqrt(temp)
    # Gaussian moments within 5 standard errors
    assert abs(g.mean()) < 5 / math.sqrt(3 * n)
    assert abs(np.mean(g ** 4) / np.mean(g ** 2) ** 2 - 3.0) < 5 * math.sqrt(96 / (3 * n))
    # different calls draw different numbers
    v2 = T.andersen(n, temp, seed=11, call=4)
    assert np.abs(v - v2).mean() > 0.1
