"""The state a replica holds after upload, computed on the host from the
seeded input (test infrastructure only: imported by tests and the smoke
check; it shares no code with the HIP library).

The oracle must never take an input read back from the device.  Where a
comparison needs the device's own starting state (the positions and
velocities rounded to the precision mode's representation), this module
derives it from the seeded FP64 input by the upload rule: each position
component is folded into [0, L) with image counter floor(x / L); then FP32
rounds positions and velocities to single precision, double-single splits
each value into hi = fl32(x) and lo = fl32(x - hi) (Sec. 2.4; the value is
hi + lo), and MIXED64 and FP64 keep the doubles.
"""
from __future__ import annotations

import numpy as np


def fold(pos: np.ndarray, box: float):
    """Positions folded into [0, box) and their integer image counters."""
    img = np.floor(pos / box)
    x = pos - img * box
    hi = x >= box
    x[hi] -= box
    img[hi] += 1
    lo = x < 0
    x[lo] += box
    img[lo] -= 1
    return x, img.astype(np.int32)


def ds_value(x: np.ndarray) -> np.ndarray:
    """hi + lo of the double-single split of x (Sec. 2.4)."""
    hi = x.astype(np.float32)
    lo = (x - hi.astype(np.float64)).astype(np.float32)
    return hi.astype(np.float64) + lo.astype(np.float64)


def state_after_upload(pos: np.ndarray, vel: np.ndarray, box: float, precision: str):
    """(positions in [0, box), velocities, image counters) as the precision
    mode holds them after upload, in FP64."""
    x, img = fold(np.array(pos, dtype=np.float64), box)
    v = np.array(vel, dtype=np.float64)
    if precision == "fp32":
        x = x.astype(np.float32).astype(np.float64)
        v = v.astype(np.float32).astype(np.float64)
    elif precision == "ds":
        x = ds_value(x)
        v = ds_value(v)
    elif precision not in ("mixed64", "fp64"):
        raise ValueError(precision)
    return x, v, img
