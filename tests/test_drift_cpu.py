"""Host-side statistics of the energy-drift measurement (no GPU): the OLS
slope and its block-averaged error, and the ensemble mean with its error
from the spread of the replicas."""
import math

import numpy as np
import pytest

from paper_0912_3824_amd.drift import ensemble, slope_with_error


def test_slope_of_a_noiseless_line_is_exact():
    t = np.arange(0, 100001, 100, dtype=float)
    b, se, g = slope_with_error(t, -5.0 + 3e-9 * t)
    assert b == pytest.approx(3e-9, rel=1e-9)
    assert se == pytest.approx(0.0, abs=1e-18)


def test_white_noise_error_matches_the_textbook_formula():
    rng = np.random.default_rng(3)
    t = np.arange(1001, dtype=float)
    e = 2.0 + 1e-4 * t + rng.normal(0, 0.01, t.size)
    b, se, g = slope_with_error(t, e)
    resid = e - np.polyval(np.polyfit(t, e, 1), t)
    textbook = math.sqrt(resid @ resid / (t.size - 2) / np.sum((t - t.mean()) ** 2))
    assert b == pytest.approx(np.polyfit(t, e, 1)[0], rel=1e-12)
    assert se >= textbook * (1 - 1e-12) and se <= textbook * math.sqrt(g) * (1 + 1e-12)


def test_correlated_noise_inflates_the_error():
    rng = np.random.default_rng(4)
    t = np.arange(2000, dtype=float)
    walk = np.cumsum(rng.normal(0, 1e-3, t.size))  # a random walk: strongly correlated residuals
    _, se_w, g_w = slope_with_error(t, rng.normal(0, 1e-3, t.size))
    _, se_c, g_c = slope_with_error(t, walk)
    assert g_w < 3 and g_c > 10


def test_ensemble_mean_and_error_from_the_spread():
    slopes = [1.0, 3.0, 2.0, 6.0]
    recs = [{"slope_per_1e5_steps": x, "relative_slope_per_1e5_steps": x / 4, "stderr_per_1e5_steps": 0.1,
             "relative_stderr": 0.025, "rms_dev_from_e0": 0.5, "max_abs_momentum_per_particle": 1e-15 * (k + 1)}
            for k, x in enumerate(slopes)]
    r = ensemble(recs)
    assert r["replicas"] == 4
    assert r["slope_per_1e5_steps"] == pytest.approx(3.0)
    assert r["stderr_per_1e5_steps"] == pytest.approx(np.std(slopes, ddof=1) / 2)
    assert r["relative_slope_per_1e5_steps"] == pytest.approx(0.75)
    assert r["mean_block_stderr_per_1e5_steps"] == pytest.approx(0.1)
    assert r["max_abs_momentum_per_particle"] == pytest.approx(4e-15)
    one = ensemble(recs[:1])
    assert one["stderr_per_1e5_steps"] == 0.1 and one["slope_per_1e5_steps"] == 1.0
