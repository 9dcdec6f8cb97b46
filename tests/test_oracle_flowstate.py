"""Pins of the flow-state classifier (oracle/flowstate.py): signals whose
state and period are known in closed form."""
import math

import numpy as np
import pytest

from oracle import flowstate as F

K = np.arange(3000, dtype=np.float64)


def test_lag_mismatch_is_the_mean_squared_lag_difference():
    rng = np.random.default_rng(0)
    u = rng.normal(size=50)
    for lag in (1, 7, 49):
        want = sum((u[k + lag] - u[k]) ** 2 for k in range(50 - lag)) / (50 - lag)
        assert math.isclose(F.lag_mismatch2(u, lag), want, rel_tol=1e-13)


def test_steady():
    r = F.classify(0.01 + 1e-10 * np.sin(K), 1e-7, 0.02)
    assert r["state"] == "steady" and r["period"] == 0.0
    assert math.isclose(r["amplitude"], 2e-10, rel_tol=1e-3)
    assert math.isclose(r["mean"], 0.01, rel_tol=1e-9)


@pytest.mark.parametrize("P", [37.25, 125.4, 900.7])
def test_sinusoid_period(P):
    """A sampled sinusoid of period P samples (P need not be an integer)."""
    for a, b, phase in ((0.02, 0.01, 0.3), (3.0, -1.0, 2.0)):
        r = F.classify(a * np.sin(2 * np.pi * K / P + phase) + b, 1e-7, 0.02)
        assert r["state"] == "periodic"
        assert r["lag"] == round(P)
        assert abs(r["period"] - P) <= 0.01
        assert r["mismatch"] <= 0.01
        if P < 150:     # the window holds many periods: std -> |a| / sqrt(2)
            assert math.isclose(r["std"], abs(a) / math.sqrt(2), rel_tol=2e-3)


def test_non_sinusoidal_and_period_doubled_signals():
    sq = np.sign(np.sin(2 * np.pi * (K + 0.5) / 40)) + 0.3 * np.sin(6 * np.pi * K / 40)
    r = F.classify(sq, 1e-7, 0.02)
    assert r["state"] == "periodic" and r["lag"] == 40 and abs(r["period"] - 40) <= 0.01
    # a sub-harmonic makes the fundamental period 40, not 20
    pd = np.sin(2 * np.pi * K / 20) + 0.5 * np.sin(2 * np.pi * K / 40)
    r = F.classify(pd, 1e-7, 0.02)
    assert r["state"] == "periodic" and r["lag"] == 40


def test_modulated_oscillation_cycle_and_period():
    """A 30-sample oscillation whose amplitude repeats every 5 cycles: it
    returns closely after one cycle (the dominant cycle) but exactly only
    after five (the period)."""
    u = (1 + 0.2 * np.sin(2 * np.pi * K / 150)) * np.sin(2 * np.pi * K / 30)
    r = F.classify(u, 1e-7, 0.02)
    assert r["state"] == "periodic" and r["lag"] == 150 and abs(r["period"] - 150) <= 0.01
    assert abs(r["cycle"] - 30) <= 0.3 and 0.02 < r["cycle_mismatch"] < 0.5
    s = F.classify(np.sin(2 * np.pi * K / 37.25), 1e-7, 0.02)
    assert s["cycle"] == s["period"] and s["cycle_mismatch"] == s["mismatch"]


def test_noisy_sinusoid_is_periodic():
    rng = np.random.default_rng(1)
    r = F.classify(np.sin(2 * np.pi * K / 63.7) + 1e-3 * rng.normal(size=K.size), 1e-7, 0.02)
    assert r["state"] == "periodic" and abs(r["period"] - 63.7) <= 0.02


def test_aperiodic_signals():
    x = np.empty(3000)
    x[0] = 0.3
    for i in range(1, 3000):                     # logistic map, chaotic at 3.9
        x[i] = 3.9 * x[i - 1] * (1 - x[i - 1])
    assert F.classify(x, 1e-7, 0.02)["state"] == "aperiodic"
    rng = np.random.default_rng(2)
    assert F.classify(rng.normal(size=3000), 1e-7, 0.02)["state"] == "aperiodic"
    phi = (1 + math.sqrt(5)) / 2                 # two incommensurate frequencies
    q = np.sin(2 * np.pi * K / 20) + np.sin(2 * np.pi * K * phi / 20)
    r = F.classify(q, 1e-7, 0.02)
    assert r["state"] == "aperiodic" and r["period"] == 0.0 and r["mismatch"] > 0.02


def test_monotone_approaches_are_drifts():
    """A linear drift and an exponential approach to a steady value never
    return within the window: drift, not an aperiodic oscillation."""
    for u in (1e-3 * K, 0.3 + 1e-4 * np.exp(-K / 2000.0)):
        r = F.classify(u, 1e-7, 0.02)
        assert r["state"] == "drift" and r["mismatch"] == math.inf and r["period"] == 0.0
    # a period longer than the lag range is a drift too
    r = F.classify(np.sin(2 * np.pi * K / 5000.0), 1e-7, 0.02)
    assert r["state"] == "drift"
