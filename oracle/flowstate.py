"""Flow state of a probe time series (oracle; test infrastructure only).

Sec. 3.3 sorts each cavity into a stable, a periodic or an aperiodic
(unstable) state from the velocity at an observing point over a late window
of the run, and Table 3 lists periods.  The paper judges this from plots; the
definition used here (and by the library) is:

* amplitude A = max u - min u over the window; steady if A <= steady_tol;
* otherwise, with sigma the standard deviation of u over the window, the
  lag mismatch of every lag T in [min_lag, max_lag] (max_lag = n // 3 by
  default) is
      D(T) = mean_{k < n - T} (u[k + T] - u[k])^2 / sigma^2;
  a candidate is a lag T with min_lag < T < max_lag, D(T - 1) > D(T) <=
  D(T + 1), reached after D has exceeded 1 at a smaller lag (the series has
  decorrelated; over a whole period D averages 2, so every period passes
  this); the parabola through D at T - 1, T, T + 1 gives the refined period
  (its vertex) and the mismatch sqrt(max(vertex value, 0)); the series is
  periodic at the first candidate with mismatch <= periodic_tol;
* drift if there is no candidate at all: the series never returns towards
  an earlier value within the window (a monotone approach, e.g. to a steady
  state, or a period longer than max_lag);
* aperiodic otherwise (returns, but none close enough).

Returns a dict: state ("steady", "periodic", "drift", "aperiodic"), lag (the
integer lag, periodic only), period (samples; 0 unless periodic), amplitude,
mean, std, mismatch (at the chosen candidate; for an aperiodic series the
smallest over all candidates; inf for a drift), and the dominant cycle:
cycle (the refined lag of the first candidate whatever its mismatch, in
samples; 0 if none) with cycle_mismatch.  A modulated oscillation repeats
exactly only after several cycles: its period is that repeat, its cycle the
oscillation itself.

The parabola models D near a period well when the period spans a dozen or
more samples; a period of a few samples can come out as a multiple of itself.
"""
from __future__ import annotations

import math

import numpy as np


def lag_mismatch2(u, lag):
    """mean_{k < n - lag} (u[k + lag] - u[k])^2 (not yet divided by sigma^2)."""
    u = np.asarray(u, dtype=np.float64)
    d = u[lag:] - u[:len(u) - lag]
    return float(np.mean(d * d))


def classify(u, steady_tol, periodic_tol, min_lag=1, max_lag=None):
    u = np.asarray(u, dtype=np.float64)
    n = len(u)
    if n < 8:
        raise ValueError("need at least 8 samples")
    amp = float(u.max() - u.min())
    mean = float(u.mean())
    std = float(u.std())
    out = {"state": "steady", "lag": 0, "period": 0.0, "amplitude": amp, "mean": mean,
           "std": std, "mismatch": 0.0, "cycle": 0.0, "cycle_mismatch": 0.0}
    if amp <= steady_tol:
        return out
    if max_lag is None:
        max_lag = n // 3
    max_lag = min(max_lag, n - 2)
    lags = list(range(min_lag, max_lag + 1))
    D = [lag_mismatch2(u, T) / (std * std) for T in lags]
    best = math.inf
    decorrelated = False
    for j in range(1, len(lags) - 1):
        decorrelated = decorrelated or D[j - 1] > 1.0
        if not (decorrelated and D[j - 1] > D[j] <= D[j + 1]):
            continue
        curv = D[j - 1] - 2.0 * D[j] + D[j + 1]
        period, vertex = float(lags[j]), D[j]
        if curv > 0.0:
            period = lags[j] + 0.5 * (D[j - 1] - D[j + 1]) / curv
            vertex = D[j] - (D[j - 1] - D[j + 1]) ** 2 / (8.0 * curv)
        mismatch = math.sqrt(max(vertex, 0.0))
        if best == math.inf:
            out.update(cycle=period, cycle_mismatch=mismatch)
        best = min(best, mismatch)
        if mismatch <= periodic_tol:
            out.update(state="periodic", lag=lags[j], period=period, mismatch=mismatch)
            return out
    out.update(state="drift" if best == math.inf else "aperiodic", mismatch=best)
    if best == math.inf:
        out["cycle_mismatch"] = math.inf
    return out
