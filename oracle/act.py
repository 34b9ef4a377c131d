"""Autocorrelation decay time, the paper's heuristic for the Theiler window.
TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper (section on autocorrelation in real data) sizes the window of
excluded time neighbours by the autocorrelation decay time: the shortest time
shift at which the autocorrelation function has dropped by a factor 1/e from
its zero-shift value.  Written out:

  mu   = (1/T) sum_t x_t
  r(L) = (1/T) sum_{t=0}^{T-1-L} (x_t - mu)(x_{t+L} - mu)     (biased estimate)
  ACT  = min { L >= 1 : r(L) < r(0)/e },  or max_lag if no L <= max_lag qualifies.

Sums are float64 and strictly sequential in t (np.cumsum), so that a
library computing the same sums in the same order takes the same decision.
"""

from __future__ import annotations

import math

import numpy as np


def _seq_sum(v: np.ndarray) -> float:
    return float(np.cumsum(v, dtype=np.float64)[-1]) if len(v) else 0.0


def autocorr(x, lag: int) -> float:
    x = np.asarray(x, dtype=np.float64)
    t = len(x)
    mu = _seq_sum(x) / t
    c = x - mu
    return _seq_sum(c[: t - lag] * c[lag:]) / t


def decay_time(x, max_lag: int) -> int:
    """Shortest lag L >= 1 with r(L) < r(0)/e (max_lag if none)."""
    x = np.asarray(x, dtype=np.float64)
    if len(x) < 2 or max_lag < 1:
        raise ValueError("need T >= 2 and max_lag >= 1")
    r0 = autocorr(x, 0)
    thr = r0 / math.e
    for lag in range(1, min(max_lag, len(x) - 1) + 1):
        if autocorr(x, lag) < thr:
            return lag
    return max_lag
