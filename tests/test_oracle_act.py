"""Pins for the autocorrelation decay time (oracle/act.py): sequences whose
autocorrelation function is known in closed form."""

import math

import numpy as np
import pytest

from oracle import act


def test_alternating_sequence():
    # x_t = (-1)^t: r(1) = -(T-1)/T r(0) < r(0)/e at once
    x = np.array([(-1.0) ** t for t in range(1000)])
    assert act.decay_time(x, 50) == 1


@pytest.mark.parametrize("period,expect", [(50, 10), (80, 16), (36, 7)])
def test_sinusoid(period, expect):
    # r(L)/r(0) -> cos(2 pi L / P) (1 - L/T): the first L with cos(2 pi L/P) < 1/e
    t = np.arange(period * 2000)
    x = np.sin(2 * np.pi * t / period)
    first = next(L for L in range(1, period) if math.cos(2 * math.pi * L / period) < 1 / math.e)
    assert first == expect
    assert act.decay_time(x, period) == expect


@pytest.mark.parametrize("phi,expect", [(0.8, 5), (0.5, 2), (0.9, 10)])
def test_ar1(phi, expect):
    # AR(1): r(L)/r(0) = phi^L, so ACT = min{L : phi^L < 1/e}
    assert min(L for L in range(1, 100) if phi ** L < 1 / math.e) == expect
    g = np.random.default_rng(7)
    n = 400000
    e = g.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0] / math.sqrt(1 - phi * phi)
    for i in range(1, n):
        x[i] = phi * x[i - 1] + e[i]
    assert act.decay_time(x, 100) == expect


def test_white_noise_and_cap():
    x = np.random.default_rng(3).standard_normal(5000)
    assert act.decay_time(x, 20) == 1
    # a constant-slope ramp never decays within a short max_lag
    assert act.decay_time(np.arange(10000, dtype=float), 5) == 5
