"""Statistical pins for the oracle's greedy mTE inference (oracle/greedy.py).

The paper prints no CMI or TE values, so the greedy selections are pinned only
by behaviour the paper's statements imply: strong couplings at known lags are
recovered (Validation tasks, Results), nothing is selected on independent
series beyond the error rate the tests control (False positive rate on empty
networks), and the surrogate-count rule is enforced (Maximum statistic test).
Exact selections beyond that are parity unpinned.
"""

import numpy as np
import pytest

from oracle import cksg, greedy


def est(x, y, z, k):
    return cksg.cmi_ksg(x, y, z, k)


def test_recovers_a_strong_coupling():
    g = np.random.default_rng(7)
    t = 405
    s = np.zeros((3, t))
    s[0] = g.standard_normal(t)
    s[2] = g.standard_normal(t)
    s[1, 3:] = 0.9 * s[0, :-3] + 0.3 * g.standard_normal(t - 3)
    s = s.astype(np.float32)
    res = greedy.select_sources(s, 1, [0, 2], max_lag_sources=5, max_lag_target=5,
                                alpha=0.1, k=4, n_surr=20, seed=3, estimator=est)
    assert [(n, l) for (n, l, _, _) in res["sources"]] == [(0, 3)]
    assert res["significant"] and res["omnibus_p"] < 0.1
    assert res["n_estimates"] > 0


def test_independent_series_select_nothing_mostly():
    hits = 0
    for seed in range(6):
        g = np.random.default_rng(100 + seed)
        s = g.standard_normal((3, 305)).astype(np.float32)
        res = greedy.select_sources(s, 0, [1, 2], max_lag_sources=2, max_lag_target=2,
                                    alpha=0.1, k=4, n_surr=20, seed=seed, estimator=est)
        hits += len(res["sources"]) > 0
    assert hits <= 2


def test_rejects_too_few_surrogates():
    s = np.zeros((2, 50), np.float32)
    with pytest.raises(ValueError):
        greedy.select_sources(s, 0, [1], alpha=0.05, n_surr=20)
    with pytest.raises(ValueError):
        greedy.select_sources(s, 0, [0], alpha=0.5, n_surr=20)
