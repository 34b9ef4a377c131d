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


def test_analytic_null_recovers_var_parents():
    # Gaussian estimator with the chi^2 null on a linear VAR: the paper's
    # choice for its VAR experiments.  Target 0 of the 5-node network has the
    # parents (2, lag 2) and (4, lag 2).
    from synth import gen
    s, _ = gen.var_network(5, 2000, seed=1)
    res = greedy.select_sources(s, 0, [1, 2, 3, 4], max_lag_sources=3, max_lag_target=3,
                                alpha=0.05, seed=0, null="analytic")
    assert sorted((n, l) for (n, l, _, _) in res["sources"]) == [(2, 2), (4, 2)]
    assert res["significant"] and res["omnibus_p"] < 1e-10
    # no surrogates: one estimate per candidate test
    assert res["n_estimates"] < 60


def test_analytic_null_on_independent_series_selects_little():
    hits = 0
    for seed in range(10):
        g = np.random.default_rng(300 + seed)
        s = g.standard_normal((3, 1000)).astype(np.float32)
        res = greedy.select_sources(s, 0, [1, 2], max_lag_sources=3, max_lag_target=2,
                                    alpha=0.05, null="analytic")
        hits += len(res["sources"]) > 0
    assert hits <= 3


def test_standardise_definition():
    # mean 0 and variance 1 (float32 rounding), constant node -> zeros,
    # scaling a node by a power of two leaves its z-scores bit-identical
    # (mean and sd scale exactly), and replications are pooled per node.
    g = np.random.default_rng(3)
    s = (g.standard_normal((4, 3001)) * [[3.0], [0.01], [100.0], [1.0]] + [[5], [-2], [0], [1e3]])
    s = s.astype(np.float32)
    s[3] = 7.25
    z = greedy.standardise(s)
    for p in range(3):
        assert abs(z[p].astype(np.float64).mean()) < 1e-6
        assert abs(z[p].astype(np.float64).var() - 1.0) < 1e-5
    assert np.all(z[3] == 0)
    s2 = s.copy()
    s2[0] *= np.float32(8.0)
    s2[1] *= np.float32(0.125)
    z2 = greedy.standardise(s2)
    assert np.array_equal(z2.view(np.uint32), z.view(np.uint32))
    r = g.standard_normal((3, 2, 500)).astype(np.float32)
    zr = greedy.standardise(r)
    pooled = greedy.standardise(np.concatenate([r[0], r[1], r[2]], axis=1))
    assert np.array_equal(np.concatenate([zr[0], zr[1], zr[2]], axis=1), pooled)
