"""Pins of the replication (trial) surrogates of the oracle (oracle/perm.py,
Maximum statistic test section: shuffle the order of the candidate's
replications when there are enough of them, else the samples within each
trial), and of the greedy search over pooled replications."""

import math
from collections import Counter

import numpy as np
import pytest
from scipy.stats import chi2

from oracle import cksg, greedy, perm


def blocks(src, reps):
    n_r = len(src) // reps
    return [src[r * n_r:(r + 1) * n_r] for r in range(reps)], n_r


@pytest.mark.parametrize("reps,n_r", [(2, 5), (5, 7), (7, 1), (12, 33)])
def test_replication_shuffle_moves_whole_blocks(reps, n_r):
    for s in range(20):
        src = perm.replication_source_rows(9, 4, s, reps * n_r, reps, perm.REPLICATIONS).astype(np.int64)
        bl, _ = blocks(src, reps)
        sigma = []
        for r, b in enumerate(bl):
            q = int(b[0]) // n_r
            assert np.array_equal(b, q * n_r + np.arange(n_r))      # offsets kept
            sigma.append(q)
        assert sorted(sigma) == list(range(reps))                     # a bijection of replications
        assert sigma == list(perm.permutation(9, 4, s, reps))


def test_replication_shuffle_is_uniform_over_orderings():
    reps, draws = 3, 6000
    seen = Counter()
    for s in range(draws):
        src = perm.replication_source_rows(1, 0, s, reps * 2, reps, perm.REPLICATIONS)
        seen[tuple(int(src[r * 2]) // 2 for r in range(reps))] += 1
    assert len(seen) == math.factorial(reps)
    exp = draws / 6
    stat = sum((v - exp) ** 2 / exp for v in seen.values())
    assert chi2.sf(stat, 5) > 1e-3


@pytest.mark.parametrize("reps,n_r", [(2, 9), (4, 4), (3, 1000)])
def test_within_shuffle_keeps_rows_in_their_trial(reps, n_r):
    src = perm.replication_source_rows(2, 7, 3, reps * n_r, reps, perm.WITHIN).astype(np.int64)
    bl, _ = blocks(src, reps)
    for r, b in enumerate(bl):
        assert sorted(b.tolist()) == list(range(r * n_r, (r + 1) * n_r))
    if n_r > 3:
        # trials draw different permutations
        rel = [tuple(b - r * n_r) for r, b in enumerate(bl)]
        assert len(set(rel)) == reps


def test_within_shuffle_is_uniform_per_trial():
    reps, n_r, draws = 2, 4, 4800
    seen = [Counter(), Counter()]
    for s in range(draws):
        src = perm.replication_source_rows(5, 1, s, reps * n_r, reps, perm.WITHIN).astype(np.int64)
        for r in range(reps):
            seen[r][tuple(src[r * n_r:(r + 1) * n_r] - r * n_r)] += 1
    for c in seen:
        assert len(c) == 24
        exp = draws / 24
        stat = sum((v - exp) ** 2 / exp for v in c.values())
        assert chi2.sf(stat, 23) > 1e-3


def test_one_replication_is_the_plain_permutation():
    for n in (1, 2, 17, 1000):
        assert np.array_equal(perm.replication_source_rows(3, 2, 1, n, 1, perm.WITHIN),
                              perm.permutation(3, 2, 1, n))


def test_shuffle_mode_rule():
    assert perm.shuffle_mode(1, 2) == perm.WITHIN
    assert perm.shuffle_mode(3, 6) == perm.REPLICATIONS        # 3! = 6 orderings for 6 surrogates
    assert perm.shuffle_mode(3, 7) == perm.WITHIN
    assert perm.shuffle_mode(5, 200) == perm.WITHIN            # 120 < 200
    assert perm.shuffle_mode(6, 200) == perm.REPLICATIONS      # 720 >= 200
    assert perm.shuffle_mode(30, 10 ** 6) == perm.REPLICATIONS


def test_rows_must_split_into_replications():
    with pytest.raises(ValueError):
        perm.replication_source_rows(0, 0, 0, 10, 3, perm.WITHIN)


def test_greedy_over_replications_recovers_a_coupling():
    # 6 trials of 120 samples: the coupling 0 -> 1 at lag 2 holds in every trial
    g = np.random.default_rng(4)
    reps, t = 6, 125
    s = np.zeros((reps, 3, t))
    s[:, 0] = g.standard_normal((reps, t))
    s[:, 2] = g.standard_normal((reps, t))
    s[:, 1, 2:] = 0.9 * s[:, 0, :-2] + 0.3 * g.standard_normal((reps, t - 2))
    s = s.astype(np.float32)
    res = greedy.select_sources(s, 1, [0, 2], max_lag_sources=3, max_lag_target=2, alpha=0.05,
                                k=4, n_surr=30, seed=1, estimator=lambda x, y, z, k: cksg.cmi_ksg(x, y, z, k))
    assert [(n, l) for (n, l, _, _) in res["sources"]] == [(0, 2)]
    assert res["significant"]


def test_replication_surrogates_destroy_a_cross_trial_free_coupling():
    # independent trials: the replication-shuffled null matches the real value's law
    g = np.random.default_rng(8)
    hits = 0
    for rep in range(5):
        s = g.standard_normal((8, 2, 130)).astype(np.float32)
        res = greedy.select_sources(s, 0, [1], max_lag_sources=2, max_lag_target=1, alpha=0.05, k=4, n_surr=40,
                                    seed=rep, estimator=lambda x, y, z, k: cksg.cmi_ksg(x, y, z, k))
        hits += len(res["sources"]) > 0
    assert hits <= 1
