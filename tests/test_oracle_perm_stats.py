"""Pins for the oracle's surrogate permutations (oracle/perm.py) and its
significance tests (oracle/stats.py)."""

import itertools
import math

import numpy as np
import pytest

import synth
from oracle import perm, stats


# ---------------------------------------------------------------- SplitMix64
def test_splitmix64_published_outputs():
    # the first outputs of SplitMix64 started at state 0, as listed with the
    # generator's reference implementation (Steele, Lea and Flood; Vigna)
    assert perm.splitmix64(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert perm.splitmix64(0, 1)[0] == 16294208416658607535


def _inverse(y, keys, n):
    # every swap-or-not round is an involution, so running the rounds in
    # reverse order undoes the permutation
    for rk, k in reversed(keys):
        yp = k - y if y <= k else k - y + n
        if perm.mix64(max(y, yp) ^ rk) >> 63:
            y = yp
    return y


def test_rounds_are_involutions_and_invert():
    for n in (1, 2, 3, 10, 97):
        keys = perm.round_keys(7, 3, 11, n)
        p = perm.permutation_scalar(7, 3, 11, n)
        assert all(_inverse(p[i], keys, n) == i for i in range(n))
        assert all(0 <= k < n for _, k in keys)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 16, 17, 100, 255, 256, 257, 1000, 4097])
def test_permutation_is_a_bijection(n):
    for (seed, cand, s) in [(0, 0, 0), (1, 2, 3), (2 ** 63 + 5, 2 ** 31, 2 ** 32 - 1)]:
        p = perm.permutation(seed, cand, s, n)
        assert sorted(p.tolist()) == list(range(n))
        if n <= 300:
            assert p.tolist() == perm.permutation_scalar(seed, cand, s, n)


def test_round_count():
    assert [perm.n_rounds(n) for n in (1, 2, 16, 17, 10000, 2 ** 20 + 1)] == [24, 24, 24, 30, 84, 126]


def test_permutations_look_uniform():
    # all 24 orderings of 4 items over many keys: chi-square with 23 d.o.f.
    counts = {}
    trials = 24 * 400
    for s in range(trials):
        key = tuple(perm.permutation(99, 5, s, 4).tolist())
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 24
    exp = trials / 24
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    assert chi2 < 60          # the 0.9999 quantile of chi2(23) is about 56.8
    # and all 120 orderings of 5 items: chi-square with 119 d.o.f.
    counts = {}
    trials = 120 * 150
    for s in range(trials):
        key = tuple(perm.permutation(42, 9, s, 5).tolist())
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 120
    exp = trials / 120
    assert sum((c - exp) ** 2 / exp for c in counts.values()) < 185   # 0.9999 quantile ~ 181
    # position marginals for n = 10
    m = np.zeros((10, 10))
    for s in range(2000):
        p = perm.permutation(3, 1, s, 10)
        m[np.arange(10), p] += 1
    assert np.all(np.abs(m / 2000 - 0.1) < 0.035)


def test_keys_differ_between_tests_and_surrogates():
    a = perm.permutation(5, 0, 0, 1000)
    assert not np.array_equal(a, perm.permutation(5, 0, 1, 1000))
    assert not np.array_equal(a, perm.permutation(5, 1, 0, 1000))
    assert not np.array_equal(a, perm.permutation(6, 0, 0, 1000))


# ---------------------------------------------------------------- tests
def test_max_statistic_table1_example():
    # three candidates, S = 10 surrogates (Table 1 layout): I* = 0.30 from
    # candidate 1; the column maxima exceed 0.30 in columns 2 and 7 only
    real = [0.10, 0.30, 0.20]
    surr = np.full((3, 10), 0.05)
    surr[0, 2] = 0.31
    surr[2, 7] = 0.45
    surr[1, 4] = 0.30          # equal, not larger: not counted
    j, p, sig = stats.max_statistic(real, surr, alpha=0.25)
    assert j == 1 and p == pytest.approx(0.2) and sig
    j, p, sig = stats.max_statistic(real, surr, alpha=0.2)
    assert not sig             # p must be strictly smaller than alpha


def test_min_statistic_example():
    real = [0.10, 0.30, 0.05]
    surr = np.full((3, 10), 0.20)
    surr[:, :3] = 0.01         # three columns whose minimum is below 0.05
    j, p, sig = stats.min_statistic(real, surr, alpha=0.5)
    assert j == 2 and p == pytest.approx(0.7) and not sig


def test_ties_take_the_first_candidate():
    j, _, _ = stats.max_statistic([0.2, 0.5, 0.5], np.zeros((3, 20)), 0.1)
    assert j == 1
    j, _, _ = stats.min_statistic([0.2, 0.1, 0.1], np.zeros((3, 20)), 0.1)
    assert j == 1


def test_surrogate_count_must_exceed_inverse_alpha():
    with pytest.raises(ValueError):
        stats.max_statistic([0.1], np.zeros((1, 20)), 0.05)
    stats.max_statistic([0.1], np.zeros((1, 21)), 0.05)


def test_max_statistic_size_under_complete_null():
    # real and surrogate estimates i.i.d.: the real maximum's rank among S+1
    # column maxima is uniform, so P(p < alpha) = ceil(alpha*S)/(S+1)
    g = np.random.default_rng(0)
    n_cand, n_surr, alpha, trials = 4, 50, 0.1, 20000
    hits = 0
    for _ in range(trials):
        v = g.random((n_cand, n_surr + 1))
        hits += stats.max_statistic(v[:, 0], v[:, 1:], alpha)[2]
    expect = math.ceil(alpha * n_surr) / (n_surr + 1)
    sd = math.sqrt(expect * (1 - expect) / trials)
    assert abs(hits / trials - expect) < 4 * sd


def test_exact_size_by_enumeration():
    # S = 4, alpha = 0.3: over all (S+1)! equally likely orderings of the real
    # and surrogate maxima, the test rejects in ceil(1.2)/5 = 2/5 of them
    rej = 0
    for order in itertools.permutations(range(5)):
        real = [float(order[0])]
        surr = np.array([[float(o) for o in order[1:]]])
        rej += stats.max_statistic(real, surr, 0.3)[2]
    assert rej * 5 == 2 * math.factorial(5)


def test_sidak_forms():
    # Family-wise error rate correction section
    for alpha in (0.05, 0.01, 0.001):
        for n in (1, 5, 50):
            v = stats.sidak_variable_fpr(alpha, n)
            assert abs(1 - (1 - v) ** n - alpha) < 1e-14      # defining relation
            assert v >= alpha / n - 1e-16                   # Bonferroni lower bound
            assert abs(v - alpha / n) < alpha ** 2          # first-order Taylor term
            t = stats.target_fpr(alpha, n)
            assert abs(t - sum(alpha ** j for j in range(1, n + 1))) < 1e-15
            assert abs(t - alpha) <= alpha ** 2 / (1 - alpha) + 1e-16
    # Monte Carlo: threshold set so that P(max of n uniforms > th) = alpha
    g = np.random.default_rng(1)
    alpha, n = 0.05, 10
    th = (1 - alpha) ** (1 / n)
    u = g.random((200000, n))
    assert abs(np.mean(u.max(1) > th) - alpha) < 0.003
    assert abs(np.mean(u[:, 0] > th) - stats.sidak_variable_fpr(alpha, n)) < 0.001


def test_omnibus_and_bh():
    p, sig = stats.omnibus(0.5, np.linspace(0, 1, 101)[1:], 0.6)
    assert p == pytest.approx(0.5) and sig
    keep = stats.benjamini_hochberg([0.01, 0.04, 0.03, 0.005], 0.05)
    assert keep.tolist() == [True, True, True, True]
    keep = stats.benjamini_hochberg([0.01, 0.2, 0.03, 0.005], 0.05)
    assert keep.tolist() == [True, False, True, True]


def test_link_metrics_hand_example():
    # 3 nodes; truth 0->1, 1->2; inferred 0->1, 2->0
    from oracle import network
    truth = np.zeros((3, 3), np.uint8)
    truth[0, 1] = truth[1, 2] = 1
    inf = np.zeros((3, 3), np.uint8)
    inf[0, 1] = inf[2, 0] = 1
    m = network.link_metrics(inf, truth)
    assert (m["tp"], m["fp"], m["tn"], m["fn"]) == (1, 1, 3, 1)
    assert m["precision"] == 0.5 and m["recall"] == 0.5 and m["specificity"] == 0.75 and m["fpr"] == 0.25
    assert np.array_equal(synth.truth_adjacency(3, [(1, 0, 2, 0.3), (2, 1, 1, 0.2)]), truth)
