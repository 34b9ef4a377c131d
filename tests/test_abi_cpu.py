"""Host-side checks of libmte.so that need no GPU: every symbol declared in
include/mte.h is exported, the host implementation of the surrogate
permutation and the significance tests agree with the oracle, and invalid
arguments are rejected before any device work."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_1902_06828_amd as mte
from oracle import perm, stats

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mte.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "cmi_ksg" in names and "mte_select_sources" in names and "mte_submit" in names
    L = ctypes.CDLL(os.path.join(ROOT, "paper_1902_06828_amd", "libmte.so"))
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(mte._lib.SIGNATURES) | {"mte_last_error"} >= set(names)


def test_abi_version():
    assert mte.lib().mte_abi_version() == 7


@pytest.mark.parametrize("n", [1, 2, 3, 5, 64, 100, 1000, 4097, 10000])
def test_host_permutation_matches_oracle(n):
    for (seed, cand, s) in [(0, 0, 0), (123, 7, 199), (2 ** 64 - 1, 2 ** 32 - 1, 2 ** 31)]:
        assert np.array_equal(mte.mte_permutation(seed, cand, s, n), perm.permutation(seed, cand, s, n))


def test_statistics_match_oracle():
    g = np.random.default_rng(3)
    for trial in range(300):
        n = int(g.integers(1, 7))
        S = int(g.integers(21, 60))
        alpha = float(g.choice([0.05, 0.1, 0.2]))
        real = g.random(n)
        surr = g.random((n, S))
        if trial % 3 == 0:              # ties between candidates and surrogates
            real = np.round(real * 4) / 4
            surr = np.round(surr * 4) / 4
        assert mte.mte_max_statistic(real, surr, alpha) == stats.max_statistic(real, surr, alpha)
        assert mte.mte_min_statistic(real, surr, alpha) == stats.min_statistic(real, surr, alpha)
        assert mte.mte_omnibus(real[0], surr[0], alpha) == stats.omnibus(real[0], surr[0], alpha)


def test_statistics_reject_too_few_surrogates():
    with pytest.raises(mte.MteError) as e:
        mte.mte_max_statistic([0.1], np.zeros((1, 20)), 0.05)
    assert e.value.code == mte._lib.MTE_EINVAL


@pytest.mark.parametrize("kw", [dict(k=0), dict(k=17), dict(n=4, k=4), dict(dx=17), dict(dy=9),
                                dict(dz=32)])
def test_estimator_argument_validation(kw):
    n = kw.get("n", 50)
    k = kw.get("k", 4)
    X = np.zeros((kw.get("dx", 1), n), np.float32)
    Y = np.zeros((kw.get("dy", 1), n), np.float32)
    Z = np.zeros((kw.get("dz", 1), n), np.float32)
    with pytest.raises(mte.MteError) as e:
        mte.cmi_ksg(X, Y, Z, k)
    assert e.value.code == mte._lib.MTE_EINVAL


def test_non_finite_inputs_rejected():
    X = np.zeros((1, 50), np.float32)
    X[0, 7] = np.nan
    with pytest.raises(mte.MteError) as e:
        mte.cmi_ksg(X, np.zeros((1, 50), np.float32), None, 4)
    assert e.value.code == mte._lib.MTE_EINVAL and "not finite" in str(e.value)


def test_greedy_argument_validation():
    data = np.zeros((3, 100), np.float32)
    with pytest.raises(mte.MteError):
        mte.mte_select_sources(data, 0, [1, 2], alpha=0.05, S=20)     # S*alpha <= 1
    with pytest.raises(mte.MteError):
        mte.mte_select_sources(data, 0, [0, 1], alpha=0.1, S=20)      # target among candidates
    with pytest.raises(mte.MteError):
        mte.mte_select_sources(data, 0, [5], alpha=0.1, S=20)         # node out of range
    with pytest.raises(mte.MteError):
        mte.mte_select_sources(data[:, :8], 0, [1], alpha=0.1, S=20)  # series too short


def test_autocorr_decay_time_matches_oracle():
    # the library's host computation takes the oracle's decisions on float32 series
    from oracle import act
    g = np.random.default_rng(9)
    for phi, n in [(0.8, 20000), (0.95, 5000), (0.3, 3000), (0.0, 500)]:
        e = g.standard_normal(n)
        x = np.empty(n)
        x[0] = e[0]
        for i in range(1, n):
            x[i] = phi * x[i - 1] + e[i]
        x32 = x.astype(np.float32)
        assert mte.mte_autocorr_decay_time(x32, 60) == act.decay_time(x32.astype(np.float64), 60)
    t = np.arange(5000)
    s = np.sin(2 * np.pi * t / 50).astype(np.float32)
    assert mte.mte_autocorr_decay_time(s, 50) == act.decay_time(s.astype(np.float64), 50) == 10


def test_theiler_argument_validation():
    x, y, z = (np.random.default_rng(1).standard_normal((1, 20)).astype(np.float32) for _ in range(3))
    with pytest.raises(mte.MteError) as e:
        mte.cmi_ksg_diag(x, y, z, 4, 0, 0, 0, theiler=8)
    assert e.value.code == mte._lib.MTE_EINVAL
    with pytest.raises(mte.MteError) as e:
        mte.cmi_ksg_diag(x, y, z, 4, 0, 0, 0, theiler=-1)
    assert e.value.code == mte._lib.MTE_EINVAL
    with pytest.raises(mte.MteError):
        mte.mte_autocorr_decay_time(np.zeros(1, np.float32), 5)


def test_fdr_bh_matches_oracle():
    g = np.random.default_rng(4)
    for m in (1, 5, 40, 200):
        for q in (0.01, 0.05, 0.2):
            p = np.concatenate([g.random(m // 2) * 0.02, g.random(m - m // 2)])
            p[g.integers(0, m, size=m // 5)] = 0.0           # ties, as from permutation tests
            assert np.array_equal(mte.mte_fdr_bh(p, q), stats.benjamini_hochberg(p, q))
    with pytest.raises(mte.MteError):
        mte.mte_fdr_bh([0.5, 1.5], 0.05)


def test_link_metrics_matches_oracle():
    from oracle import network
    g = np.random.default_rng(5)
    for P in (2, 7, 30):
        a = (g.random((P, P)) < 0.3).astype(np.uint8)
        b = (g.random((P, P)) < 0.2).astype(np.uint8)
        got, ref = mte.mte_link_metrics(a, b), network.link_metrics(a, b)
        for key in ("tp", "fp", "tn", "fn"):
            assert got[key] == ref[key]
        for key in ("precision", "recall", "specificity", "fpr"):
            assert (np.isnan(got[key]) and np.isnan(ref[key])) or got[key] == ref[key]


def test_chi2_survival_matches_scipy():
    # The analytic null of the Gaussian estimator: the library's finite
    # incomplete-gamma series against scipy's independent implementation.
    from scipy.stats import chi2
    for dof in list(range(1, 41)) + [64, 127, 128]:
        for x in [1e-8, 1e-3, 0.5, 1.0, 3.84, 10.0, 47.3, 150.0, 600.0, 1300.0]:
            got, want = mte.mte_chi2_sf(x, dof), float(chi2.sf(x, dof))
            if want > 1e-280:
                assert got == pytest.approx(want, rel=1e-10, abs=0), (dof, x)
            else:
                assert got < 1e-270, (dof, x)
    assert mte.mte_chi2_sf(0.0, 3) == 1.0
    assert mte.mte_chi2_sf(-1.0, 1) == 1.0
    with pytest.raises(mte.MteError):
        mte.mte_chi2_sf(1.0, 0)


def test_gauss_argument_validation():
    g = np.random.default_rng(0)
    x = g.standard_normal((1, 50)).astype(np.float32)
    with pytest.raises(mte.MteError):
        mte.cmi_gauss(x, x, np.zeros((63, 50), np.float32))     # 65 variables
    with pytest.raises(mte.MteError):
        mte.cmi_gauss(x[:, :1], x[:, :1])                       # N = 1
    bad = x.copy()
    bad[0, 3] = np.inf
    with pytest.raises(mte.MteError):
        mte.cmi_gauss(bad, x)
    s = g.standard_normal((3, 200)).astype(np.float32)
    with pytest.raises(mte.MteError, match="Theiler"):
        mte.mte_select_sources(s, 0, [1, 2], estimator="gauss", theiler=2)
    with pytest.raises(ValueError):
        mte.mte_select_sources(s, 0, [1, 2], estimator="nope")


@pytest.mark.parametrize("n,R", [(12, 3), (1000, 8), (999, 27), (7, 7), (4096, 1), (5000, 2)])
def test_replication_permutation_matches_oracle(n, R):
    from oracle import perm
    for mode in ("within", "replications"):
        if mode == "replications" and R < 2:
            continue
        for s in range(3):
            got = mte.mte_permutation_rep(11, 5, s, n, R, mode)
            want = perm.replication_source_rows(11, 5, s, n, R, mode)
            assert np.array_equal(got, want), (mode, s)


def test_shuffle_mode_matches_oracle():
    from oracle import perm
    for R in range(1, 12):
        for S in (1, 2, 6, 7, 24, 100, 200, 1000, 10 ** 6):
            assert mte.mte_shuffle_mode(R, S) == perm.shuffle_mode(R, S), (R, S)


def test_replication_argument_validation():
    g = np.random.default_rng(2)
    x = g.standard_normal((1, 100)).astype(np.float32)
    with pytest.raises(mte.MteError):
        mte.cmi_ksg_surrogates_rep(x, x, None, S=10, R=3)          # 100 rows do not split into 3
    with pytest.raises(mte.MteError):
        mte.mte_permutation_rep(0, 0, 0, 10, 1, "replications")      # needs R >= 2
    s = g.standard_normal((4, 3, 60)).astype(np.float32)
    with pytest.raises(mte.MteError, match="Theiler"):
        mte.mte_select_sources(s, 0, [1, 2], max_lag_sources=2, max_lag_target=2, S=40, theiler=1)


def test_standardise_matches_oracle():
    from oracle import greedy
    g = np.random.default_rng(9)
    s = (g.standard_normal((5, 2003)) * 3 + 11).astype(np.float32)
    s[2] = -1.5                                     # constant node
    assert np.array_equal(mte.mte_standardise(s).view(np.uint32), greedy.standardise(s).view(np.uint32))
    r = (g.standard_normal((3, 4, 700)) * 0.01).astype(np.float32)
    assert np.array_equal(mte.mte_standardise(r).view(np.uint32), greedy.standardise(r).view(np.uint32))


def test_tune_report_without_a_device():
    # no call has run on a device, so the report holds no choice; the length
    # is returned without a buffer, and a buffer size without a buffer is refused
    assert mte.mte_tune_report() == []
    import ctypes
    n = ctypes.c_size_t(99)
    assert mte.lib().mte_tune_report(None, 0, ctypes.byref(n)) == 0 and n.value == 0
    assert mte.lib().mte_tune_report(None, 4, ctypes.byref(n)) == mte._lib.MTE_EINVAL
