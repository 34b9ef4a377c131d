"""Replication (trial) surrogates on the GPU against the oracle: estimates and
surrogates pooled over R replications with both shuffle modes on both exact
paths, the greedy search over [R][P][T] data (KSG with replication and
within-trial surrogates, and the Gaussian estimator), and network inference
over replications."""

import sys

import numpy as np
import pytest

import paper_1902_06828_amd as mte
import synth
from oracle import cksg, gauss, greedy, network, perm

pytestmark = pytest.mark.gpu

TOL = 1e-9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def est(x, y, z, k):
    return cksg.cmi_ksg(x, y, z, k)


def trial_data(g, n, R, dz):
    """X drives Y within each trial, Z is a shared common input."""
    z = g.standard_normal((max(dz, 1), n)).astype(np.float32)
    x = (g.standard_normal((1, n)) + 0.5 * z[0]).astype(np.float32)
    y = (0.6 * x + 0.4 * z[0] + g.standard_normal((1, n))).astype(np.float32)
    return x, y, (z[:dz] if dz else None)


@pytest.mark.parametrize("path", ["list", "brute"])
@pytest.mark.parametrize("n,R,dz,mode,S", [
    (2400, 8, 2, "replications", 20), (2400, 8, 2, "within", 20), (1001, 7, 0, "replications", 12),
    (6000, 6, 3, "within", 8), (777, 3, 1, "auto", 10),
])
def test_replication_surrogates_match_oracle(monkeypatch, path, n, R, dz, mode, S):
    monkeypatch.setenv("MTE_FORCE_MODE", path)
    say("replication surrogates", path, n, R, dz, mode, S)
    g = np.random.default_rng(n + R + dz)
    x, y, z = trial_data(g, n, R, dz)
    real, surr = mte.cmi_ksg_surrogates_rep(x, y, z, k=4, S=S, R=R, seed=3, cand=9, mode=mode)
    m = perm.shuffle_mode(R, S) if mode == "auto" else mode
    assert abs(real - est(x, y, z, 4)) <= TOL
    for s in range(S):
        src = perm.replication_source_rows(3, 9, s, n, R, m)
        want = est(np.ascontiguousarray(x[:, src]), y, z, 4)
        assert abs(surr[s] - want) <= TOL, s
    # replication surrogates break the X -> Y coupling
    assert np.all(surr < real)


def test_one_replication_equals_plain_surrogates():
    g = np.random.default_rng(1)
    x, y, z = trial_data(g, 900, 1, 2)
    real, surr = mte.cmi_ksg_surrogates_rep(x, y, z, k=4, S=10, R=1, seed=5, cand=0, mode="within")
    real2, surr2 = mte.cmi_ksg_surrogates(x, y, z, k=4, S=10, seed=5)
    assert real == real2 and np.array_equal(surr, surr2)


def _vars(lst):
    return [(n, l) for (n, l, _, _) in lst]


def _same(lib_res, ora):
    for key in ("target_past", "sources"):
        assert _vars(lib_res[key]) == _vars(ora[key])
        for v, w in zip(lib_res[key], ora[key]):
            assert abs(v[2] - w[2]) <= TOL and v[3] == w[3]
    assert lib_res["significant"] == ora["significant"]
    assert abs(lib_res["omnibus_te"] - ora["omnibus_te"]) <= TOL
    assert lib_res["omnibus_p"] == ora["omnibus_p"]
    assert lib_res["n_estimates"] == ora["n_estimates"]


@pytest.mark.parametrize("R,S", [(6, 20), (3, 20)])      # 6! >= 20: replications; 3! < 20: within
def test_greedy_over_replications_matches_oracle(R, S):
    series, _ = synth.var_network_trials(3, 150, R, seed=5)
    say("greedy replications", R, S, perm.shuffle_mode(R, S))
    kw = dict(max_lag_sources=3, max_lag_target=2, alpha=0.1, k=4, seed=2)
    got = mte.mte_select_sources(series, 0, [1, 2], S=S, **kw)
    want = greedy.select_sources(series, 0, [1, 2], n_surr=S, estimator=est, **kw)
    _same(got, want)


def test_gauss_greedy_over_replications_matches_oracle():
    series, _ = synth.var_network_trials(5, 400, 5, seed=1)
    got = mte.mte_select_sources(series, 0, [1, 2, 3, 4], max_lag_sources=3, max_lag_target=3, alpha=0.05,
                                 estimator="gauss")
    want = greedy.select_sources(series, 0, [1, 2, 3, 4], max_lag_sources=3, max_lag_target=3, alpha=0.05,
                                 null="analytic")
    for key in ("target_past", "sources"):
        assert _vars(got[key]) == _vars(want[key])
        for v, w in zip(got[key], want[key]):
            assert abs(v[2] - w[2]) <= TOL
            assert v[3] == pytest.approx(w[3], rel=1e-6, abs=1e-12)
    assert abs(got["omnibus_te"] - want["omnibus_te"]) <= TOL


def test_network_over_replications_matches_oracle():
    series, links = synth.var_network_trials(4, 130, 5, seed=3)
    kw = dict(max_lag_sources=2, max_lag_target=2, alpha=0.1, k=4, seed=7)
    say("network replications, 4 nodes, R=5")
    adj, summ = mte.mte_infer_network(series, alpha_fdr=0.1, S=20, **kw)
    ref_adj, ref_res, ref_keep = network.infer_network(series, alpha_fdr=0.1, n_surr=20, estimator=est, **kw)
    assert np.array_equal(adj, ref_adj)
    for t, (s, r) in enumerate(zip(summ, ref_res)):
        assert s["omnibus_p"] == r["omnibus_p"] and bool(s["significant"]) == r["significant"]
        assert abs(s["omnibus_te"] - r["omnibus_te"]) <= TOL
        assert s["n_estimates"] == r["n_estimates"]
        assert bool(s["fdr_kept"]) == bool(ref_keep[t])
