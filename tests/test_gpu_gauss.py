"""Gaussian estimator on the GPU against the oracle (oracle/gauss.py): the
float64 covariance, I(X;Y|Z) and its analytic p-value at small and large N
(several row chunks, ragged tails, several Gram tiles), the equality of an
estimate taken from a small and from a large covariance matrix, the error on
a singular block, the greedy search with the analytic null (direct and
served) and network inference on the linear VAR, where the paper uses this
estimator."""

import sys

import numpy as np
import pytest
import torch

import paper_1902_06828_amd as mte
import synth
from oracle import gauss, greedy, network

pytestmark = pytest.mark.gpu

TOL = 1e-9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed(g, d, n, base=None):
    """d correlated float32 columns of n rows: a random linear mix of d+2
    independent normals, plus half of the first column of `base` (to make
    the sets dependent) and offsets (so the two-pass centering matters)."""
    v = g.standard_normal((d, d + 2)) @ g.standard_normal((d + 2, n))
    if base is not None:
        v = v + 0.5 * base[0].astype(np.float64)
    v += g.uniform(-30, 30, (d, 1))
    return v.astype(np.float32)


CASES = [
    (1, 1, 0, 2000), (1, 1, 1, 257), (2, 3, 5, 1000), (1, 1, 4, 65537), (4, 2, 10, 70001),
    (16, 8, 31, 3000), (1, 1, 62, 5000), (3, 1, 2, 300000),
]


@pytest.mark.parametrize("dx,dy,dz,n", CASES)
def test_cmi_gauss_matches_oracle(dx, dy, dz, n):
    say("cmi_gauss", dx, dy, dz, n)
    g = np.random.default_rng(dx * 1000 + dy * 100 + dz + n)
    z = mixed(g, dz, n) if dz else None
    y = mixed(g, dy, n, base=z)
    x = mixed(g, dx, n, base=y)
    got, p = mte.cmi_gauss(x, y, z)
    want = gauss.cmi_gauss(x, y, z)
    assert abs(got - want) <= TOL, (got, want)
    wp = gauss.p_value(want, n, dx * dy)
    assert p == pytest.approx(wp, rel=1e-6, abs=1e-12)


def test_cmi_gauss_independent_near_zero_and_p_uniformish():
    g = np.random.default_rng(5)
    ps = []
    for r in range(40):
        x, y, z = (g.standard_normal((1, 500)).astype(np.float32) for _ in range(3))
        got, p = mte.cmi_gauss(x, y, z)
        want = gauss.cmi_gauss(x, y, z)
        assert abs(got - want) <= TOL
        assert p == pytest.approx(gauss.p_value(want, 500, 1), rel=1e-6)
        ps.append(p)
    ps = np.array(ps)
    assert 0.15 < ps.mean() < 0.85 and ps.min() > 1e-4


def test_covariance_matches_oracle_across_tiles():
    g = np.random.default_rng(11)
    for d, n, ld in [(1, 2, 2), (65, 1001, 1003), (130, 70001, 70001), (200, 4097, 4100)]:
        say("covariance", d, n, ld)
        v = np.zeros((d, ld), np.float32)
        v[:, :n] = mixed(g, d, n)
        V = torch.from_numpy(v).cuda()
        cov = torch.empty((d, d), dtype=torch.float64, device="cuda")
        mte.mte_gauss_covariance_dev(V, cov, n=n)
        torch.cuda.synchronize()
        got = cov.cpu().numpy()
        want = gauss.covariance(v[:, :n])
        assert np.array_equal(got, got.T)
        scale = np.sqrt(np.outer(np.diag(want), np.diag(want)))
        assert np.max(np.abs(got - want) / scale) < 1e-12


def test_estimate_from_large_matrix_is_bitwise_the_small_one():
    g = np.random.default_rng(3)
    n, d = 20000, 100
    v = mixed(g, d, n)
    V = torch.from_numpy(v).cuda()
    cov = torch.empty((d, d), dtype=torch.float64, device="cuda")
    mte.mte_gauss_covariance_dev(V, cov)
    sets = [([5], [0], [1, 2, 3]), ([70, 71], [99], [64, 3, 40]), ([7], [8], [])]
    got = mte.mte_gauss_cmi_sets(cov, sets)
    for (xs, ys, zs), gv in zip(sets, got):
        small, _ = mte.cmi_gauss(v[xs], v[ys], v[zs] if zs else None)
        assert gv == small
        assert abs(gv - gauss.cmi_gauss(v[xs], v[ys], v[zs] if zs else None)) <= TOL


def test_singular_block_is_an_error():
    g = np.random.default_rng(1)
    x = g.standard_normal((1, 400)).astype(np.float32)
    y = g.standard_normal((1, 400)).astype(np.float32)
    z = np.full((1, 400), 2.5, np.float32)                # constant: zero variance
    with pytest.raises(mte.MteError, match="positive definite"):
        mte.cmi_gauss(x, y, z)


def _vars(lst):
    return [(n, l) for (n, l, _, _) in lst]


@pytest.mark.parametrize("target", [0, 3])
def test_greedy_analytic_matches_oracle(target):
    series, _ = synth.var_network(5, 2000, seed=1)
    cands = [j for j in range(5) if j != target]
    say("greedy gauss, target", target)
    got = mte.mte_select_sources(series, target, cands, max_lag_sources=3, max_lag_target=3, alpha=0.05,
                                 estimator="gauss")
    want = greedy.select_sources(series, target, cands, max_lag_sources=3, max_lag_target=3, alpha=0.05,
                                 null="analytic")
    for key in ("target_past", "sources"):
        assert _vars(got[key]) == _vars(want[key])
        for v, w in zip(got[key], want[key]):
            assert abs(v[2] - w[2]) <= TOL
            assert v[3] == pytest.approx(w[3], rel=1e-6, abs=1e-12)
    assert got["significant"] == want["significant"]
    assert abs(got["omnibus_te"] - want["omnibus_te"]) <= TOL
    assert got["omnibus_p"] == pytest.approx(want["omnibus_p"], rel=1e-6, abs=1e-12)
    assert got["n_estimates"] == want["n_estimates"]
    # served form: same bits
    sid = mte.mte_series_register(series)
    try:
        srv = mte.mte_select_sources_sid(sid, target, cands, max_lag_sources=3, max_lag_target=3, alpha=0.05,
                                         estimator="gauss")
    finally:
        mte.mte_series_release(sid)
    for key in ("target_past", "sources", "omnibus_te", "omnibus_p", "n_estimates"):
        assert srv[key] == got[key]


def test_network_gauss_recovers_var_and_matches_oracle():
    series, links = synth.var_network(10, 3000, seed=0)
    truth = synth.truth_adjacency(10, links)
    say("network gauss, 10 nodes, T=3000")
    adj, summ = mte.mte_infer_network(series, max_lag_sources=5, alpha=0.05, alpha_fdr=0.05, estimator="gauss")
    ref_adj, ref_res, ref_keep = network.infer_network(series, alpha=0.05, alpha_fdr=0.05, null="analytic")
    assert np.array_equal(adj, ref_adj)
    for s, r in zip(summ, ref_res):
        assert abs(s["omnibus_te"] - r["omnibus_te"]) <= TOL
        assert s["omnibus_p"] == pytest.approx(r["omnibus_p"], rel=1e-6, abs=1e-12)
        assert s["n_estimates"] == r["n_estimates"]
    m = mte.mte_link_metrics(adj, truth)
    say("metrics", m)
    assert m["precision"] == 1.0 and m["recall"] == 1.0
