"""Network-level inference on the GPU: every target's greedy selection through
the request loop, the Benjamini-Hochberg correction over omnibus p-values and
the inferred adjacency, against the oracle; recovery of known VAR and CLM
networks; and the false positive rate on empty networks (Validation of false
positive rate: the fraction of targets with any inferred source stays near
alpha)."""

import sys

import numpy as np
import pytest

import paper_1902_06828_amd as mte
import synth
from oracle import cksg, network

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_network_matches_oracle():
    series, links = synth.var_network(4, 300, seed=8)
    kw = dict(max_lag_sources=2, max_lag_target=2, alpha=0.1, k=4, seed=11)
    say("network parity, 4 nodes")
    adj, summ = mte.mte_infer_network(series, alpha_fdr=0.1, S=20, **kw)
    ref_adj, ref_res, ref_keep = network.infer_network(series, alpha_fdr=0.1, n_surr=20, estimator=cksg.cmi_ksg,
                                                       **kw)
    assert np.array_equal(adj, ref_adj)
    for t, (s, r) in enumerate(zip(summ, ref_res)):
        assert s["omnibus_p"] == r["omnibus_p"] and bool(s["significant"]) == r["significant"]
        assert abs(s["omnibus_te"] - r["omnibus_te"]) <= 1e-9
        assert s["n_sources"] == len(r["sources"]) and s["n_target_past"] == len(r["target_past"])
        assert bool(s["fdr_kept"]) == bool(ref_keep[t])
        assert s["n_estimates"] == r["n_estimates"]


def test_network_recovers_var_links():
    # the benchmark's 10-node VAR at T = 10000.  The paper reports high precision
    # and recall at T = 10000; here the KSG search finds about half of the 26
    # links (those with the smallest rescaled coefficients stay below what
    # S = 100 surrogates detect), with no false link.  The Gaussian estimator
    # finds all of them (tests/test_gpu_gauss.py).
    series, links = synth.var_network(10, 10000, seed=2)
    truth = synth.truth_adjacency(10, links)
    say("network recovery, 10 nodes, links", int(truth.sum()))
    adj, summ = mte.mte_infer_network(series, max_lag_sources=5, alpha=0.05, alpha_fdr=0.05, S=100, seed=4)
    m = mte.mte_link_metrics(adj, truth)
    say("metrics", m)
    assert m["precision"] >= 0.8 and m["recall"] >= 0.4
    assert m == network.link_metrics(adj, truth)


def test_network_recovers_paper_clm_links():
    # The paper's own KSG workload (CLM section): coupled logistic maps on a
    # 10-node Erdos-Renyi network (expected in-degree 3), T = 10000, k = 4,
    # with its significance level alpha = 0.001.  The paper states S > 1/alpha
    # surrogates and runs S = 1000 at alpha = 0.001, on the boundary of that
    # rule; 1001 meets it.  The paper reports precision, recall and
    # specificity above 98% on average at T = 10000 (Results, influence of
    # network size and length of the time series); one network of 28 links
    # allows no missed and no false link at that level, so the thresholds
    # leave room for one of each.
    series, links = synth.paper_clm_network(10, 10000, seed=1)
    truth = synth.truth_adjacency(10, links)
    say("CLM recovery, 10 nodes, links", int(truth.sum()))
    adj, summ = mte.mte_infer_network(series, max_lag_sources=5, alpha=0.001, alpha_fdr=0.001, S=1001, seed=1)
    m = mte.mte_link_metrics(adj, truth)
    say("metrics", m)
    assert m["precision"] >= 0.96 and m["recall"] >= 0.96 and m["specificity"] >= 0.98
    assert m == network.link_metrics(adj, truth)


def test_false_positive_rate_on_empty_networks():
    # 6 empty networks of 8 independent AR(1) nodes: every inferred link is a
    # false positive; the per-target false positive rate is controlled at alpha
    alpha, P, R = 0.05, 8, 6
    false_targets, links = 0, 0
    for rep in range(R):
        series = synth.empty_network(P, 1000, seed=100 + rep)
        adj, summ = mte.mte_infer_network(series, max_lag_sources=3, max_lag_target=3, alpha=alpha,
                                          alpha_fdr=0.0, S=40, seed=rep)
        false_targets += int(np.sum(adj.sum(0) > 0))
        links += int(adj.sum())
        say("empty network", rep, "false targets so far", false_targets)
    # P(Binomial(48, 0.05) > 9) < 1e-3
    assert false_targets <= 9
    m = mte.mte_link_metrics(adj, np.zeros((P, P), np.uint8))
    assert m["tp"] == 0 and m["fn"] == 0
