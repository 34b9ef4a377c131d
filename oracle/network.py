"""Network-level inference: the greedy source selection for every target, the
Benjamini-Hochberg correction over the targets' omnibus p-values, the
inferred adjacency, and the link statistics of the paper's validation.
TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed:
  * Combining across multiple targets (Statistical tests section): the omnibus
    p-values of the targets go through an FDR correction (Benjamini-Hochberg);
    a target's sources are kept only if its omnibus test passes and the
    correction keeps it.
  * Influence of network size (Validation section): a directed link X -> Y is
    inferred whenever some past variable of X is among Y's selected sources;
    precision = TP/(TP+FP), recall = TP/(TP+FN), specificity = TN/(TN+FP).
  * Validation of false positive rate: FP/(FP+TN), and the per-target rate
    (the fraction of targets with at least one false source) on empty networks.

Readings: the candidates of target t are all other nodes in index order; the
greedy run of target t uses surrogate seed (seed + t) mod 2^64; targets without
selected sources take omnibus p = 1; the correction runs over all P targets.
"""

from __future__ import annotations

import numpy as np

from . import greedy, stats


def infer_network(series, max_lag_sources: int = 5, max_lag_target: int = 5, alpha: float = 0.05,
                  alpha_fdr: float | None = 0.05, k: int = 4, n_surr: int = 200, seed: int = 0,
                  estimator=None, theiler: int = 0, null: str = "surrogate", standardise_series: bool = True):
    """Returns (adjacency uint8 [P][P] with A[s][t] = 1 for an inferred link
    s -> t, per-target results of greedy.select_sources, FDR keep mask [P])."""
    series = np.asarray(series)
    P = series.shape[-2]
    results = []
    for t in range(P):
        cands = [j for j in range(P) if j != t]
        results.append(greedy.select_sources(series, t, cands, max_lag_sources=max_lag_sources,
                                             max_lag_target=max_lag_target, alpha=alpha, k=k,
                                             n_surr=n_surr, seed=(seed + t) % (1 << 64),
                                             estimator=estimator, theiler=theiler, null=null,
                                             standardise_series=standardise_series))
    pvals = np.array([r["omnibus_p"] for r in results])
    if alpha_fdr is None:
        keep = np.ones(P, dtype=bool)
    else:
        keep = stats.benjamini_hochberg(pvals, alpha_fdr)
    adj = np.zeros((P, P), dtype=np.uint8)
    for t, r in enumerate(results):
        if r["significant"] and keep[t]:
            for (node, _lag, _c, _p) in r["sources"]:
                adj[node, t] = 1
    return adj, results, keep


def link_metrics(inferred, truth):
    """precision, recall, specificity and false positive rate over the
    off-diagonal entries (a link per ordered pair of distinct nodes)."""
    a = np.asarray(inferred).astype(bool)
    b = np.asarray(truth).astype(bool)
    off = ~np.eye(a.shape[0], dtype=bool)
    tp = int(np.sum(a & b & off))
    fp = int(np.sum(a & ~b & off))
    tn = int(np.sum(~a & ~b & off))
    fn = int(np.sum(~a & b & off))
    div = lambda x, y: float(x) / y if y else float("nan")
    return {"tp": tp, "fp": fp, "tn": tn, "fn": fn, "precision": div(tp, tp + fp), "recall": div(tp, tp + fn),
            "specificity": div(tn, tn + fp), "fpr": div(fp, fp + tn)}
