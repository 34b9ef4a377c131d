"""Greedy multivariate transfer-entropy inference for one target, in the paper's
four steps (Inference algorithm section).  TEST INFRASTRUCTURE ONLY.

  Step 1  target past: from the candidates Y_{t-1..t-l_target}, repeatedly take
          the C maximising I(C; Y_t | Y^S), keep it if the maximum statistic test
          is significant, stop at the first non-significant test or when no
          candidate is left.
  Step 2  sources past: the same over X_{i,t-1..t-l_sources} of every candidate
          source with conditioning set Y^S u X^S.
  Step 3  pruning: find the C in X^S minimising I(C; Y_t | Y^S u X^S \\ {C}); if
          the minimum statistic test is NOT significant remove it and repeat;
          stop when it is significant or X^S is empty.
  Step 4  omnibus: T* = I(X^S; Y_t | Y^S) against surrogates in which the rows
          of all selected source columns are shuffled jointly; the sources are
          accepted only if this test is significant as well.

Readings fixed where the paper is silent (each also used by the library):
  * embedding rows t = l_M .. T-1 with l_M = max(l_target, l_sources), so
    N = T - l_M; variable (node, lag) is series[node][t - lag];
  * candidate order: target lags ascending; sources in the given order, each
    with lags ascending; removal keeps the order of the rest; ties go to the
    first candidate in that order;
  * surrogate keys: a running test counter `tid` starts at 0 for the target;
    every candidate of every max/min-statistic round takes the next tid, in
    candidate order, and draws its S surrogates with keys (seed, tid, s); the
    omnibus test takes the next tid after pruning;
  * each node series is z-scored once before embedding (standardise());
  * alpha_max = alpha_min = alpha_omnibus = alpha;
  * the reported CMI and p of a selected variable are those of the test that
    selected it; an empty X^S skips the omnibus test (p = 1, not significant);
"""

from __future__ import annotations

import numpy as np

from . import gauss, ksg, perm, stats


def standardise(series: np.ndarray) -> np.ndarray:
    """Per-node z-score (reading: the paper is silent on normalisation; every
    node is put on one scale before embedding).  For each node, over its
    samples in order (replications, then time): mean = sum / count and
    variance = sum((x - mean)^2) / count, both sums float64 and sequential
    (np.cumsum), sd = sqrt(variance); each value (x - mean) / sd in float64,
    rounded to float32; a constant node becomes 0."""
    s = np.asarray(series)
    out = np.empty(s.shape, dtype=np.float32)
    nodes = s.shape[-2]
    for p in range(nodes):
        v = (s[:, p, :] if s.ndim == 3 else s[p]).astype(np.float64)
        flat = v.reshape(-1)
        mean = np.cumsum(flat)[-1] / flat.size
        dev = flat - mean
        sd = np.sqrt(np.cumsum(dev * dev)[-1] / flat.size)
        z = (dev / sd if sd > 0 else np.zeros_like(dev)).astype(np.float32).reshape(v.shape)
        if s.ndim == 3:
            out[:, p, :] = z
        else:
            out[p] = z
    return out


def embed(series: np.ndarray, node: int, lag: int, l_m: int) -> np.ndarray:
    """Column of variable (node, lag): rows t = l_m..T-1 of series[node][t-lag];
    with replications (series [R][P][T]) the rows of every replication in
    replication order."""
    if series.ndim == 3:
        t = series.shape[2]
        return np.ascontiguousarray(np.concatenate([series[r, node, l_m - lag: t - lag]
                                                    for r in range(series.shape[0])])[None, :])
    t = series.shape[1]
    return np.ascontiguousarray(series[node, l_m - lag: t - lag][None, :])


class _Run:
    def __init__(self, series, target, k, n_surr, seed, l_m, estimator):
        self.series = series
        self.target = target
        self.k = k
        self.n_surr = n_surr
        self.seed = seed
        self.l_m = l_m
        self.tid = 0
        self.n_estimates = 0
        self.est = estimator
        self.y = embed(series, target, 0, l_m)
        self.reps = series.shape[0] if series.ndim == 3 else 1
        self.mode = perm.shuffle_mode(self.reps, n_surr)

    def source_rows(self, s, n_rows):
        return perm.replication_source_rows(self.seed, self.tid, s, n_rows, self.reps, self.mode)

    def cols(self, variables):
        if not variables:
            return None
        return np.concatenate([embed(self.series, n, l, self.l_m) for (n, l) in variables], axis=0)

    def test_candidates(self, cands, cond_of):
        """CMI of each candidate and of its S surrogates: ([n], [n][S])."""
        n_rows = self.y.shape[1]
        real = np.empty(len(cands))
        surr = np.empty((len(cands), self.n_surr))
        for j, c in enumerate(cands):
            x = self.cols([c])
            z = self.cols(cond_of(c))
            real[j] = self.est(x, self.y, z, self.k)
            for s in range(self.n_surr):
                p = self.source_rows(s, n_rows)
                surr[j, s] = self.est(ksg.permute_rows(x, p), self.y, z, self.k)
            self.tid += 1
            self.n_estimates += 1 + self.n_surr
        return real, surr


def _numpy_estimator(x, y, z, k, theiler=0):
    return ksg.cmi_ksg(x, y, z, k, theiler=theiler)


def select_sources(series, target: int, candidates, max_lag_sources: int = 5,
                   max_lag_target: int = 5, alpha: float = 0.05, k: int = 4,
                   n_surr: int = 200, seed: int = 0, estimator=None, theiler: int = 0,
                   null: str = "surrogate", standardise_series: bool = True):
    """null = "surrogate": the KSG estimator (or `estimator`) with the
    surrogate tests.  null = "analytic": the Gaussian estimator with the
    analytic (chi^2) null of oracle/gauss.py; no surrogates are drawn.
    series: [P][T], or [R][P][T] for R replications (rows of all
    replications pooled; surrogates shuffle the replications of the candidate
    when R! >= S, else the samples within each replication, oracle/perm.py)."""
    series = np.asarray(series)
    if series.dtype != np.float32:
        raise TypeError("series must be float32")
    if series.ndim == 3 and theiler:
        raise ValueError("the Theiler window is defined for a single replication")
    if standardise_series:
        series = standardise(series)
    analytic = null == "analytic"
    if analytic:
        n_surr = 0
        estimator = lambda x, y, z, kk, theiler=0: gauss.cmi_gauss(x, y, z)
    else:
        stats.require_surrogates(n_surr, alpha)
    if target in candidates:
        raise ValueError("target among candidates")
    l_m = max(max_lag_target, max_lag_sources)
    est = estimator or _numpy_estimator
    run = _Run(series, target, k, n_surr, seed, l_m,
               (lambda x, y, z, kk: est(x, y, z, kk, theiler=theiler)) if theiler else est)

    n_rows = run.y.shape[1]

    def max_test(real, surr):
        if not analytic:
            return stats.max_statistic(real, surr, alpha)
        j = int(np.argmax(real))
        p = gauss.p_max(float(real[j]), len(real), n_rows, 1)
        return j, p, p < alpha

    def min_test(real, surr):
        if not analytic:
            return stats.min_statistic(real, surr, alpha)
        j = int(np.argmin(real))
        p = gauss.p_min(float(real[j]), len(real), n_rows, 1)
        return j, p, p < alpha

    # Step 1: target past
    ycand = [(target, lag) for lag in range(1, max_lag_target + 1)]
    ysel = []
    while ycand:
        yv = [(n, l) for (n, l, _, _) in ysel]
        real, surr = run.test_candidates(ycand, lambda c: yv)
        j, p, sig = max_test(real, surr)
        if not sig:
            break
        ysel.append(ycand[j] + (float(real[j]), p))
        del ycand[j]
    yvars = [(n, l) for (n, l, _, _) in ysel]

    # Step 2: sources past
    xcand = [(src, lag) for src in candidates for lag in range(1, max_lag_sources + 1)]
    xsel = []
    while xcand:
        xvars = [(n, l) for (n, l, _, _) in xsel]
        real, surr = run.test_candidates(xcand, lambda c: yvars + xvars)
        j, p, sig = max_test(real, surr)
        if not sig:
            break
        xsel.append(xcand[j] + (float(real[j]), p))
        del xcand[j]

    # Step 3: pruning
    while xsel:
        xvars = [(n, l) for (n, l, _, _) in xsel]
        real, surr = run.test_candidates(
            xvars, lambda c: yvars + [v for v in xvars if v != c])
        j, p, sig = min_test(real, surr)
        if sig:
            break
        del xsel[j]

    # Step 4: omnibus
    omni_te, omni_p, omni_sig = 0.0, 1.0, False
    if xsel:
        xvars = [(n, l) for (n, l, _, _) in xsel]
        x = run.cols(xvars)
        z = run.cols(yvars)
        omni_te = run.est(x, run.y, z, k)
        if analytic:
            run.tid += 1
            run.n_estimates += 1
            omni_p = gauss.p_value(omni_te, n_rows, len(xvars))
            omni_sig = omni_p < alpha
        else:
            surr = np.empty(n_surr)
            for s in range(n_surr):
                p_ = run.source_rows(s, n_rows)
                surr[s] = run.est(ksg.permute_rows(x, p_), run.y, z, k)
            run.tid += 1
            run.n_estimates += 1 + n_surr
            omni_p, omni_sig = stats.omnibus(omni_te, surr, alpha)
    return {
        "target_past": ysel,
        "sources": xsel if omni_sig else [],
        "sources_before_omnibus": xsel,
        "omnibus_te": omni_te,
        "omnibus_p": omni_p,
        "significant": bool(omni_sig),
        "n_estimates": run.n_estimates,
    }
