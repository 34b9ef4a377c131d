"""Surrogate-based significance tests.  TEST INFRASTRUCTURE ONLY.

Maximum statistic test (Maximum statistic test section, Table 1): given the CMI
I_j of every candidate j and the CMI I'_{j,s} of its surrogates s = 1..S,
  I* = max_j I_j (first candidate on ties), null I*_s = max_j I'_{j,s},
  p = #{s : I*_s > I*} / S, significant iff p < alpha.  S must exceed 1/alpha.
Minimum statistic test (Minimum statistic test section): the same with minimum
in place of maximum, i.e. I_min = min_j I_j, null min_j I'_{j,s},
  p = #{s : null_s > I_min} / S, significant iff p < alpha.
Omnibus test (Omnibus test section): p = #{s : T*_s > T*} / S for the collective
TE T* against jointly shuffled surrogates, significant iff p < alpha.

Family-wise error (Family-wise error rate correction section): the per-variable
false positive rate of the maximum statistic is 1-(1-alpha)^(1/n) (the Sidak
form), bounded below by the Bonferroni alpha/n, and the per-target rate over the
step-down iterations is alpha(1-alpha^n)/(1-alpha).
"""

from __future__ import annotations

import numpy as np


def require_surrogates(n_surr: int, alpha: float) -> None:
    if not (n_surr * alpha > 1.0):
        raise ValueError("the number of surrogates must exceed 1/alpha")


def max_statistic(real, surr, alpha: float):
    """Returns (index of I*, p, significant)."""
    real = np.asarray(real, dtype=np.float64)
    surr = np.asarray(surr, dtype=np.float64).reshape(len(real), -1)
    require_surrogates(surr.shape[1], alpha)
    j = int(np.argmax(real))
    null = surr.max(axis=0)
    p = float(np.count_nonzero(null > real[j])) / surr.shape[1]
    return j, p, p < alpha


def min_statistic(real, surr, alpha: float):
    """Returns (index of I_min, p, significant)."""
    real = np.asarray(real, dtype=np.float64)
    surr = np.asarray(surr, dtype=np.float64).reshape(len(real), -1)
    require_surrogates(surr.shape[1], alpha)
    j = int(np.argmin(real))
    null = surr.min(axis=0)
    p = float(np.count_nonzero(null > real[j])) / surr.shape[1]
    return j, p, p < alpha


def omnibus(real: float, surr, alpha: float):
    """Returns (p, significant)."""
    surr = np.asarray(surr, dtype=np.float64).ravel()
    require_surrogates(len(surr), alpha)
    p = float(np.count_nonzero(surr > real)) / len(surr)
    return p, p < alpha


def sidak_variable_fpr(alpha: float, n: int) -> float:
    return 1.0 - (1.0 - alpha) ** (1.0 / n)


def target_fpr(alpha: float, n: int) -> float:
    return alpha * (1.0 - alpha ** n) / (1.0 - alpha)


def benjamini_hochberg(pvals, q: float):
    """Boolean mask of the p-values rejected by the Benjamini-Hochberg step-up
    procedure at level q (Combining across multiple targets section)."""
    p = np.asarray(pvals, dtype=np.float64)
    m = len(p)
    order = np.argsort(p, kind="stable")
    passed = p[order] <= q * (np.arange(1, m + 1) / m)
    keep = np.zeros(m, dtype=bool)
    if np.any(passed):
        last = int(np.max(np.nonzero(passed)[0]))
        keep[order[: last + 1]] = True
    return keep
