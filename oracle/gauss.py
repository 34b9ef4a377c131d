"""Gaussian (linear) estimator of conditional mutual information and its
analytic null.  TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper names the Gaussian estimator as its second estimator (VAR section:
used for the VAR processes; Estimators section: compared with the
nearest-neighbour estimator on the coupled logistic maps) and notes that with
it the surrogate null can be replaced by an analytic one (Maximum statistic
test section).  Written out:

  Sigma_V  = (1/N) sum_t (v_t - mean v)(v_t - mean v)^T     (float64, two passes)
  I(X;Y|Z) = 1/2 [ln det Sigma_XZ + ln det Sigma_YZ - ln det Sigma_Z - ln det Sigma_XYZ]
             (ln det of an empty matrix = 0), in nats;
  null:      2 N I ~ chi^2 with dx*dy degrees of freedom (asymptotically).

Tests with the analytic null (readings: the surrogate tests of the Statistical
tests section with the null distribution of each estimate replaced by the chi^2
law, the n candidates treated as independent, as in the FWER section):
  maximum statistic over n candidates: p = 1 - (1 - sf(2 N I_max))^n
  minimum statistic over n candidates: p = sf(2 N I_min)^n
  omnibus test of the d_S selected source variables: p = sf_{d_S * dy}(2 N T)
"""

from __future__ import annotations

import math

import numpy as np
from scipy.stats import chi2


def _stack(*parts):
    cols = [np.asarray(p, dtype=np.float64) for p in parts if p is not None and np.asarray(p).size]
    return np.concatenate(cols, axis=0) if cols else None


def covariance(v) -> np.ndarray:
    """(1/N) sum_t (v_t - mean)(v_t - mean)^T for v [d][N] (two passes, float64)."""
    v = np.asarray(v, dtype=np.float64)
    n = v.shape[1]
    c = v - v.sum(axis=1, keepdims=True) / n
    return (c @ c.T) / n


def logdet(m) -> float:
    if m is None or m.size == 0:
        return 0.0
    sign, val = np.linalg.slogdet(m)
    if sign <= 0:
        raise ValueError("covariance matrix is not positive definite")
    return float(val)


def cmi_gauss(x, y, z=None) -> float:
    """I(X;Y|Z) in nats for float32 columns [dx][N], [dy][N], [dz][N] or None."""
    dx = np.asarray(x).reshape(-1, np.shape(x)[-1]).shape[0]
    dy = np.asarray(y).reshape(-1, np.shape(y)[-1]).shape[0]
    dz = 0 if z is None else np.asarray(z).reshape(-1, np.shape(z)[-1]).shape[0]
    s = covariance(_stack(x, y, z))
    ix, iy, iz = list(range(dx)), list(range(dx, dx + dy)), list(range(dx + dy, dx + dy + dz))
    sub = lambda idx: s[np.ix_(idx, idx)] if idx else None
    return 0.5 * (logdet(sub(ix + iz)) + logdet(sub(iy + iz)) - logdet(sub(iz)) - logdet(sub(ix + iy + iz)))


def p_value(i: float, n: int, dof: int) -> float:
    return float(chi2.sf(2.0 * n * i, dof))


def p_max(i_max: float, n_cands: int, n: int, dof: int) -> float:
    return 1.0 - (1.0 - p_value(i_max, n, dof)) ** n_cands


def p_min(i_min: float, n_cands: int, n: int, dof: int) -> float:
    return p_value(i_min, n, dof) ** n_cands
