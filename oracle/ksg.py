"""Brute-force KSG conditional mutual information, written from the estimator's
definition.  TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper uses the nearest-neighbour estimator for its coupled-logistic-map runs
(CLM section: Kraskov's estimator I^(1) with k=4 and its extension to CMI) but
prints no formula.  This module writes out that cited definition:

  1. Joint points p_i = (x_i, y_i, z_i), i < N, from float32 columns.
  2. Per-dimension distance |fl32(a_i - a_j)|: one IEEE binary32 subtraction,
     round to nearest even, denormals kept; the absolute value is exact.
  3. Subspace max-norms d_X, d_Y, d_Z (maxima over that subspace's columns;
     d_Z = 0 when there is no conditioning set) and d = max(d_X, d_Y, d_Z).
  4. eps_i = k-th smallest of the multiset {d(i,j) : j in R_i}, where R_i is
     the set of rows outside row i's Theiler window: |i - j| > w (the paper's
     dynamic correlation exclusion, section on autocorrelation in real data;
     w = 0 leaves R_i = {j != i}).
  5. Strict counts n_xz(i) = #{j in R_i : max(d_X, d_Z) < eps_i}, n_yz
     likewise, n_z(i) = #{j in R_i : d_Z < eps_i} (= |R_i| when dz = 0).
  6. I = psi(k) - (1/N) sum_i [psi(n_xz+1) + psi(n_yz+1) - psi(n_z+1)] in nats,
     float64, with scipy's digamma and an exactly rounded sum (math.fsum).
     Negative values are returned as they are (Statistical tests section: the
     estimator can be negative when its bias exceeds the true CMI).

No blocking or reordering beyond evaluating step 2-5 for a block of queries at a
time, which changes nothing since every step is exact.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import digamma


def _cols(a, n):
    if a is None:
        return np.zeros((0, n), dtype=np.float32)
    a = np.asarray(a)
    if a.dtype != np.float32:
        raise TypeError("columns must be float32")
    if a.ndim == 1:
        a = a[None, :]
    if a.shape[1] != n:
        raise ValueError("column length mismatch")
    return np.ascontiguousarray(a)


def subspace_dist(cols: np.ndarray, qidx: np.ndarray) -> np.ndarray:
    """max over columns of |fl32(a[q] - a[j])| for every query q in qidx and
    every j: float32 array [len(qidx)][N].  Zero when there are no columns."""
    d, n = cols.shape
    out = np.zeros((len(qidx), n), dtype=np.float32)
    for c in range(d):
        diff = cols[c, qidx][:, None] - cols[c][None, :]   # float32 - float32 -> float32
        np.maximum(out, np.abs(diff), out=out)
    return out


def eps_and_counts(x, y, z, k: int, queries=None, block: int = 256, theiler: int = 0):
    """Steps 1-5 for the given query indices (all by default), with Theiler
    window w = theiler.

    Returns (eps float32, n_xz int64, n_yz int64, n_z int64), one entry per query.
    """
    x = np.asarray(x)
    n = x.shape[-1]
    X, Y, Z = _cols(x, n), _cols(y, n), _cols(z, n)
    if theiler < 0:
        raise ValueError("Theiler window must be >= 0")
    if not (1 <= k <= n - 1 - 2 * theiler):
        raise ValueError("need 1 <= k <= N-1-2w")
    qs = np.arange(n) if queries is None else np.asarray(queries, dtype=np.int64)
    eps = np.empty(len(qs), dtype=np.float32)
    nxz = np.empty(len(qs), dtype=np.int64)
    nyz = np.empty(len(qs), dtype=np.int64)
    nz = np.empty(len(qs), dtype=np.int64)
    for b0 in range(0, len(qs), block):
        q = qs[b0:b0 + block]
        dx = subspace_dist(X, q)
        dy = subspace_dist(Y, q)
        dz = subspace_dist(Z, q)
        d = np.maximum(np.maximum(dx, dy), dz)
        # rows inside row q's Theiler window (q itself when w = 0)
        self_mask = np.abs(q[:, None] - np.arange(n)[None, :]) <= theiler
        d_noself = np.where(self_mask, np.float32(np.inf), d)
        e = np.partition(d_noself, k - 1, axis=1)[:, k - 1]
        eps[b0:b0 + len(q)] = e
        et = e[:, None]
        nxz[b0:b0 + len(q)] = ((np.maximum(dx, dz) < et) & ~self_mask).sum(1)
        nyz[b0:b0 + len(q)] = ((np.maximum(dy, dz) < et) & ~self_mask).sum(1)
        if Z.shape[0] == 0:
            nz[b0:b0 + len(q)] = (~self_mask).sum(1)
        else:
            nz[b0:b0 + len(q)] = ((dz < et) & ~self_mask).sum(1)
    return eps, nxz, nyz, nz


def cmi_from_counts(k: int, nxz, nyz, nz) -> float:
    """Step 6: psi(k) - mean_i[psi(n_xz+1) + psi(n_yz+1) - psi(n_z+1)]."""
    nxz = np.asarray(nxz, dtype=np.float64)
    nyz = np.asarray(nyz, dtype=np.float64)
    nz = np.asarray(nz, dtype=np.float64)
    terms = (digamma(nxz + 1.0) + digamma(nyz + 1.0)) - digamma(nz + 1.0)
    return float(digamma(float(k)) - math.fsum(terms.tolist()) / len(terms))


def cmi_ksg(x, y, z, k: int = 4, diag: bool = False, theiler: int = 0):
    """I(X;Y|Z) in nats.  x, y: float32 [dx][N], [dy][N]; z: float32 [dz][N] or
    None.  With diag=True also returns (eps, n_xz, n_yz, n_z)."""
    eps, nxz, nyz, nz = eps_and_counts(x, y, z, k, theiler=theiler)
    val = cmi_from_counts(k, nxz, nyz, nz)
    if diag:
        return val, (eps, nxz, nyz, nz)
    return val


def permute_rows(x: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """Surrogate columns: row i of the result is row perm[i] of x, the same
    permutation for every column (a joint shuffle of the realisations)."""
    return np.ascontiguousarray(np.asarray(x)[:, perm])
