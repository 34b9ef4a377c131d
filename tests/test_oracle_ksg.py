"""Pins for the oracle's KSG estimator (oracle/ksg.py and oracle/ksg_oracle.c).

Each check ties the oracle to something other than itself: a hand-counted case,
an exact rational brute force, scipy's k-d tree, closed forms of the estimator
on special inputs, invariances the definition implies, and the Gaussian closed
form of the conditional mutual information.
"""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.special import digamma

import synth
from oracle import cksg, ksg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1, np.shape(a)[-1]))


# ---------------------------------------------------------------- hand-counted
def test_hand_counted_case():
    g = json.load(open(os.path.join(GOLD, "hand_counted_k2_n6.json")))
    X, Y, Z = f32([g["X"]]), f32([g["Y"]]), f32([g["Z"]])
    val, (eps, a, b, c) = ksg.cmi_ksg(X, Y, Z, g["k"], diag=True)
    assert eps.tolist() == g["eps"]
    assert a.tolist() == g["n_xz"] and b.tolist() == g["n_yz"] and c.tolist() == g["n_z"]
    assert abs(val - g["cmi_numerator"] / g["cmi_denominator"]) < 1e-14
    e2, a2, b2, c2, v2 = cksg.eps_and_counts(X, Y, Z, g["k"])
    assert e2.tolist() == g["eps"] and a2.tolist() == g["n_xz"]
    assert b2.tolist() == g["n_yz"] and c2.tolist() == g["n_z"]
    assert abs(v2 - g["cmi_numerator"] / g["cmi_denominator"]) < 1e-14


# ---------------------------------------------------------------- exact brute force
def _exact_ksg(cols_x, cols_y, cols_z, k):
    """Exact rational brute force: distances as Fractions, eps from a full sort,
    the estimate as an exact rational via psi(m+1) - psi(1) = H_m."""
    n = len(cols_x[0])
    fr = lambda cols: [[Fraction(float(v)) for v in c] for c in cols]
    X, Y, Z = fr(cols_x), fr(cols_y), fr(cols_z)

    def dist(cols, i, j):
        return max([abs(c[i] - c[j]) for c in cols], default=Fraction(0))

    H = [Fraction(0)]
    for m in range(1, n + 1):
        H.append(H[-1] + Fraction(1, m))
    eps, cnt, total = [], [], Fraction(0)
    for i in range(n):
        dxs = [dist(X, i, j) for j in range(n)]
        dys = [dist(Y, i, j) for j in range(n)]
        dzs = [dist(Z, i, j) for j in range(n)]
        d = sorted(max(dxs[j], dys[j], dzs[j]) for j in range(n) if j != i)
        e = d[k - 1]
        nxz = sum(1 for j in range(n) if j != i and max(dxs[j], dzs[j]) < e)
        nyz = sum(1 for j in range(n) if j != i and max(dys[j], dzs[j]) < e)
        nz = sum(1 for j in range(n) if j != i and dzs[j] < e)
        eps.append(e)
        cnt.append((nxz, nyz, nz))
        total += H[nxz] + H[nyz] - H[nz]
    return eps, cnt, H[k - 1] - total / n


@pytest.mark.parametrize("seed,n,dims,k", [(1, 7, (1, 1, 1), 1), (2, 9, (2, 1, 2), 2),
                                          (3, 12, (1, 2, 0), 3), (4, 10, (1, 1, 3), 4),
                                          (5, 11, (3, 1, 1), 2)])
def test_exact_rational_bruteforce(seed, n, dims, k):
    # coarse dyadic grid: float32 differences are exact and ties are frequent
    x, y, z = synth.random_points(n, dims, seed, kind="grid")
    exact_eps, exact_cnt, exact_val = _exact_ksg(x, y, [] if z is None else z, k)
    val, (eps, a, b, c) = ksg.cmi_ksg(x, y, z, k, diag=True)
    assert [Fraction(float(e)) for e in eps] == exact_eps
    assert list(zip(a.tolist(), b.tolist(), c.tolist())) == exact_cnt
    assert abs(val - float(exact_val)) < 1e-12


# ---------------------------------------------------------------- k-d tree
@pytest.mark.parametrize("seed,dims,k", [(11, (1, 1, 1), 4), (12, (1, 1, 5), 4), (13, (2, 2, 0), 3),
                                         (14, (1, 1, 3), 1)])
def test_against_kdtree(seed, dims, k):
    n = 400
    g = np.random.default_rng(seed)
    # values on a dyadic grid fine enough to make ties rare, so eps > 0 everywhere
    mk = lambda d: None if d == 0 else (g.integers(-4096, 4097, size=(d, n)) / 512.0).astype(np.float32)
    x, y, z = mk(dims[0]), mk(dims[1]), mk(dims[2])
    eps, a, b, c = ksg.eps_and_counts(x, y, z, k)
    parts = [x, y] + ([] if z is None else [z])
    joint = np.concatenate(parts, axis=0).T.astype(np.float64)
    dk, _ = cKDTree(joint).query(joint, k=k + 1, p=np.inf)
    ref_eps = dk[:, k]
    assert np.array_equal(eps.astype(np.float64), ref_eps)
    assert np.all(ref_eps > 0)

    def count(sub):
        if sub is None:
            return np.full(n, n - 1)
        pts = sub.T.astype(np.float64)
        r = np.nextafter(ref_eps, 0)
        return np.array([len(cKDTree(pts).query_ball_point(pts[i], r[i], p=np.inf)) - 1
                         for i in range(n)])

    xz = x if z is None else np.concatenate([x, z], 0)
    yz = y if z is None else np.concatenate([y, z], 0)
    assert np.array_equal(a, count(xz))
    assert np.array_equal(b, count(yz))
    assert np.array_equal(c, count(z))


# ---------------------------------------------------------------- closed forms
def test_x_equals_y_without_z_is_psi_n_minus_psi_k():
    # X = Y and no ties: n_x = n_y = k-1, so I = psi(N) - psi(k)
    n, k = 500, 4
    x = synth.random_points(n, (1,), 21)[0]
    val = ksg.cmi_ksg(x, x.copy(), None, k)
    assert abs(val - (digamma(n) - digamma(k))) < 1e-12


def test_x_equals_y_with_z():
    # X = Y: n_xz = n_yz = k-1 (no ties), so I = mean psi(n_z+1) - psi(k)
    n, k = 400, 3
    x, z = synth.random_points(n, (1, 2), 22)
    val, (eps, a, b, c) = ksg.cmi_ksg(x, x.copy(), z, k, diag=True)
    assert np.all(a == k - 1) and np.all(b == k - 1)
    assert abs(val - (np.mean(digamma(c + 1.0)) - digamma(k))) < 1e-12


def test_no_conditioning_is_ksg_algorithm_1():
    # dz = 0: n_z = N-1 and I = psi(k) + psi(N) - <psi(n_x+1) + psi(n_y+1)>
    n, k = 300, 4
    x, y = synth.random_points(n, (1, 2), 23)
    val, (eps, a, b, c) = ksg.cmi_ksg(x, y, None, k, diag=True)
    assert np.all(c == n - 1)
    ref = digamma(k) + digamma(n) - np.mean(digamma(a + 1.0) + digamma(b + 1.0))
    assert abs(val - ref) < 1e-12


# ---------------------------------------------------------------- invariances
def test_invariances():
    n, k = 300, 4
    x, y, z = synth.random_points(n, (1, 1, 2), 31, kind="dup")
    val, (eps, a, b, c) = ksg.cmi_ksg(x, y, z, k, diag=True)
    # joint row permutation permutes eps and counts
    p = np.random.default_rng(5).permutation(n)
    v2, (e2, a2, b2, c2) = ksg.cmi_ksg(x[:, p], y[:, p], z[:, p], k, diag=True)
    assert np.array_equal(e2, eps[p]) and np.array_equal(a2, a[p])
    assert np.array_equal(b2, b[p]) and np.array_equal(c2, c[p])
    assert abs(v2 - val) < 1e-12
    # X <-> Y swap exchanges n_xz and n_yz and leaves I unchanged
    v3, (e3, a3, b3, c3) = ksg.cmi_ksg(y, x, z, k, diag=True)
    assert np.array_equal(a3, b) and np.array_equal(b3, a) and v3 == val
    # scaling every variable by a power of two keeps all counts
    v4, (e4, a4, b4, c4) = ksg.cmi_ksg(x * 8, y * 8, z * 8, k, diag=True)
    assert np.array_equal(e4, eps * 8) and np.array_equal(a4, a) and v4 == val
    # a duplicated or constant extra Z column changes nothing
    zd = np.concatenate([z, z[:1]], 0)
    zc = np.concatenate([z, np.full((1, n), 3.0, np.float32)], 0)
    for zz in (zd, zc):
        v5, (e5, a5, b5, c5) = ksg.cmi_ksg(x, y, zz, k, diag=True)
        assert np.array_equal(e5, eps) and np.array_equal(c5, c) and v5 == val


# ---------------------------------------------------------------- numpy vs C
@pytest.mark.parametrize("kind", ["normal", "grid", "dup", "tiny", "wide"])
@pytest.mark.parametrize("dims,k", [((1, 1, 1), 4), ((1, 1, 5), 4), ((2, 1, 0), 2), ((1, 3, 4), 7)])
def test_numpy_and_c_oracles_agree(kind, dims, k):
    n = 257
    x, y, z = synth.random_points(n, dims, hash((kind, dims, k)) % 1000, kind=kind)
    v1, (e1, a1, b1, c1) = ksg.cmi_ksg(x, y, z, k, diag=True)
    e2, a2, b2, c2, v2 = cksg.eps_and_counts(x, y, z, k)
    assert np.array_equal(e1, e2)
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2) and np.array_equal(c1, c2)
    assert abs(v1 - v2) < 1e-12


def test_denormals_are_kept():
    # the distances of this input are all denormal: a flush to zero would make
    # every eps zero and every count zero
    x, y, z = synth.random_points(64, (1, 1, 1), 41, kind="tiny")
    eps, a, b, c = ksg.eps_and_counts(x, y, z, 4)
    assert np.all(eps > 0) and np.all(eps < np.finfo(np.float32).tiny)
    e2, *_ = cksg.eps_and_counts(x, y, z, 4)
    assert np.array_equal(eps, e2)


def test_sampled_queries_match_full():
    x, y, z = synth.random_points(1000, (1, 1, 3), 51)
    full = ksg.eps_and_counts(x, y, z, 4)
    q = np.array([0, 17, 500, 999])
    part = ksg.eps_and_counts(x, y, z, 4, queries=q)
    cpart = cksg.eps_and_counts(x, y, z, 4, queries=q)
    for f, p, c in zip(full, part, cpart[:4]):
        assert np.array_equal(f[q], p) and np.array_equal(p, c)


# ---------------------------------------------------------------- statistics
def test_gaussian_closed_form():
    # I(X;Y|Z) = -0.5 log(1 - 0.6^2) = 0.2231435513 nats for the jointly
    # Gaussian construction; the KSG estimate at N=1000, k=4 carries a small
    # positive bias and a spread of about 0.03 over seeds
    vals = []
    for seed in range(1, 21):
        x, y, z, true = synth.c1_gaussian(1000, seed)
        vals.append(cksg.cmi_ksg(x, y, z, 4))
    assert abs(true - 0.2231435513) < 1e-9
    assert max(abs(v - true) for v in vals) < 0.10
    assert abs(np.mean(vals) - true) < 0.02


def test_independent_data_near_zero():
    vals = []
    for seed in range(1, 21):
        x, y, z = synth.random_points(1000, (1, 1, 1), 100 + seed)
        vals.append(cksg.cmi_ksg(x, y, z, 4))
    assert max(abs(v) for v in vals) < 0.07
    assert abs(np.mean(vals)) < 0.02


def test_rejects_bad_arguments():
    x, y = synth.random_points(5, (1, 1), 1)
    with pytest.raises(ValueError):
        ksg.cmi_ksg(x, y, None, 5)
    with pytest.raises(ValueError):
        cksg.eps_and_counts(x, y, None, 0)


def test_psi_identity_used_by_the_c_oracle():
    # the C oracle evaluates psi(m+1) + gamma as the harmonic number H_m
    h = np.concatenate([[0.0], np.cumsum(1.0 / np.arange(1, 20001))])
    m = np.arange(0, 20001)
    assert np.max(np.abs((digamma(m + 1.0) + np.euler_gamma) - h)) < 1e-11
    assert math.isclose(h[3], 1 + 1 / 2 + 1 / 3)


# ---------------------------------------------------------------- Theiler window
def _exact_ksg_window(cols_x, cols_y, cols_z, k, w):
    """Exact rational brute force with the rows |i - j| <= w left out of row i's
    neighbour set (no Z: n_z is the size of that set)."""
    n = len(cols_x[0])
    fr = lambda cols: [[Fraction(float(v)) for v in c] for c in cols]
    X, Y, Z = fr(cols_x), fr(cols_y), fr(cols_z)

    def dist(cols, i, j):
        return max([abs(c[i] - c[j]) for c in cols], default=Fraction(0))

    out = []
    for i in range(n):
        R = [j for j in range(n) if abs(i - j) > w]
        d = sorted(max(dist(X, i, j), dist(Y, i, j), dist(Z, i, j)) for j in R)
        e = d[k - 1]
        nxz = sum(1 for j in R if max(dist(X, i, j), dist(Z, i, j)) < e)
        nyz = sum(1 for j in R if max(dist(Y, i, j), dist(Z, i, j)) < e)
        nz = len(R) if not Z else sum(1 for j in R if dist(Z, i, j) < e)
        out.append((e, nxz, nyz, nz))
    return out


@pytest.mark.parametrize("seed,n,dims,k,w", [(21, 12, (1, 1, 1), 2, 1), (22, 15, (2, 1, 2), 3, 3),
                                            (23, 13, (1, 2, 0), 2, 2), (24, 16, (1, 1, 3), 4, 5)])
def test_theiler_window_exact(seed, n, dims, k, w):
    x, y, z = synth.random_points(n, dims, seed, kind="grid")
    ref = _exact_ksg_window(x, y, [] if z is None else z, k, w)
    eps, a, b, c = ksg.eps_and_counts(x, y, z, k, theiler=w)
    assert [(Fraction(float(e)), int(p), int(q), int(r)) for e, p, q, r in zip(eps, a, b, c)] == ref
    e2, a2, b2, c2, _ = cksg.eps_and_counts(x, y, z, k, theiler=w)
    assert np.array_equal(eps, e2) and np.array_equal(a, a2) and np.array_equal(b, b2) and np.array_equal(c, c2)


def test_theiler_window_against_kdtree():
    # k-th neighbour outside the window: query k + 2w + 1 neighbours with a
    # k-d tree and drop those inside the window
    n, k, w = 500, 4, 3
    g = np.random.default_rng(31)
    pts = (g.integers(-4096, 4097, size=(3, n)) / 512.0).astype(np.float32)
    x, y, z = pts[:1], pts[1:2], pts[2:]
    eps, *_ = ksg.eps_and_counts(x, y, z, k, theiler=w)
    tree = cKDTree(pts.T.astype(np.float64))
    d, idx = tree.query(pts.T.astype(np.float64), k=k + 2 * w + 1 + 1, p=np.inf)
    for i in range(n):
        keep = [dd for dd, j in zip(d[i], idx[i]) if abs(int(j) - i) > w]
        assert eps[i] == np.float32(keep[k - 1])


def test_theiler_window_reversal_and_rejection():
    # reversing the time order maps every window onto itself
    x, y, z = synth.random_points(300, (1, 1, 2), seed=41)
    rev = lambda a: np.ascontiguousarray(a[:, ::-1])
    r1 = ksg.eps_and_counts(x, y, z, 4, theiler=6)
    r2 = ksg.eps_and_counts(rev(x), rev(y), rev(z), 4, theiler=6)
    for a, b in zip(r1, r2):
        assert np.array_equal(a, b[::-1])
    # w = 0 is the plain estimator
    for a, b in zip(ksg.eps_and_counts(x, y, z, 4, theiler=0), ksg.eps_and_counts(x, y, z, 4)):
        assert np.array_equal(a, b)
    # too few rows outside the window
    with pytest.raises(ValueError):
        ksg.eps_and_counts(x[:, :20], y[:, :20], z[:, :20], 4, theiler=8)
    with pytest.raises(ValueError):
        cksg.eps_and_counts(x[:, :20], y[:, :20], z[:, :20], 4, theiler=8)
