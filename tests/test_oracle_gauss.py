"""Pins for the Gaussian CMI oracle (oracle/gauss.py): partial correlation
from least-squares residuals, the Pearson correlation without Z, the Gaussian
closed form, affine invariance, closed forms of the chi^2 survival function and
the calibration of the analytic null."""

import math

import numpy as np
import pytest
from scipy.special import erfc

import synth
from oracle import gauss


def resid(v, z):
    if z is None:
        return v - v.mean()
    A = np.vstack([z, np.ones(z.shape[1])]).T
    coef, *_ = np.linalg.lstsq(A, v, rcond=None)
    return v - A @ coef


@pytest.mark.parametrize("seed,dz", [(1, 0), (2, 1), (3, 4)])
def test_partial_correlation_form(seed, dz):
    # 1-D X and Y: I = -1/2 ln(1 - r^2), r the correlation of the residuals of
    # X and Y after least-squares regression on Z (and a constant)
    g = np.random.default_rng(seed)
    n = 2000
    z = g.standard_normal((dz, n)) if dz else None
    x = g.standard_normal(n) + (z.sum(0) if dz else 0)
    y = 0.5 * x + g.standard_normal(n) + (0.3 * z[0] if dz else 0)
    rx, ry = resid(x, z), resid(y, z)
    r = np.dot(rx, ry) / math.sqrt(np.dot(rx, rx) * np.dot(ry, ry))
    ref = -0.5 * math.log(1 - r * r)
    f = lambda a: None if a is None else np.atleast_2d(a).astype(np.float32)
    got = gauss.cmi_gauss(f(x), f(y), f(z))
    # the oracle sees the float32-rounded values: recompute the reference on them
    x32, y32 = f(x)[0].astype(np.float64), f(y)[0].astype(np.float64)
    z32 = None if z is None else f(z).astype(np.float64)
    rx, ry = resid(x32, z32), resid(y32, z32)
    r = np.dot(rx, ry) / math.sqrt(np.dot(rx, rx) * np.dot(ry, ry))
    assert abs(got - (-0.5 * math.log(1 - r * r))) < 1e-10
    assert abs(got - ref) < 1e-5
    if not dz:
        assert abs(got - (-0.5 * math.log(1 - np.corrcoef(x32, y32)[0, 1] ** 2))) < 1e-10


def test_gaussian_closed_form_and_invariance():
    X, Y, Z, true = synth.c1_gaussian(200000, 5)
    got = gauss.cmi_gauss(X, Y, Z)
    assert abs(got - true) < 0.01
    # affine maps of each variable leave the estimate unchanged
    a = gauss.cmi_gauss((3 * X + 1).astype(np.float32), (-2 * Y).astype(np.float32), (Z / 4 - 7).astype(np.float32))
    small = gauss.cmi_gauss(X[:, :5000], Y[:, :5000], Z[:, :5000])
    assert abs(a - got) < 1e-6 and small != got


def test_chi2_survival_closed_forms():
    for x in (0.0, 0.3, 2.0, 9.5):
        assert abs(gauss.p_value(x / 2.0, 1, 2) - math.exp(-x / 2)) < 1e-14
        assert abs(gauss.p_value(x / 2.0, 1, 1) - erfc(math.sqrt(x / 2))) < 1e-14
        assert abs(gauss.p_value(x / 2.0, 1, 4) - math.exp(-x / 2) * (1 + x / 2)) < 1e-14
    assert gauss.p_max(0.0, 5, 100, 1) == 1.0
    assert abs(gauss.p_max(0.02, 5, 100, 2) - (1 - (1 - math.exp(-2.0)) ** 5)) < 1e-14
    assert abs(gauss.p_min(0.01, 3, 100, 2) - math.exp(-1.0) ** 3) < 1e-15


def test_analytic_null_is_calibrated():
    # independent Gaussian X, Y given Z: the p-values are near uniform
    g = np.random.default_rng(11)
    ps = []
    for _ in range(400):
        z = g.standard_normal((2, 500))
        x = (z[0] + g.standard_normal(500))[None, :].astype(np.float32)
        y = (z[1] + g.standard_normal(500))[None, :].astype(np.float32)
        ps.append(gauss.p_value(gauss.cmi_gauss(x, y, z.astype(np.float32)), 500, 1))
    ps = np.array(ps)
    assert 0.03 < np.mean(ps < 0.05) < 0.08
    assert abs(np.mean(ps) - 0.5) < 0.05


def test_analytic_network_recovers_the_linear_var():
    # Statistical pin of the Gaussian network inference (VAR section: the
    # Gaussian estimator on linear VAR processes reaches high precision and
    # recall once T is in the thousands): every link of the 10-node VAR.
    from oracle import network
    from synth import gen
    s, links = gen.var_network(10, 3000, seed=0)
    adj, _, _ = network.infer_network(s, null="analytic")
    m = network.link_metrics(adj, synth.truth_adjacency(10, links))
    assert m["precision"] == 1.0 and m["recall"] == 1.0
