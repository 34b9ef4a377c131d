"""The Theiler window (rows |i - j| <= w left out of row i's neighbours) on both
GPU paths against the oracle, and through the greedy driver and the request
loop."""

import sys

import numpy as np
import pytest

import paper_1902_06828_amd as mte
import synth
from oracle import cksg, greedy, ksg, perm

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check(X, Y, Z, k, S, w, seed=5, cand=2):
    cmi, eps, cx, cy, cz = mte.cmi_ksg_diag(X, Y, Z, k, S, seed, cand, theiler=w)
    n = X.shape[1]
    for e in range(S + 1):
        Xe = X if e == 0 else ksg.permute_rows(X, perm.permutation(seed, cand, e - 1, n))
        re, ra, rb, rc, v = cksg.eps_and_counts(Xe, Y, Z, k, theiler=w)
        assert np.array_equal(eps[e], re), (e, w)
        assert np.array_equal(cx[e], ra) and np.array_equal(cy[e], rb) and np.array_equal(cz[e], rc), (e, w)
        assert abs(cmi[e] - v) <= 1e-9
    return cmi


CASES = [
    # (n, dims, k, kind, w)
    (200, (1, 1, 0), 4, "normal", 1),
    (257, (1, 1, 2), 4, "grid", 3),
    (600, (1, 1, 5), 4, "normal", 7),
    (300, (2, 1, 3), 3, "dup", 2),
    (130, (1, 2, 1), 1, "wide", 10),
    (1000, (1, 2, 0), 4, "grid", 5),
    # one Z and one Y column: counts from ranks of z, window rows taken out
    (400, (1, 1, 1), 4, "grid", 4),
    (700, (2, 1, 1), 4, "dup", 2),
    (513, (1, 1, 1), 3, "normal", 70),
]


@pytest.mark.parametrize("mode", ["brute", "list"])
@pytest.mark.parametrize("n,dims,k,kind,w", CASES)
def test_theiler_parity(monkeypatch, mode, n, dims, k, kind, w):
    monkeypatch.setenv("MTE_FORCE_MODE", mode)
    say("theiler", mode, n, dims, k, kind, w)
    X, Y, Z = synth.random_points(n, dims, seed=n + w, kind=kind)
    check(X, Y, Z, k, 9, w)


def test_theiler_small_caps_and_full_size(monkeypatch):
    # list path with tiny capacities (most pairs redone over all rows)
    monkeypatch.setenv("MTE_FORCE_MODE", "list")
    monkeypatch.setenv("MTE_LIST_CAP", "3,5")
    X, Y, Z = synth.random_points(400, (1, 1, 3), seed=77)
    say("theiler, tiny caps")
    check(X, Y, Z, 4, 9, 4)
    X, Y, _ = synth.random_points(400, (1, 1, 0), seed=78)
    say("theiler, tiny caps, no Z")
    check(X, Y, None, 4, 9, 4)
    monkeypatch.delenv("MTE_LIST_CAP")
    # the benchmark's sample with a window of 5: both paths, same bits
    X, Y, Z, _ = synth.c2_te_inputs(10000, seed=2)
    out = {}
    for mode in ("brute", "list"):
        monkeypatch.setenv("MTE_FORCE_MODE", mode)
        say("C2 with w = 5, mode", mode)
        out[mode] = mte.cmi_ksg_diag(X, Y, Z, 4, 40, 2, 0, theiler=5)
    for a, b in zip(out["brute"], out["list"]):
        assert np.array_equal(a, b)
    rows = np.array([0, 1, 2, 3, 4, 5, 6, 9994, 9999, 5000])
    eps, cx = out["list"][1], out["list"][2]
    re, ra, _, _, _ = cksg.eps_and_counts(X, Y, Z, 4, queries=rows, theiler=5)
    assert np.array_equal(eps[0, rows], re) and np.array_equal(cx[0, rows], ra)


def test_theiler_greedy_and_served():
    series, links = synth.var_network(4, 500, seed=3)
    target = min(i for (i, _, _, _) in links)
    cands = [j for j in range(4) if j != target]
    w = int(mte.mte_autocorr_decay_time(series[target], 20))
    say("greedy with theiler", w)
    kw = dict(max_lag_sources=2, alpha=0.1, k=4, max_lag_target=2, seed=3)
    res = mte.mte_select_sources(series, target, cands, S=20, theiler=w, **kw)
    ora = greedy.select_sources(series, target, cands, max_lag_sources=2, max_lag_target=2, alpha=0.1, k=4,
                                n_surr=20, seed=3, estimator=cksg.cmi_ksg, theiler=w)
    key = lambda v: [(a, b) for (a, b, _, _) in v]
    assert key(res["target_past"]) == key(ora["target_past"])
    assert key(res["sources"]) == key(ora["sources"])
    assert abs(res["omnibus_te"] - ora["omnibus_te"]) <= 1e-9 and res["omnibus_p"] == ora["omnibus_p"]
    sid = mte.mte_series_register(series)
    served = mte.mte_select_sources_sid(sid, target, cands, S=20, theiler=w, **kw)
    mte.mte_series_release(sid)
    for name in ("target_past", "sources", "omnibus_te", "omnibus_p"):
        assert served[name] == res[name]
