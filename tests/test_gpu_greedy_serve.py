"""The library's greedy selection and request loop against the oracle.

Greedy: the same readings of the paper on both sides (see oracle/greedy.py),
so the selections, p-values and every reported estimate must agree; the
library's values within 1e-9 of the oracle's.  Request loop: each request's
result is bitwise the same alone and in a mix of concurrent requests of uneven
N and conditioning dimension, and equal to the direct estimator.
"""

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


def est(x, y, z, k):
    return cksg.cmi_ksg(x, y, z, k)


def compare_results(lib_res, ora):
    def same(a, b):
        assert [(n, l) for (n, l, _, _) in a] == [(n, l) for (n, l, _, _) in b]
        for (_, _, c1, p1), (_, _, c2, p2) in zip(a, b):
            assert abs(c1 - c2) <= 1e-9 and p1 == p2
    same(lib_res["target_past"], ora["target_past"])
    same(lib_res["sources_before_omnibus"], ora["sources_before_omnibus"])
    same(lib_res["sources"], ora["sources"])
    assert abs(lib_res["omnibus_te"] - ora["omnibus_te"]) <= 1e-9
    assert lib_res["omnibus_p"] == ora["omnibus_p"]
    assert lib_res["significant"] == ora["significant"]
    assert lib_res["n_estimates"] == ora["n_estimates"]


@pytest.mark.parametrize("seed", [1, 2])
def test_greedy_matches_oracle(seed):
    series, links = synth.var_network(5, 400, seed=seed)
    target = min(i for (i, _, _, _) in links)
    cands = [j for j in range(5) if j != target]
    kw = dict(max_lag_sources=3, alpha=0.1, k=4, max_lag_target=3, seed=seed)
    say("greedy", seed, "target", target)
    lib_res = mte.mte_select_sources(series, target, cands, S=20, **kw)
    ora = greedy.select_sources(series, target, cands, max_lag_sources=3, max_lag_target=3,
                                alpha=0.1, k=4, n_surr=20, seed=seed, estimator=est)
    compare_results(lib_res, ora)
    say("served greedy", seed)
    sid = mte.mte_series_register(series)
    served = mte.mte_select_sources_sid(sid, target, cands, S=20, **kw)
    mte.mte_series_release(sid)
    compare_results(served, ora)


def test_greedy_recovers_var_parents():
    # 10-node VAR, N = 3000: the selected sources are true parents
    series, links = synth.var_network(10, 3000, seed=3)
    target = min(i for (i, _, _, _) in links)
    parents = {(j, l) for (i, j, l, _) in links if i == target}
    cands = [j for j in range(10) if j != target]
    say("recovery", target, parents)
    res = mte.mte_select_sources(series, target, cands, max_lag_sources=5, alpha=0.05, S=100, seed=3)
    got = {(n, l) for (n, l, _, _) in res["sources"]}
    assert res["significant"]
    assert len(got & parents) >= 1 and len(got - parents) <= 1


def _requests(P, T, count, seed):
    g = np.random.default_rng(seed)
    reqs = []
    for r in range(count):
        n = int(g.choice([400, 1000, 2500]))
        dz = int(g.integers(0, 7))
        S = int(g.choice([0, 5, 20]))
        d = 2 + dz
        nodes = g.integers(0, P, size=d).astype(np.int32)
        lags = np.concatenate([[int(g.integers(1, 6))], [0], g.integers(1, 6, size=dz)]).astype(np.int32)
        t0 = 5 + int(g.integers(0, T - n - 5))
        reqs.append(dict(nodes=nodes, lags=lags, dx=1, dy=1, dz=dz, t0=t0, n=n, k=4, S=S,
                         seed=int(seed), cand=r))
    return reqs


def test_request_loop_alone_vs_mix():
    P, T = 20, 3005
    series, _ = synth.clm_network(P, T - 5, seed=4)
    sid = mte.mte_series_register(series)
    reqs = _requests(P, T, 40, 8)
    mte.mte_serve_get_stats(reset=True)
    say("mix of", len(reqs))
    tickets = [mte.mte_submit(sid, **q) for q in reqs]
    mix = [mte.mte_wait(t, q["S"]) for t, q in zip(tickets, reqs)]
    st = mte.mte_serve_get_stats(reset=True)
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    # latency phases: none negative, each p99 within the total's, and the
    # tail's phases add up to its latencies (at least the p99 latency)
    for ph in ("queue", "host", "device"):
        assert 0.0 <= st[ph + "_p50_s"] <= st[ph + "_p99_s"] <= st["p99_latency_s"] * (1 + 1e-9)
    assert 1 <= st["tail_requests"] <= len(reqs)
    tail = st["tail_queue_s"] + st["tail_host_s"] + st["tail_device_s"]
    assert tail >= st["p99_latency_s"] * (1 - 1e-9)
    assert st["tail_mean_n"] in {400.0, 1000.0, 2500.0} or 400.0 <= st["tail_mean_n"] <= 2500.0
    assert 1.0 <= st["tail_mean_batch_requests"] <= len(reqs)
    say("alone")
    for q, (v, s) in zip(reqs, mix):
        t = mte.mte_submit(sid, **q)
        v1, s1 = mte.mte_wait(t, q["S"])
        assert v1 == v and np.array_equal(s1, s)
    # and the same as the direct estimator on the same windows
    for q, (v, s) in list(zip(reqs, mix))[:6]:
        cols = [series[nd, q["t0"] - lg: q["t0"] - lg + q["n"]] for nd, lg in zip(q["nodes"], q["lags"])]
        X = np.ascontiguousarray(np.array(cols[:1], np.float32))
        Y = np.ascontiguousarray(np.array(cols[1:2], np.float32))
        Z = np.ascontiguousarray(np.array(cols[2:], np.float32)) if q["dz"] else None
        cmi = mte.cmi_ksg_diag(X, Y, Z, 4, q["S"], q["seed"], q["cand"])[0]
        assert cmi[0] == v and np.array_equal(cmi[1:], s)
        if q["n"] <= 1000:
            assert abs(v - cksg.cmi_ksg(X, Y, Z, 4)) <= 1e-9
    mte.mte_series_release(sid)


def test_admission_rejects_oversized_request():
    series = np.random.default_rng(1).standard_normal((3, 5000)).astype(np.float32)
    sid = mte.mte_series_register(series)
    mte.mte_init(0, 1 << 20)                  # 1 MiB budget
    try:
        t = mte.mte_submit(sid, [0, 1, 2], [1, 0, 1], 1, 1, 1, 5, 4900, k=4, S=200)
        with pytest.raises(mte.MteError) as e:
            mte.mte_wait(t, 200)
        assert e.value.code == mte._lib.MTE_ENOMEM
        t = mte.mte_submit(sid, [0, 1], [1, 0], 1, 1, 0, 5, 300, k=4, S=0)
        v, _ = mte.mte_wait(t, 0)
        assert np.isfinite(v)
    finally:
        mte.mte_init(0, 64 << 30)
    mte.mte_series_release(sid)


def _req(S, cand):
    return dict(nodes=[1, 0, 0, 0, 0], lags=[1, 0, 1, 2, 3], dx=1, dy=1, dz=3, t0=5, n=3000, k=4, S=S, seed=3,
                cand=cand)


def test_admission_waits_for_memory():
    # two requests that each fit the HBM budget but not together: the second
    # waits at the queue front until the first retires, and both give the
    # results they give alone
    series, _ = synth.var_network(6, 3000, seed=13)
    sid = mte.mte_series_register(series)
    S = 60
    mte.mte_serve_get_stats(reset=True)
    alone = []
    for c in (0, 1):
        say("alone, request", c)
        alone.append(mte.mte_wait(mte.mte_submit(sid, **_req(S, c)), S))
    st = mte.mte_serve_get_stats(reset=True)
    one, old_budget = st["peak_bytes_in_use"], st["budget_bytes"]
    assert one > 0 and st["waited"] == 0
    mte.mte_init(0, one + one // 2)
    try:
        say("together under a budget of 1.5 requests")
        tickets = [mte.mte_submit(sid, **_req(S, c)) for c in (0, 1)]
        mix = [mte.mte_wait(t, S) for t in tickets]
        st = mte.mte_serve_get_stats(reset=True)
    finally:
        mte.mte_init(0, old_budget)
    assert st["completed"] == 2 and st["rejected"] == 0 and st["waited"] >= 1
    assert st["peak_bytes_in_use"] <= one + one // 2
    for (v, s), (v1, s1) in zip(alone, mix):
        assert v == v1 and np.array_equal(s, s1)
    mte.mte_series_release(sid)


def test_wait_timeout_keeps_the_ticket():
    # a zero timeout on a 201-estimate request at N = 10^4 returns
    # MTE_ETIMEOUT (nothing finishes that fast); the ticket stays valid and a
    # second wait returns the result
    series, _ = synth.var_network(4, 10000, seed=14)
    sid = mte.mte_series_register(series)
    q = dict(nodes=[1, 0, 0, 0], lags=[2, 0, 1, 2], dx=1, dy=1, dz=2, t0=5, n=10000, k=4, S=200, seed=5, cand=2)
    say("wait with timeout 0")
    t = mte.mte_submit(sid, **q)
    with pytest.raises(mte.MteError) as e:
        mte.mte_wait(t, 200, timeout_s=0.0)
    assert e.value.code == mte._lib.MTE_ETIMEOUT
    v, s = mte.mte_wait(t, 200)
    cols = [series[nd, 5 - lg: 5 - lg + 10000] for nd, lg in zip(q["nodes"], q["lags"])]
    f = lambda a: np.ascontiguousarray(np.array(a, np.float32))
    cmi = mte.cmi_ksg_diag(f(cols[:1]), f(cols[1:2]), f(cols[2:]), 4, 200, 5, 2)[0]
    assert cmi[0] == v and np.array_equal(cmi[1:], s)
    mte.mte_series_release(sid)


def test_cancel_stops_a_running_search():
    import threading
    import time
    series, links = synth.var_network(10, 10000, seed=15)
    sid = mte.mte_series_register(series)
    target = min(i for (i, _, _, _) in links)
    box = {}

    def run():
        try:
            box["res"] = mte.mte_select_sources_sid(sid, target, [j for j in range(10) if j != target],
                                                    max_lag_sources=5, S=200, seed=1)
        except mte.MteError as err:
            box["err"] = err

    say("search, then cancel")
    th = threading.Thread(target=run)
    th.start()
    time.sleep(0.02)
    mte.mte_serve_cancel(sid)
    th.join(timeout=60)
    assert not th.is_alive()
    assert "err" in box and box["err"].code == mte._lib.MTE_ECANCELED
    with pytest.raises(mte.MteError) as e:
        mte.mte_submit(sid, [1, 0], [1, 0], 1, 1, 0, 5, 300, k=4, S=0)
    assert e.value.code == mte._lib.MTE_ECANCELED
    mte.mte_series_release(sid)
