"""Parity of the HIP estimator with the oracle.

Radii and the three neighbour counts must match the oracle bit for bit
(they are exact: one float32 subtraction per coordinate, exact |.| and max,
strict integer counts); the CMI must match within 1e-9 absolute (both sides
sum float64 digamma terms, in different but fixed orders).  Every surrogate is
checked against the oracle run on X permuted with the oracle's own
implementation of the permutation.
"""

import json
import os
import sys

import numpy as np
import pytest

import paper_1902_06828_amd as mte
import synth
from oracle import cksg, ksg, perm

pytestmark = pytest.mark.gpu

TOL = 1e-9
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_estimates(X, Y, Z, k, S, seed, cand, queries=None, theiler=0):
    """[(cmi or None, eps, nxz, nyz, nz)] for the estimate and its S surrogates."""
    n = X.shape[1]
    out = []
    for e in range(S + 1):
        Xe = X if e == 0 else ksg.permute_rows(X, perm.permutation(seed, cand, e - 1, n))
        eps, a, b, c, v = cksg.eps_and_counts(Xe, Y, Z, k, queries=queries, theiler=theiler)
        out.append((v, eps, a, b, c))
    return out


def check_against_oracle(X, Y, Z, k, S=0, seed=11, cand=3):
    cmi, eps, cx, cy, cz = mte.cmi_ksg_diag(X, Y, Z, k, S, seed, cand)
    ref = oracle_estimates(X, Y, Z, k, S, seed, cand)
    for e, (v, re, ra, rb, rc) in enumerate(ref):
        assert np.array_equal(eps[e].view(np.uint32), re.view(np.uint32)), f"eps differ, estimate {e}"
        assert np.array_equal(cx[e], ra), f"n_xz differ, estimate {e}"
        assert np.array_equal(cy[e], rb), f"n_yz differ, estimate {e}"
        assert np.array_equal(cz[e], rc), f"n_z differ, estimate {e}"
        assert abs(cmi[e] - v) <= TOL, (e, cmi[e], v)
    return cmi, eps, cx, cy, cz


def test_hand_counted_case():
    g = json.load(open(os.path.join(GOLD, "hand_counted_k2_n6.json")))
    f = lambda a: np.array([a], np.float32)
    say("hand-counted case")
    cmi, eps, cx, cy, cz = mte.cmi_ksg_diag(f(g["X"]), f(g["Y"]), f(g["Z"]), g["k"])
    assert eps[0].tolist() == g["eps"]
    assert cx[0].tolist() == g["n_xz"] and cy[0].tolist() == g["n_yz"] and cz[0].tolist() == g["n_z"]
    assert abs(cmi[0] + 1 / 120) < 1e-14
    assert abs(mte.cmi_ksg(f(g["X"]), f(g["Y"]), f(g["Z"]), g["k"]) + 1 / 120) < 1e-14


CASES = [
    # (n, (dx, dy, dz), k, kind, S)
    (2, (1, 1, 0), 1, "normal", 0),
    (5, (1, 1, 0), 4, "normal", 2),
    (17, (1, 1, 1), 4, "grid", 3),
    (64, (1, 1, 5), 4, "normal", 2),
    (65, (2, 1, 3), 3, "dup", 2),
    (300, (1, 1, 5), 4, "normal", 3),
    (777, (1, 2, 4), 7, "grid", 2),
    (1500, (3, 1, 9), 8, "wide", 1),
    (2000, (1, 1, 15), 16, "normal", 1),
    (513, (16, 8, 31), 5, "tiny", 1),
    (256, (1, 1, 0), 4, "tiny", 2),
    (129, (4, 1, 2), 1, "dup", 4),
]


@pytest.mark.parametrize("n,dims,k,kind,S", CASES)
def test_random_parity(n, dims, k, kind, S):
    say("case", n, dims, k, kind, S)
    X, Y, Z = synth.random_points(n, dims, seed=n * 7 + k, kind=kind)
    check_against_oracle(X, Y, Z, k, S)


def test_c1_gaussian_parity():
    X, Y, Z, true = synth.c1_gaussian(1000, 1)
    say("C1 gaussian")
    cmi, *_ = check_against_oracle(X, Y, Z, 4, 0)
    assert abs(cmi[0] - true) < 0.1


def test_all_duplicates_give_zero_radius():
    n = 50
    X = np.zeros((1, n), np.float32)
    say("all duplicates")
    cmi, eps, cx, cy, cz = check_against_oracle(X, X.copy(), X.copy(), 4, 1)
    assert np.all(eps == 0) and np.all(cx == 0)


def test_overflowing_differences():
    g = np.random.default_rng(5)
    n = 200
    vals = np.array([-3e38, 3e38, 0.0, 1.0, -2.5e38], np.float32)
    X, Y, Z = (vals[g.integers(0, 5, size=(d, n))] for d in (1, 1, 2))
    say("overflow to inf")
    check_against_oracle(np.ascontiguousarray(X), np.ascontiguousarray(Y), np.ascontiguousarray(Z), 4, 2)


def test_splits_do_not_change_results(monkeypatch):
    monkeypatch.setenv("MTE_FORCE_MODE", "brute")
    X, Y, Z = synth.random_points(3000, (1, 1, 5), seed=9)
    res = []
    for split in ("0", "1", "4"):
        monkeypatch.setenv("MTE_FORCE_SPLIT", split)
        say("split multiplier", split)
        res.append(mte.cmi_ksg_diag(X, Y, Z, 4, 3, 5, 1))
    for r in res[1:]:
        for a, b in zip(res[0], r):
            assert np.array_equal(a, b)


def test_every_tile_configuration(monkeypatch):
    # some tile configurations spill registers and need the runtime's scratch
    # memory: the device must have room left for it
    torch = pytest.importorskip("torch")
    free, total = torch.cuda.mem_get_info()
    say("device memory free", free >> 20, "MiB of", total >> 20)
    monkeypatch.setenv("MTE_FORCE_MODE", "brute")
    X, Y, Z = synth.random_points(700, (1, 1, 4), seed=21)
    ref = mte.cmi_ksg_diag(X, Y, Z, 4, 9, 2, 0)
    tested = 0
    for idx, cfg in enumerate(mte.mte_tile_configs()):
        kmax, g, qp, dzm, dym, dxm = cfg
        if kmax != 4:
            continue
        for split in ("0", "2"):
            monkeypatch.setenv("MTE_FORCE_VARIANT", str(idx))
            monkeypatch.setenv("MTE_FORCE_SPLIT", split)
            say("variant", idx, cfg, "split", split)
            got = mte.cmi_ksg_diag(X, Y, Z, 4, 9, 2, 0)
            for a, b in zip(ref, got):
                assert np.array_equal(a, b), (idx, cfg, split)
            tested += 1
    assert tested >= 8
    # the radius list capacities 8 and 16 against the oracle
    for k in (6, 12):
        for idx, cfg in enumerate(mte.mte_tile_configs()):
            if cfg[0] == (8 if k <= 8 else 16) and cfg[5] == 1 and cfg[3] >= 4:
                monkeypatch.setenv("MTE_FORCE_VARIANT", str(idx))
                monkeypatch.setenv("MTE_FORCE_SPLIT", "0")
                say("k", k, "variant", idx, cfg)
                check_against_oracle(X, Y, Z, k, 2)


def test_batched_equals_plain():
    X, Y, Z = synth.random_points(1200, (1, 1, 3), seed=33)
    S, seed = 6, 99
    say("batched vs plain")
    v, surr = mte.cmi_ksg_surrogates(X, Y, Z, 4, S, seed)
    assert v == mte.cmi_ksg(X, Y, Z, 4)
    for s in range(S):
        Xs = ksg.permute_rows(X, perm.permutation(seed, 0, s, X.shape[1]))
        assert surr[s] == mte.cmi_ksg(Xs, Y, Z, 4)


def test_stage_timing_events():
    # timed launches bracket each stage with events, sharing one where two
    # stages meet on a stream; every launch adds one to each list stage and
    # the results are those of untimed launches (one job, then the several-job
    # launches of a greedy search, which join after the row-order kernel)
    torch = pytest.importorskip("torch")
    X, Y, Z = synth.random_points(2500, (1, 1, 5), seed=46)
    S, seed, cand = 20, 9, 2
    ref = mte.cmi_ksg_diag(X, Y, Z, 4, S, seed, cand)[0]
    dev = torch.device("cuda:0")
    dX, dY, dZ = (torch.from_numpy(a).to(dev) for a in (X, Y, Z))
    out = torch.zeros(S + 1, dtype=torch.float64, device=dev)
    series, _ = synth.var_network(4, 2000, seed=3)
    kw = dict(max_lag_sources=3, alpha=0.05, S=50, seed=2)
    stages = ("build", "scan", "fallback", "reduce", "permute")
    for st in mte._lib.STAGES:
        mte.mte_kernel_timing_stage(st, reset=True)
    mte.mte_kernel_timing(True)
    try:
        for rep in range(3):
            say("timed one-job launch", rep)
            out.zero_()
            mte.cmi_ksg_surrogates_dev(dX, dY, dZ, 4, S, seed, cand, out)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref), rep
            for st in stages:
                n, ms = mte.mte_kernel_timing_stage(st)
                assert n == rep + 1 and ms > 0.0, (st, n, ms)
        say("timed greedy search")
        timed = mte.mte_select_sources(series, 0, [1, 2, 3], **kw)
        for st in stages:
            n, ms = mte.mte_kernel_timing_stage(st)
            assert n > 3 and ms > 0.0, (st, n, ms)
    finally:
        mte.mte_kernel_timing(False)
        for st in mte._lib.STAGES:
            mte.mte_kernel_timing_stage(st, reset=True)
    say("untimed greedy search")
    plain = mte.mte_select_sources(series, 0, [1, 2, 3], **kw)
    for key in ("target_past", "sources", "sources_before_omnibus", "omnibus_te", "omnibus_p", "n_estimates"):
        assert timed[key] == plain[key]


def test_device_api_and_graph_replay():
    torch = pytest.importorskip("torch")
    X, Y, Z = synth.random_points(2500, (1, 1, 5), seed=44)
    S, seed, cand = 20, 7, 5
    ref = mte.cmi_ksg_diag(X, Y, Z, 4, S, seed, cand)[0]
    dev = torch.device("cuda:0")
    dX, dY, dZ = (torch.from_numpy(a).to(dev) for a in (X, Y, Z))
    out = torch.zeros(S + 1, dtype=torch.float64, device=dev)
    for rep in range(4):
        say("device call", rep)
        out.zero_()
        mte.cmi_ksg_surrogates_dev(dX, dY, dZ, 4, S, seed, cand, out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), rep
    # direct launches with per-stage events (the timing path) on the same shape
    say("device call with kernel timing")
    mte.mte_kernel_timing(True)
    try:
        out.zero_()
        mte.cmi_ksg_surrogates_dev(dX, dY, dZ, 4, S, seed, cand, out)
        torch.cuda.synchronize()
    finally:
        mte.mte_kernel_timing(False)
        for st in mte._lib.STAGES:
            mte.mte_kernel_timing_stage(st, reset=True)
    assert np.array_equal(out.cpu().numpy(), ref)
    # inputs changed in place reach the next replay: every launch rebuilds the
    # permuted X and the build's copy of Y and Z
    X2, _, Z2 = synth.random_points(2500, (1, 1, 5), seed=45)
    dX.copy_(torch.from_numpy(X2))
    dZ.copy_(torch.from_numpy(Z2))
    ref3 = mte.cmi_ksg_diag(X2, Y, Z2, 4, S, seed, cand)[0]
    assert abs(ref3[0] - cksg.cmi_ksg(X2, Y, Z2, 4)) <= TOL
    for rep in range(2):
        say("device call after an in-place update", rep)
        out.zero_()
        mte.cmi_ksg_surrogates_dev(dX, dY, dZ, 4, S, seed, cand, out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref3), rep
    dX.copy_(torch.from_numpy(X))
    dZ.copy_(torch.from_numpy(Z))
    one = torch.zeros(1, dtype=torch.float64, device=dev)
    mte.cmi_ksg_dev(dX, dY, dZ, 4, one)
    torch.cuda.synchronize()
    assert one.item() == ref[0]
    # a strided view: rows 100..2099 of columns with leading dimension 2500
    sub = torch.zeros(S + 1, dtype=torch.float64, device=dev)
    mte.cmi_ksg_surrogates_dev(dX[:, 100:], dY[:, 100:], dZ[:, 100:], 4, S, seed, cand, sub, n=2000)
    torch.cuda.synchronize()
    ref2 = mte.cmi_ksg_diag(np.ascontiguousarray(X[:, 100:2100]), np.ascontiguousarray(Y[:, 100:2100]),
                            np.ascontiguousarray(Z[:, 100:2100]), 4, S, seed, cand)[0]
    assert np.array_equal(sub.cpu().numpy(), ref2)


def test_full_size_c2_sampled():
    # one TE estimate and 200 surrogates at N = 10000 (10-node VAR), as timed
    # by the benchmark; rows sampled from every 25th estimate are checked
    # against the oracle one query at a time, estimate 0 and surrogate 0 in full
    X, Y, Z, meta = synth.c2_te_inputs(10000, seed=2)
    S, seed, k = 200, 2, 4
    say("C2 full size")
    cmi, eps, cx, cy, cz = mte.cmi_ksg_diag(X, Y, Z, k, S, seed, 0)
    n = X.shape[1]
    rows = np.random.default_rng(0).choice(n, size=24, replace=False)
    rows = np.concatenate([rows, [0, 1, n - 1, n - 64, 63, 64]])
    for e in range(0, S + 1, 25):
        Xe = X if e == 0 else ksg.permute_rows(X, perm.permutation(seed, 0, e - 1, n))
        re, ra, rb, rc, _ = cksg.eps_and_counts(Xe, Y, Z, k, queries=rows)
        assert np.array_equal(eps[e, rows], re) and np.array_equal(cx[e, rows], ra)
        assert np.array_equal(cy[e, rows], rb) and np.array_equal(cz[e, rows], rc)
    for e in (0, 1):
        Xe = X if e == 0 else ksg.permute_rows(X, perm.permutation(seed, 0, e - 1, n))
        assert abs(cmi[e] - cksg.cmi_ksg(Xe, Y, Z, k)) <= TOL
    # properties at any size
    assert np.all((cx >= 0) & (cx <= cz) & (cy <= cz) & (cz <= n - 1))
    assert cmi[0] > np.max(cmi[1:])          # a true coupling beats every surrogate
    # the device form used by the benchmark gives the same bits
    torch = pytest.importorskip("torch")
    dev = torch.device("cuda:0")
    out = torch.zeros(S + 1, dtype=torch.float64, device=dev)
    mte.cmi_ksg_surrogates_dev(*(torch.from_numpy(a).to(dev) for a in (X, Y, Z)), k, S, seed, 0, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), cmi)


@pytest.mark.parametrize("n,dims,k,S,w", [(1, (1, 1, 0), 1, 0, 0), (130, (1, 1, 3), 4, 0, 0), (1000, (2, 1, 5), 8, 2, 1),
                                          (777, (1, 2, 0), 4, 6, 0), (3001, (1, 1, 12), 16, 1, 3),
                                          (513, (3, 4, 20), 5, 3, 0), (2048, (1, 1, 5), 4, 30, 2)])
def test_solo_equals_persistent(monkeypatch, n, dims, k, S, w):
    # jobs with few estimates take the few-estimate kernel (a wave per query
    # tile, lanes striding over the reference rows); forced onto it or onto
    # the persistent kernel, every radius, count and estimate must agree, and
    # agree with the oracle
    n = max(n, k + 1 + 2 * w)
    X, Y, Z = synth.random_points(n, dims, seed=n + S, kind="grid" if S == 2 else "normal")
    out = {}
    for mode in ("solo", "brute"):
        monkeypatch.setenv("MTE_FORCE_MODE", mode)
        say("solo vs persistent", n, dims, k, S, w, mode)
        out[mode] = mte.cmi_ksg_diag(X, Y, Z, k, S, 4, 2, theiler=w)
    for a, b in zip(out["solo"], out["brute"]):
        assert np.array_equal(a, b)
    cmi, eps, cx, cy, cz = out["solo"]
    for e, (v, re, ra, rb, rc) in enumerate(oracle_estimates(X, Y, Z, k, min(S, 3), 4, 2, theiler=w)):
        assert np.array_equal(eps[e], re) and np.array_equal(cx[e], ra)
        assert np.array_equal(cy[e], rb) and np.array_equal(cz[e], rc)
        assert abs(cmi[e] - v) <= TOL
