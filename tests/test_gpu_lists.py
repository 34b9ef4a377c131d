"""The neighbour-list path against the oracle and against the all-pairs kernel.

The list path decides each (row, estimate) pair from per-row neighbour lists
in the (Y,Z) and Z subspaces and redoes the pairs the lists cannot decide over
all rows.  Its radii and counts must equal the oracle's bit for bit, whatever
the list capacities (tiny capacities force most pairs through the redo), and
its CMI values must be bitwise those of the all-pairs kernel (same counts, same
fixed summation order).
"""

import sys

import numpy as np
import pytest

import paper_1902_06828_amd as mte
import synth
from test_gpu_parity import CASES, check_against_oracle

pytestmark = pytest.mark.gpu

# every case with Z, and the cases without Z with one X column (their n_x
# comes from range counts on the sorted X column)
LIST_CASES = [c for c in CASES if c[1][2] > 0 or c[1][0] == 1] + [
    (3000, (1, 2, 0), 4, "grid", 3), (1000, (1, 1, 0), 4, "dup", 2), (4097, (1, 1, 0), 8, "wide", 1)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("caps", ["default", "16,40", "2,3"])
@pytest.mark.parametrize("n,dims,k,kind,S", LIST_CASES)
def test_list_path_parity(monkeypatch, caps, n, dims, k, kind, S):
    monkeypatch.setenv("MTE_FORCE_MODE", "list")
    if caps != "default":
        monkeypatch.setenv("MTE_LIST_CAP", caps)
    say("list case", n, dims, k, kind, S, "caps", caps)
    X, Y, Z = synth.random_points(n, dims, seed=n * 7 + k, kind=kind)
    mte.mte_list_stats(reset=True)
    check_against_oracle(X, Y, Z, k, S + 8)
    pairs, undecided = mte.mte_list_stats(reset=True)
    assert pairs == n * (S + 9)
    if caps == "2,3" and n > 4 * k:
        assert undecided > 0          # the redo over all rows was exercised


@pytest.mark.parametrize("n,dims,kind,seed", [(3000, (1, 1, 5), "normal", 1), (2048, (2, 1, 3), "dup", 2),
                                              (1000, (1, 2, 7), "grid", 3), (4097, (1, 1, 1), "wide", 4),
                                              # more dimensions outside Z than in it: the capacities
                                              # grow (to 8192 / 16384 entries) but stay below N - 1
                                              (20000, (3, 1, 1), "normal", 5), (12000, (2, 1, 2), "normal", 6),
                                              # without Z: up to the largest N of the in-LDS X sort
                                              (4000, (1, 1, 0), "grid", 7), (16384, (1, 2, 0), "normal", 8),
                                              (10000, (1, 1, 0), "dup", 9)])
def test_list_equals_all_pairs(monkeypatch, n, dims, kind, seed):
    X, Y, Z = synth.random_points(n, dims, seed=seed, kind=kind)
    out = {}
    for mode in ("brute", "list"):
        monkeypatch.setenv("MTE_FORCE_MODE", mode)
        say("mode", mode, n, dims, kind)
        out[mode] = mte.cmi_ksg_diag(X, Y, Z, 4, 30, seed, 2)
    for a, b in zip(out["brute"], out["list"]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("S", [63, 99, 127, 130])
def test_estimate_groups(monkeypatch, S):
    # a launch of one job runs its lanes over groups of 64 estimates, the last
    # group taking the remainder (E = 64, 100, 128, 131: one group, one group
    # of 100, two groups, two groups of 64 and 67), and renumbers the blocks
    # across the XCDs; every (row, estimate) result must be unchanged
    X, Y, Z = synth.random_points(1500, (1, 1, 3), seed=S)
    out = {}
    for mode in ("brute", "list"):
        monkeypatch.setenv("MTE_FORCE_MODE", mode)
        say("estimate groups, S", S, "mode", mode)
        out[mode] = mte.cmi_ksg_diag(X, Y, Z, 4, S, 3, 1)
    for a, b in zip(out["brute"], out["list"]):
        assert np.array_equal(a, b)


def test_full_size_c2_list_equals_all_pairs(monkeypatch):
    # the benchmark's workload (N = 10000, 201 estimates) on both paths
    X, Y, Z, _ = synth.c2_te_inputs(10000, seed=2)
    out = {}
    for mode in ("brute", "list"):
        monkeypatch.setenv("MTE_FORCE_MODE", mode)
        say("C2 full size, mode", mode)
        mte.mte_list_stats(reset=True)
        out[mode] = mte.cmi_ksg_diag(X, Y, Z, 4, 200, 2, 0)
        if mode == "list":
            pairs, undecided = mte.mte_list_stats(reset=True)
            say("pairs", pairs, "redone over all rows", undecided)
            assert pairs == 10000 * 201 and undecided < pairs // 100
    for a, b in zip(out["brute"], out["list"]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("quantised", [False, True])
def test_shared_lists_across_jobs(monkeypatch, quantised):
    # several candidates with the same Y and Z (one list set) in one launch:
    # the greedy driver's batches; each must equal its own single-job result.
    # Such launches scan rows in a Morton order of (Y,Z); quantised values
    # put many rows in one cell (equal codes, told apart by the row index)
    series, links = synth.var_network(6, 1500, seed=6)
    if quantised:
        series = np.round(series * 2.0) / 2.0
    monkeypatch.setenv("MTE_FORCE_MODE", "list")
    target = min(i for (i, _, _, _) in links)
    cands = [j for j in range(6) if j != target]
    say("greedy with shared lists, target", target)
    res = mte.mte_select_sources(series, target, cands, max_lag_sources=3, alpha=0.05, S=40, seed=6)
    monkeypatch.setenv("MTE_FORCE_MODE", "brute")
    ref = mte.mte_select_sources(series, target, cands, max_lag_sources=3, alpha=0.05, S=40, seed=6)
    for key in ("target_past", "sources", "sources_before_omnibus"):
        assert res[key] == ref[key]
    assert res["omnibus_te"] == ref["omnibus_te"] and res["omnibus_p"] == ref["omnibus_p"]


@pytest.mark.parametrize("n", [16384, 16385])
def test_row_order_size_limit(monkeypatch, n):
    # launches of several jobs order the rows of sets with N <= 16384 (one
    # block, counting sort) and keep the index order above; both sides of the
    # limit against the all-pairs kernel (the series hold n + 5 samples, so
    # with a largest lag of 5 the embedding has N = n rows)
    series, links = synth.var_network(4, n, seed=7)
    assert series.shape[1] == n + 5
    target = min(i for (i, _, _, _) in links)
    cands = [j for j in range(4) if j != target]
    out = {}
    for mode in ("list", "brute"):
        monkeypatch.setenv("MTE_FORCE_MODE", mode)
        say("row order limit, N", n, "mode", mode)
        out[mode] = mte.mte_select_sources(series, target, cands, max_lag_sources=3, max_lag_target=5,
                                           alpha=0.05, S=40, seed=7)
    for key in ("target_past", "sources", "sources_before_omnibus", "omnibus_te", "omnibus_p", "n_estimates"):
        assert out["list"][key] == out["brute"][key]


def test_large_n_unpacked_histograms(monkeypatch):
    # N above 2^16 takes the build variant with 32-bit histograms; rows sampled
    # against the oracle, and the whole output against the all-pairs kernel
    from oracle import cksg, ksg, perm
    n, S, seed = 70000, 8, 12
    X, Y, Z = synth.random_points(n, (1, 1, 2), seed=seed)
    out = {}
    for mode in ("brute", "list"):
        monkeypatch.setenv("MTE_FORCE_MODE", mode)
        say("N = 70000, mode", mode)
        out[mode] = mte.cmi_ksg_diag(X, Y, Z, 4, S, seed, 1)
    for a, b in zip(out["brute"], out["list"]):
        assert np.array_equal(a, b)
    cmi, eps, cx, cy, cz = out["list"]
    rows = np.array([0, 1, 65535, 65536, 65537, n - 1] + list(np.random.default_rng(3).choice(n, 10, replace=False)))
    for e in (0, S):
        Xe = X if e == 0 else ksg.permute_rows(X, perm.permutation(seed, 1, e - 1, n))
        re, ra, rb, rc, _ = cksg.eps_and_counts(Xe, Y, Z, 4, queries=rows)
        assert np.array_equal(eps[e, rows], re) and np.array_equal(cx[e, rows], ra)
        assert np.array_equal(cy[e, rows], rb) and np.array_equal(cz[e, rows], rc)


def _overflow_points(n, dims, seed, kind):
    if kind == "mixed":
        # values whose differences are finite or overflow depending on the pair
        g = np.random.default_rng(seed)
        vals = np.array([-3e38, 3e38, 0.0, 1.0, -2.5e38], np.float32)
        return [None if d == 0 else np.ascontiguousarray(vals[g.integers(0, 5, size=(d, n))]) for d in dims]
    return synth.random_points(n, dims, seed=seed, kind=kind)


@pytest.mark.parametrize("caps", ["default", "16,40", "2,3"])
@pytest.mark.parametrize("n,dims,kind,some_inf", [(3000, (3, 1, 5), "cells", True), (2000, (1, 1, 5), "split", False),
                                                  (3000, (1, 2, 3), "cells", False), (200, (1, 1, 2), "mixed", False),
                                                  (3000, (1, 1, 0), "cells", False)])
def test_list_path_overflowing_differences(monkeypatch, caps, n, dims, kind, some_inf):
    # Differences that overflow to +inf.  With the default capacities a row's
    # rows at a finite (Y,Z) or Z distance fit its lists and the rest are at
    # +inf, so the first bucket a list leaves out is the +inf bucket; in the
    # "cells" inputs many rows also have fewer than k rows at a finite joint
    # distance (512 joint sign cells for 9 columns, ~6 rows each), so their
    # radius is +inf and their scans run to the sentinels.
    # Radii and counts bit for bit against the oracle on every estimate.
    monkeypatch.setenv("MTE_FORCE_MODE", "list")
    if caps != "default":
        monkeypatch.setenv("MTE_LIST_CAP", caps)
    X, Y, Z = _overflow_points(n, dims, 40 + n, kind)
    if kind != "mixed" and caps == "default" and Z is not None:
        # every row's finite (Y,Z) neighbours fit the smallest default list,
        # and some rows lie outside them
        yz = np.concatenate([Z, Y]) > 0
        _, inv, size = np.unique(yz.T, axis=0, return_inverse=True, return_counts=True)
        assert size.max() - 1 <= 1024 and size.min() - 1 < n - 1
    say("overflow case", n, dims, kind, "caps", caps)
    cmi, eps, *_ = check_against_oracle(X, Y, Z, 4, 8, seed=5, cand=1)
    if some_inf:
        assert np.isinf(eps).any() and np.isfinite(eps).any()


@pytest.mark.parametrize("dims,n,w", [((1, 1, 1), 4500, 0), ((1, 1, 5), 6000, 0), ((2, 1, 7), 5001, 3),
                                      ((1, 1, 12), 4097, 0), ((1, 1, 4), 9000, 2)])
def test_build_forms_agree(monkeypatch, dims, n, w):
    # the neighbour lists come from the generic two-pass build or, for one Y
    # column and dz <= 12, from the compiled-dimension build with 2 or 4 rows
    # per block (query rows counted in the first pass and taken out after it,
    # Theiler windows included); every form must give the oracle's radii and
    # counts bit for bit
    X, Y, Z = synth.random_points(n, dims, seed=n + w, kind="normal")
    monkeypatch.setenv("MTE_FORCE_MODE", "list")
    out = {}
    for kind, qb in (("0", "2"), ("1", "2"), ("1", "4")):
        monkeypatch.setenv("MTE_BUILD_KIND", kind)
        monkeypatch.setenv("MTE_BUILD_QB", qb)
        say("build form", kind, qb, dims, n, "window", w)
        out[(kind, qb)] = mte.cmi_ksg_diag(X, Y, Z, 4, 8, 3, 1, theiler=w)
    ref = out[("0", "2")]
    for key, o in out.items():
        for a, b in zip(ref, o):
            assert np.array_equal(a, b), key
    from test_gpu_parity import oracle_estimates
    rows = np.array([0, 1, n // 2, n - 2, n - 1])
    for e, (_, re, ra, rb, rc) in enumerate(oracle_estimates(X, Y, Z, 4, 8, 3, 1, queries=rows, theiler=w)):
        cmi, eps, cx, cy, cz = ref
        assert np.array_equal(eps[e, rows], re) and np.array_equal(cx[e, rows], ra)
        assert np.array_equal(cy[e, rows], rb) and np.array_equal(cz[e, rows], rc)


# One Z column and one Y column: the counts come from ranges of ranks of z
# (rows sorted by z, two binary searches per pair) instead of the Z list.
RANK_CASES = [
    # (n, dx, k, kind, S)
    (3, 1, 1, "normal", 7),
    (9, 1, 4, "grid", 9),
    (65, 2, 3, "dup", 9),
    (1000, 1, 4, "grid", 15),
    (3001, 3, 8, "normal", 9),
    (4097, 1, 4, "wide", 9),
    (2000, 1, 4, "tiny", 9),
    (1500, 1, 16, "dup", 9),
]


@pytest.mark.parametrize("n,dx,k,kind,S", RANK_CASES)
def test_rank_counts_parity(monkeypatch, n, dx, k, kind, S):
    # radii and counts bit for bit against the oracle, and the whole output
    # equal to that of the same launch counted on the Z list
    monkeypatch.setenv("MTE_FORCE_MODE", "list")
    X, Y, Z = synth.random_points(n, (dx, 1, 1), seed=n + 31 * k, kind=kind)
    say("rank counts", n, dx, k, kind, S)
    mte.mte_list_stats(reset=True)
    ranked = check_against_oracle(X, Y, Z, k, S)
    pairs, _ = mte.mte_list_stats(reset=True)
    assert pairs == n * (S + 1)
    monkeypatch.setenv("MTE_RANK_COUNTS", "0")
    say("  the same launch on the Z list")
    zlist = mte.cmi_ksg_diag(X, Y, Z, k, S, 11, 3)
    for a, b in zip(ranked, zlist):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("n,dx,kind", [(2000, 1, "split"), (200, 1, "mixed"), (3000, 2, "cells")])
def test_rank_counts_overflowing_differences(monkeypatch, n, dx, kind):
    # z differences that overflow to +inf fall outside every range (the range
    # test is strict on both sides, like the distance test)
    monkeypatch.setenv("MTE_FORCE_MODE", "list")
    X, Y, Z = _overflow_points(n, (dx, 1, 1), 60 + n, kind)
    say("rank counts, overflowing differences", n, dx, kind)
    check_against_oracle(X, Y, Z, 4, 8, seed=5, cand=1)


@pytest.mark.parametrize("n", [32768, 32769])
def test_rank_size_limit(monkeypatch, n):
    # sets of up to 32768 rows are ranked, larger ones keep the Z list; both
    # sides of the limit against the all-pairs kernel
    X, Y, Z = synth.random_points(n, (1, 1, 1), seed=n)
    out = {}
    for mode in ("brute", "list"):
        monkeypatch.setenv("MTE_FORCE_MODE", mode)
        say("rank size limit, N", n, "mode", mode)
        out[mode] = mte.cmi_ksg_diag(X, Y, Z, 4, 8, 5, 1)
    for a, b in zip(out["brute"], out["list"]):
        assert np.array_equal(a, b)
