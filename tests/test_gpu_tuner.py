"""The autotuner's launch choices change no result, and persist.

The list path's knobs (rows per block of the compiled-dimension build, the
scan's cooperative-finish threshold and entries per step, the permutation's
blocks per CU beside the build, the estimate-group lane order of one-job
launches) are forced through their environment overrides and every
combination must give the bits of the default.  The batched device call
tunes a shape once, writes the choice to the tuning file and, after a new
start, reads it back instead of tuning again."""

import sys

import numpy as np
import pytest
import torch

import paper_1902_06828_amd as mte
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("dims,n,S", [((1, 1, 5), 5000, 70), ((2, 1, 3), 3001, 130), ((1, 1, 1), 4000, 63)])
def test_list_knobs_change_no_result(monkeypatch, dims, n, S):
    X, Y, Z = synth.random_points(n, dims, seed=n + S)
    monkeypatch.setenv("MTE_FORCE_MODE", "list")
    monkeypatch.setenv("MTE_TUNE", "0")
    say("knobs: default", dims, n, S)
    ref = mte.cmi_ksg_diag(X, Y, Z, 4, S, 7, 1)
    for qb, coop, grouped, step, pcu in (("2", "2", "1", "4", "1"), ("4", "8", "0", "8", "3"),
                                         ("4", "4", "1", "4", "0"), ("2", "8", "0", "4", "2"),
                                         ("4", "2", "0", "8", "5")):
        monkeypatch.setenv("MTE_BUILD_QB", qb)
        monkeypatch.setenv("MTE_COOP_LANES", coop)
        monkeypatch.setenv("MTE_GROUPED", grouped)
        monkeypatch.setenv("MTE_SCAN_STEP", step)
        monkeypatch.setenv("MTE_PERMUTE_BLOCKS_PER_CU", pcu)
        say("knobs: build rows", qb, "coop lanes", coop, "grouped", grouped, "scan step", step,
            "permutation blocks per CU", pcu)
        out = mte.cmi_ksg_diag(X, Y, Z, 4, S, 7, 1)
        for a, b in zip(ref, out):
            assert np.array_equal(a, b)


def test_tuner_persists_its_choice(tmp_path, monkeypatch):
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("MTE_TUNE_FILE", str(path))
    monkeypatch.delenv("MTE_TUNE", raising=False)
    mte.mte_shutdown()                      # the next call starts anew and reads this file
    X, Y, Z, _ = synth.c2_te_inputs(10000, seed=2)
    dev = torch.device("cuda:0")
    dX, dY, dZ = (torch.from_numpy(a).to(dev) for a in (X, Y, Z))
    out = torch.zeros(201, dtype=torch.float64, device=dev)
    say("tuner: first call")
    mte.cmi_ksg_surrogates_dev(dX, dY, dZ, 4, 200, 2, 0, out)
    torch.cuda.synchronize()
    first = out.cpu().numpy().copy()
    rep = [r for r in mte.mte_tune_report() if r["key"].startswith("L:n10000:dx1:dy1:dz5")]
    say("report", rep)
    assert len(rep) == 1 and rep[0]["from"] == "tuned" and rep[0]["coop_lanes"] in (2, 4, 8)
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and " L:n10000:dx1:dy1:dz5:" in lines[0]
    mte.mte_shutdown()
    say("tuner: after a new start")
    out.zero_()
    mte.cmi_ksg_surrogates_dev(dX, dY, dZ, 4, 200, 2, 0, out)
    torch.cuda.synchronize()
    rep2 = [r for r in mte.mte_tune_report() if r["key"].startswith("L:n10000:dx1:dy1:dz5")]
    assert len(rep2) == 1 and rep2[0]["from"] == "file"
    assert {k: v for k, v in rep2[0].items() if k not in ("from",)} == {k: v for k, v in rep[0].items() if k != "from"}
    assert path.read_text().splitlines() == lines
    assert np.array_equal(out.cpu().numpy(), first)
    mte.mte_shutdown()


def test_greedy_rounds_tuned_or_not(tmp_path, monkeypatch):
    # greedy rounds of at least 2^20 pairs tune the list knobs on one job of
    # their shape; the selection is the same with tuning off
    monkeypatch.setenv("MTE_TUNE_FILE", str(tmp_path / "tune.txt"))
    mte.mte_shutdown()
    series, links = synth.var_network(10, 10000, seed=5)
    target = min(i for (i, _, _, _) in links)
    cands = [j for j in range(10) if j != target]
    kw = dict(max_lag_sources=5, alpha=0.05, S=200, seed=3)
    say("greedy, tuned")
    tuned = mte.mte_select_sources(series, target, cands, **kw)
    keys = [r["key"] for r in mte.mte_tune_report()]
    say("tuned keys", keys)
    assert any(k.startswith("L:n10000:") and k.endswith(":many") for k in keys)
    monkeypatch.setenv("MTE_TUNE", "0")
    say("greedy, untuned")
    plain = mte.mte_select_sources(series, target, cands, **kw)
    for key in ("target_past", "sources", "sources_before_omnibus", "omnibus_te", "omnibus_p", "n_estimates"):
        assert tuned[key] == plain[key]
    mte.mte_shutdown()


def test_tuning_file_skips_foreign_and_broken_lines(tmp_path, monkeypatch):
    # a choice written by the same library build on the same device is read back; lines of
    # another architecture or another build of the library, and lines that
    # do not parse, are skipped
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("MTE_TUNE_FILE", str(path))
    mte.mte_shutdown()
    X, Y, Z = synth.random_points(4000, (1, 1, 2), seed=3)
    dev = torch.device("cuda:0")
    dX, dY, dZ = (torch.from_numpy(a).to(dev) for a in (X, Y, Z))
    out = torch.zeros(301, dtype=torch.float64, device=dev)
    mte.cmi_ksg_surrogates_dev(dX, dY, dZ, 4, 300, 1, 0, out)
    torch.cuda.synchronize()
    good = path.read_text().splitlines()
    assert len(good) == 1
    f = good[0].split()            # mte-tune 3 <arch> <build> <key> <9 numbers>
    foreign = [" ".join(f[:2] + ["gfx000"] + f[3:4] + ["L:foreign-arch"] + f[5:]),
               " ".join(f[:3] + ["another-build"] + ["L:foreign-build"] + f[5:]),
               " ".join(f[:4] + ["L:short-line"] + f[5:8]),
               "mte-tune 9 " + " ".join(f[2:]),
               "not a tuning line", ""]
    path.write_text("\n".join(foreign + good) + "\n")
    mte.mte_shutdown()
    out.zero_()
    mte.cmi_ksg_surrogates_dev(dX, dY, dZ, 4, 300, 1, 0, out)
    torch.cuda.synchronize()
    rep = mte.mte_tune_report()
    say("report after restart", rep)
    assert [r["key"] for r in rep] == [f[4]] and rep[0]["from"] == "file"
    mte.mte_shutdown()


def test_several_job_lane_orders_agree(monkeypatch):
    # a greedy round's candidates are one launch of many jobs: with at least
    # four 64-estimate units per XCD the scan deals (job, group) units to the
    # XCDs, else it keeps job-major lanes; the selection and every statistic
    # are the same either way
    monkeypatch.setenv("MTE_TUNE", "0")
    series, links = synth.var_network(6, 3000, seed=11)
    target = min(i for (i, _, _, _) in links)
    cands = [j for j in range(6) if j != target]
    kw = dict(max_lag_sources=5, alpha=0.05, S=200, seed=4)
    say("greedy, XCD-dealt units")
    units = mte.mte_select_sources(series, target, cands, **kw)
    monkeypatch.setenv("MTE_GROUPED_MANY", "0")
    say("greedy, job-major lanes")
    plain = mte.mte_select_sources(series, target, cands, **kw)
    for key in ("target_past", "sources", "sources_before_omnibus", "omnibus_te", "omnibus_p", "n_estimates"):
        assert units[key] == plain[key]
