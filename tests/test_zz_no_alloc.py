"""The allocation-free entry point against the batched device-resident call.

cmi_ksg_surrogates_dev_noalloc keeps every scratch word in the library's
static device array.  Its results must equal cmi_ksg_surrogates_dev's bit for
bit (both are exact counts summed in one fixed order), on two calls in a row
with the second on a smaller input (the array keeps the first call's
contents), and the second call also against the oracle.  No device memory may
be taken by the calls, and an input whose scratch does not fit is refused
before anything is launched.

The reference calls run first in both path modes.  In the all-pairs mode the
autotuner launches every fitting tile variant on the same stream, so the
runtime's per-queue backing for the register spills of those variants (per-lane
private memory, not a buffer of the library) is in place before the memory
check, and the allocation-free call, which takes the tuned choice, runs the same
kernels.
"""

import sys

import numpy as np
import pytest

import paper_1902_06828_amd as mte
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(torch, a):
    return None if a is None else torch.from_numpy(a).cuda()


def test_noalloc_equals_batched_call(monkeypatch):
    import torch
    from oracle import cksg, ksg, perm
    mte.mte_init(0)
    cases = [(10000, (1, 1, 5), 200, 2, 0, "normal"),     # the benchmark's test shape
             (3000, (2, 1, 3), 30, 7, 5, "grid")]         # smaller, ties, two X columns
    inputs, refs = [], []
    for n, dims, S, seed, cand, kind in cases:
        X, Y, Z = synth.random_points(n, dims, seed=n + S, kind=kind)
        d = [_dev(torch, a) for a in (X, Y, Z)]
        res = []
        for mode in ("", "brute"):
            monkeypatch.setenv("MTE_FORCE_MODE", mode)
            ref = torch.zeros(S + 1, dtype=torch.float64, device="cuda")
            say("batched call", n, dims, S, "mode", mode or "default")
            mte.cmi_ksg_surrogates_dev(d[0], d[1], d[2], 4, S, seed, cand, ref)
            torch.cuda.synchronize()
            res.append(ref.cpu().numpy())
        assert np.array_equal(res[0], res[1])
        monkeypatch.delenv("MTE_FORCE_MODE")
        inputs.append((X, Y, Z, d, S, seed, cand))
        refs.append(res[0])
    outs = [torch.full((S + 1,), float("nan"), dtype=torch.float64, device="cuda") for (*_, S, _, _) in inputs]
    torch.cuda.synchronize()
    free_before = torch.cuda.mem_get_info()[0]
    got = []
    for (X, Y, Z, d, S, seed, cand), out in zip(inputs, outs):
        say("allocation-free call", X.shape[1], S)
        mte.cmi_ksg_surrogates_dev_noalloc(d[0], d[1], d[2], 4, S, seed, cand, out)
        torch.cuda.synchronize()
        got.append(out.cpu().numpy())
    free_after = torch.cuda.mem_get_info()[0]
    assert free_after == free_before, (free_before, free_after)
    for g, r in zip(got, refs):
        assert np.array_equal(g, r)
    # the second call against the oracle, every estimate
    X, Y, Z, _, S, seed, cand = inputs[1]
    for e in range(S + 1):
        Xe = X if e == 0 else ksg.permute_rows(X, perm.permutation(seed, cand, e - 1, X.shape[1]))
        assert abs(got[1][e] - cksg.cmi_ksg(Xe, Y, Z, 4)) <= TOL, e


def test_noalloc_refuses_what_does_not_fit():
    import torch
    mte.mte_init(0)
    n, S = 100000, 200                      # 80 MB of permuted X alone
    X, Y, Z = synth.random_points(n, (1, 1, 2), seed=3)
    d = [_dev(torch, a) for a in (X, Y, Z)]
    out = torch.full((S + 1,), -7.0, dtype=torch.float64, device="cuda")
    say("oversized allocation-free call")
    with pytest.raises(mte.MteError) as ei:
        mte.cmi_ksg_surrogates_dev_noalloc(d[0], d[1], d[2], 4, S, 1, 0, out)
    assert ei.value.code == mte._lib.MTE_EINVAL and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.all(out == -7.0)
