"""Benchmark: KSG CMI evals/s at N = 10000, batched vs plain vs served.

Workload (one step): one transfer-entropy test at N = 10000 rows, D = 7
(X = a parent of the target at its true lag, Y = the target's present,
Z = the target's lags 1..5) on a 10-node linear VAR (synthetic, seeded):
the estimate and its 200 permutation surrogates in one batched launch on
device-resident inputs, the results copied back and the significance test run
on the host.  Reported beside it: the plain form (one call per estimate, 201
calls per step), the served form (requests of uneven N and conditioning
dimension through the request loop, Poisson arrivals, p50/p99 latency), the
main kernel's roofline figures and the CPU oracle on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line on stdout; progress goes to stderr.
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "KSG CMI evals/s at N=10k (batched/served vs plain); p50/p99 req latency"
N_ROWS, S, K_NN, SEED = 10000, 200, 4, 2
# MI355X FP32 vector peak 157.3 TFLOP/s counts an FMA as 2: 256 CUs x 128
# lanes per clock x 2.4 GHz = 78.6 T operations/s, the nominal ALU peak the
# rooflines are priced against.  Only some instruction forms issue at that
# rate (float add, subtract, fma; integer add, shift, and): min, max, med3,
# the three-operand forms and compares issue at 64 lanes per clock, 39.3 T
# (valu_issue_probe measures both).  The max-norm kernels' own peak is then
# set by their mix of the two kinds of operation (mix_peak).
PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
PEAK_HALF_TOPS = 256 * 64 * 2.4e9 / 1e12


def mix_peak(full, half):
    """Peak rate of a mix of `full` operations at the 128-lane rate and
    `half` at the 64-lane rate (each operation priced at the cheapest
    instruction that performs it)."""
    return (full + half) / (full / PEAK_TOPS + half / PEAK_HALF_TOPS)


def algorithmic_ops_split(n, dx, dy, dz, n_est):
    """algorithmic_ops split into subtracts and increments (128-lane rate)
    and maxima and compares (64-lane rate), per launch."""
    pairs = n * (n - 1)
    full = 2 * (dy + dz) + n_est * (2 * dx + 3)
    half = 2 * (dy + dz - 1) + n_est * (2 * dx + 4)
    return pairs * full, pairs * half


def build_ops_split(n, dy, dz):
    """build_ops split the same way: dy+dz subtracts, dy+dz-1 maxima."""
    return n * (n - 1) * (dy + dz), n * (n - 1) * (dy + dz - 1)
PEAK_HBM_GBS = 8000.0                  # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_ops(n, dx, dy, dz, n_est):
    """Method operations of one all-pairs test: per
    ordered pair (i != j), the Y,Z max-norm once per test for each pass
    (2*(dy+dz)-1 ops each: subtract, |.|-max), and per estimate 2*dx+1 ops in
    the k-NN pass (X subtract/max, compare with the current k-th) and 2*dx+6 in
    the count pass (X subtract/max, three compares, three increments)."""
    pairs = n * (n - 1)
    shared = 2 * (2 * (dy + dz) - 1)
    per_est = (2 * dx + 1) + (2 * dx + 6)
    return pairs * (shared + n_est * per_est)


def build_ops(n, dy, dz):
    """Neighbour-list build, per (Y,Z) sample: the Y,Z and Z max-norms of every
    ordered pair once (2*(dy+dz)-1 ops: subtract, |.|-max)."""
    return n * (n - 1) * (2 * (dy + dz) - 1)


def scan_bytes(dx, entries):
    """Neighbour-list scan, from the list entries it reads: an entry of a
    (Y,Z) list is 8 bytes (d_yz, row), of a Z list 12 bytes (d_z, d_yz, row),
    and each entry also reads the row's dx permuted X values (4 bytes each)."""
    knn, zl = entries
    return knn * (8 + 4 * dx) + zl * (12 + 4 * dx)


def counter_record(kernel):
    """The committed rocprofv3 counter record of `kernel` (profiles/traffic.json:
    HBM bytes per launch from FETCH_SIZE and WRITE_SIZE, each scaled by its
    factor for a plain copy of known size, and VALU instructions per launch),
    or None when it covers another kernel or the kernel sources have changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for f in rec.get("sources", []):
        try:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        except OSError:
            return None
    if rec.get("sha256") != h.hexdigest() or kernel not in rec.get("kernels", {}):
        return None
    return rec["kernels"][kernel]


def traffic_record():
    """The whole counter record, if it still covers the kernel sources."""
    return {"tuned_choice": json.load(open(os.path.join(ROOT, "profiles", "traffic.json"))).get("tuned_choice")} \
        if counter_record("scan") is not None else None


def measured_traffic(kernel):
    rec = counter_record(kernel)
    return rec["hbm_bytes_per_launch"] if rec else None


def valu_issue_frac(kernel, kernel_ms):
    """VALU lane slots the kernel's issued instructions occupy (64 per wave
    instruction, from the counter record) per second, against 78.6 T."""
    rec = counter_record(kernel)
    if not rec or "valu_insts_per_launch" not in rec:
        return None
    return rec["valu_insts_per_launch"] * 64 / (kernel_ms * 1e-3) / (PEAK_TOPS * 1e12)


TRAFFIC_SOURCES = ["paper_1902_06828_amd/csrc/lists.hip", "paper_1902_06828_amd/csrc/engine.h",
                   "paper_1902_06828_amd/csrc/ksg_device.h"]
C2_LIST_KEY = "L:n10000:dx1:dy1:dz5:k4:e201:w0:r1:one"


def write_traffic(fetch_dir, write_dir, sq_dir, pre_json):
    """profiles/traffic.json from the counter runs of the C2 leg: the
    rocprofv3 databases of a FETCH_SIZE pass and a WRITE_SIZE pass (both
    with --calibrate-copy) and of an SQ pass, and the benchmark's JSON line
    of the untimed run before them, whose tuning the passes read.  Per kernel
    the median over its dispatches; HBM bytes = FETCH_SIZE and WRITE_SIZE
    scaled by their readings for the 1 GiB copy."""
    import glob
    import hashlib
    import sqlite3
    import statistics

    def per_dispatch(d):
        dbs = sorted(glob.glob(os.path.join(d, "**", "*.db"), recursive=True), key=os.path.getmtime)
        if not dbs:
            raise SystemExit(f"no rocprofv3 database under {d}")
        out = {}
        cur = sqlite3.connect(dbs[-1]).cursor()
        for k, cn, v, di in cur.execute("select kernel_name, counter_name, value, dispatch_id "
                                        "from counters_collection"):
            out.setdefault(k, {}).setdefault(cn, {})
            out[k][cn][di] = out[k][cn].get(di, 0.0) + v
        return out

    def med(m, pick, cn):
        ks = [k for k in m if pick(k)]
        if len(ks) != 1:
            raise SystemExit(f"expected one kernel for {cn}, found {ks}")
        vals = list(m[ks[0]][cn].values())
        return statistics.median(vals), len(vals), ks[0]

    pf, pw, ps = per_dispatch(fetch_dir), per_dispatch(write_dir), per_dispatch(sq_dir)
    copy = lambda k: "neg" in k.lower()
    cf = med(pf, copy, "FETCH_SIZE")[0]
    cw = med(pw, copy, "WRITE_SIZE")[0]
    gib = 1 << 30
    cal = {"bytes_read": gib, "bytes_written": gib, "fetch_kib_raw": cf, "write_kib_raw": cw,
           "fetch_factor": gib / 1024 / cf, "write_factor": gib / 1024 / cw}
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    pre = json.loads([ln for ln in open(pre_json) if ln.startswith("{")][-1])
    choice = [c for c in pre.get("tuned_choices", {}).get("batched_and_plain", []) if c["key"] == C2_LIST_KEY]
    rec = {"workload": "C2, N=10000, 201 estimates", "sources": TRAFFIC_SOURCES, "sha256": h.hexdigest(),
           "copy_calibration": cal, "tuned_choice": choice[0] if choice else None, "kernels": {}}
    for tag, pick in (("scan", lambda k: "list_scan_kernel" in k), ("build", lambda k: "list_build" in k)):
        f, nf, kn = med(pf, pick, "FETCH_SIZE")
        w, nw, _ = med(pw, pick, "WRITE_SIZE")
        v, nv, _ = med(ps, pick, "SQ_INSTS_VALU")
        rec["kernels"][tag] = {
            "kernel": kn.replace("mte::(anonymous namespace)::", "").replace("void ", "").split("(")[0],
            "fetch_kib_raw": f, "write_kib_raw": w, "dispatches": [nf, nw, nv],
            "hbm_bytes_per_launch": (f * cal["fetch_factor"] + w * cal["write_factor"]) * 1024,
            "valu_insts_per_launch": v}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    json.dump(rec, open(path, "w"), indent=1)
    print(json.dumps(rec, indent=1))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(X, Y, Z, budget_s=15.0, single_s=6.0):
    """The C oracle (plain brute force, OpenMP over query rows) on the host:
    on all the threads OpenMP gives it over a bounded sample of the C2
    estimates, then on one thread over the first estimates."""
    from oracle import cksg, ksg, perm
    threads = cksg.max_threads()
    t = time.perf_counter()
    cksg.cmi_ksg(X, Y, Z, K_NN)
    one = time.perf_counter() - t
    count = int(max(1, min(S + 1, math.floor(budget_s / max(one, 1e-3)))))
    t = time.perf_counter()
    for e in range(count):
        Xe = X if e == 0 else ksg.permute_rows(X, perm.permutation(SEED, 0, e - 1, X.shape[1]))
        cksg.cmi_ksg(Xe, Y, Z, K_NN)
    dt = time.perf_counter() - t
    n1, t1 = 0, time.perf_counter()
    while n1 < S + 1 and (n1 == 0 or time.perf_counter() - t1 < single_s):
        Xe = X if n1 == 0 else ksg.permute_rows(X, perm.permutation(SEED, 0, n1 - 1, X.shape[1]))
        cksg.cmi_ksg(Xe, Y, Z, K_NN, threads=1)
        n1 += 1
    dt1 = time.perf_counter() - t1
    # C1 (one estimate at N = 1000, D = 3): the oracle's latency per call
    import synth
    X1, Y1, Z1, _ = synth.c1_gaussian(1000, 1)
    c1 = {}
    for name, th in (("c1_oracle_s", None), ("c1_oracle_single_thread_s", 1)):
        lat = []
        for _ in range(5):
            t = time.perf_counter()
            if th is None:
                cksg.cmi_ksg(X1, Y1, Z1, K_NN)
            else:
                cksg.cmi_ksg(X1, Y1, Z1, K_NN, threads=th)
            lat.append(time.perf_counter() - t)
        c1[name] = float(np.median(lat))
    return {"value": count / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{count} of the 201 C2 estimates (the estimate, then surrogates 0..{count - 2}), "
                      f"brute-force C oracle, OpenMP over query rows",
            "single_thread_evals_per_s": n1 / dt1, "single_thread_sample": f"the first {n1} C2 estimates",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), **c1}


def c1_leg(mte, torch, dev, reps=200):
    """C1: one KSG estimate of the Gaussian triple (N = 1000, 1-D X, Y, Z,
    partial correlation 0.6), latency per call: device-resident (its
    launch replayed as a graph, results left on the device, stream
    synchronised per call) and host arrays (copies in and out included)."""
    import synth
    X, Y, Z, true = synth.c1_gaussian(1000, 1)
    d = [torch.from_numpy(a).to(dev) for a in (X, Y, Z)]
    out = torch.zeros(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(5):
        mte.cmi_ksg_dev(d[0], d[1], d[2], K_NN, out)
    stream.synchronize()
    lat = []
    for _ in range(reps):
        t = time.perf_counter()
        mte.cmi_ksg_dev(d[0], d[1], d[2], K_NN, out)
        stream.synchronize()
        lat.append(time.perf_counter() - t)
    host = []
    for _ in range(reps // 4):
        t = time.perf_counter()
        v = mte.cmi_ksg(X, Y, Z, K_NN)
        host.append(time.perf_counter() - t)
    return {"workload": "C1: one estimate, Gaussian triple, N=1000, D=3, k=4",
            "estimate": v, "closed_form": true,
            "device_call_p50_s": float(np.percentile(lat, 50)), "device_call_p99_s": float(np.percentile(lat, 99)),
            "host_call_p50_s": float(np.percentile(host, 50))}


def c3_leg(mte):
    """C3: one target's whole greedy selection on the benchmark's 10-node VAR
    (N = 10000, lags 1..5, S = 200, alpha = 0.05, k = 4): the target with
    parents of lowest index, every other node a candidate; direct launches
    (mte_select_sources) and through the request loop (mte_select_sources_sid)."""
    import synth
    series, links = synth.var_network(10, N_ROWS, seed=SEED)
    target = min(i for (i, _, _, _) in links)
    cands = [j for j in range(10) if j != target]
    out = {"workload": "C3: greedy selection for one target, 10-node VAR, N=10000, S=200, lags 1..5",
           "target": target, "true_parents": sorted({(j, l) for (i, j, l, _) in links if i == target})}
    # an untimed first search: the autotuner's first calls for these shapes
    t = time.perf_counter()
    mte.mte_select_sources(series, target, cands, max_lag_sources=5, alpha=0.05, S=S, seed=SEED)
    out["first_search_s"] = time.perf_counter() - t
    t = time.perf_counter()
    res = mte.mte_select_sources(series, target, cands, max_lag_sources=5, alpha=0.05, S=S, seed=SEED)
    wall = time.perf_counter() - t
    out.update(direct_s=wall, estimates=res["n_estimates"], direct_evals_per_s=res["n_estimates"] / wall,
               sources=[(n, l) for (n, l, _, _) in res["sources"]])
    sid = mte.mte_series_register(series)
    t = time.perf_counter()
    res = mte.mte_select_sources_sid(sid, target, cands, max_lag_sources=5, alpha=0.05, S=S, seed=SEED)
    wall = time.perf_counter() - t
    mte.mte_series_release(sid)
    out.update(served_s=wall, served_evals_per_s=res["n_estimates"] / wall)
    return out


def c5_leg(mte, budget=2 << 30, window=2000, p_nodes=100):
    """C5: every target of a 100-node VAR (config generator, seed 5, N =
    10000, S = 200, lags 1..5, alpha = 0.05) searched at once through the
    request loop, each search in its own thread, under an HBM budget of 2 GiB:
    evals/s, latency percentiles and admission figures over the first
    `window` requests; then the series is cancelled and the searches end."""
    import threading
    import synth
    series, _ = synth.var_network(p_nodes, N_ROWS, seed=5)
    old = mte.mte_serve_get_stats()["budget_bytes"]
    mte.mte_init(0, budget)
    sid = mte.mte_series_register(series)
    errors, done = [], []

    def search(t):
        try:
            mte.mte_select_sources_sid(sid, t, [j for j in range(p_nodes) if j != t], max_lag_sources=5,
                                       alpha=0.05, S=S, seed=SEED + t)
            done.append(t)
        except mte.MteError as e:
            errors.append(e.code)

    mte.mte_serve_get_stats(reset=True)
    threads = [threading.Thread(target=search, args=(t,)) for t in range(p_nodes)]
    t0 = time.perf_counter()
    for th in threads:
        th.start()
    while True:
        st = mte.mte_serve_get_stats()
        if st["completed"] >= window or not any(th.is_alive() for th in threads):
            break
        time.sleep(0.005)
    wall = time.perf_counter() - t0
    st = mte.mte_serve_get_stats(reset=True)
    mte.mte_serve_cancel(sid)
    for th in threads:
        th.join()
    mte.mte_series_release(sid)
    mte.mte_init(0, old)
    return {"workload": f"C5: all {p_nodes} targets of a {p_nodes}-node VAR concurrently through the request loop, "
                        f"N=10000, S=200, HBM budget {budget >> 20} MiB, first {window} requests",
            "window_s": wall, "requests": st["completed"], "estimates": st["estimates"],
            "evals_per_s": st["estimates"] / wall, "p50_latency_s": st["p50_latency_s"],
            "p99_latency_s": st["p99_latency_s"], "batches": st["batches"],
            "mean_batch_requests": st["mean_batch_requests"], "peak_bytes_in_use": st["peak_bytes_in_use"],
            "budget_bytes": st["budget_bytes"], "admissions_that_waited": st["waited"],
            "latency_phases": latency_phases(st),
            "rejected": st["rejected"], "searches_cancelled": errors.count(mte._lib.MTE_ECANCELED),
            "searches_completed_in_window": len(done), "other_errors": [c for c in errors if c != mte._lib.MTE_ECANCELED]}


def latency_phases(st):
    """p50/p99 of each phase of the served latency and the phases averaged
    over the requests at or above the p99 latency (the request loop's
    statistics)."""
    keys = ["queue_p50_s", "queue_p99_s", "host_p50_s", "host_p99_s", "device_p50_s", "device_p99_s",
            "tail_queue_s", "tail_host_s", "tail_device_s", "tail_mean_n", "tail_mean_batch_requests",
            "tail_requests"]
    return {k: st[k] for k in keys}


def served(mte, torch, n_burst=768, n_poisson=384, loads=(0.5, 0.8, 0.95), load=0.8):
    """Requests of N in {1000, 3000, 10000}, Z dim 1..15, S = 200 over a
    100-node coupled-logistic-map network: a burst for saturation throughput
    (after an untimed burst of the same mix, whose rate is reported as the
    first burst's), then Poisson arrivals at each of `loads` x that rate for
    latency; the top-level latency figures are those at `load`."""
    import synth
    series, _ = synth.clm_network(100, N_ROWS, seed=4)
    sid = mte.mte_series_register(series)
    g = np.random.default_rng(4)

    def make(r):
        n = int(g.choice([1000, 3000, 10000]))
        dz = int(g.integers(1, 16))
        nodes = g.integers(0, 100, size=2 + dz).astype(np.int32)
        lags = np.concatenate([[int(g.integers(1, 6))], [0], g.integers(1, 6, size=dz)]).astype(np.int32)
        return dict(nodes=nodes, lags=lags, dx=1, dy=1, dz=dz, t0=5, n=n, k=K_NN, S=S, seed=9, cand=r)

    warm = [make(r) for r in range(6)]
    for q in warm:
        mte.mte_wait(mte.mte_submit(sid, **q), S)
    # a first burst of the same mix, untimed for the saturation figure: its
    # batches are larger than the warm-up's and take new device blocks, which
    # the allocator then keeps (its rate is reported as the cold one)
    reqs = [make(r) for r in range(n_burst)]
    mte.mte_serve_get_stats(reset=True)
    t = time.perf_counter()
    for tk in [mte.mte_submit(sid, **q) for q in reqs]:
        mte.mte_wait(tk, S)
    cold_s = time.perf_counter() - t
    cold_est = mte.mte_serve_get_stats(reset=True)["estimates"]
    t = time.perf_counter()
    tickets = [mte.mte_submit(sid, **q) for q in reqs]
    for tk in tickets:
        mte.mte_wait(tk, S)
    burst_s = time.perf_counter() - t
    st_burst = mte.mte_serve_get_stats(reset=True)
    rate = n_burst / burst_s

    def poisson(ld):
        reqs = [make(r) for r in range(n_poisson)]
        gaps = g.exponential(1.0 / (ld * rate), size=n_poisson)
        t = time.perf_counter()
        tickets = []
        next_t = t
        for q, gap in zip(reqs, gaps):
            next_t += gap
            while time.perf_counter() < next_t:
                time.sleep(min(0.0005, max(0.0, next_t - time.perf_counter())))
            tickets.append(mte.mte_submit(sid, **q))
        for tk in tickets:
            mte.mte_wait(tk, S)
        wall = time.perf_counter() - t
        st = mte.mte_serve_get_stats(reset=True)
        return {"offered_load": ld, "requests": n_poisson, "evals_per_s": st["estimates"] / wall,
                "p50_latency_s": st["p50_latency_s"], "p99_latency_s": st["p99_latency_s"],
                "batches": st["batches"], "mean_batch_requests": st["mean_batch_requests"],
                "latency_phases": latency_phases(st)}

    by_load = [poisson(ld) for ld in loads]
    mte.mte_series_release(sid)
    main = next(x for x in by_load if x["offered_load"] == load)
    return {
        "workload": "100-node CLM, requests of N in {1000,3000,10000}, Z dim 1..15, S=200",
        "saturation_evals_per_s": st_burst["estimates"] / burst_s,
        "first_burst_evals_per_s": cold_est / cold_s,
        "saturation_requests_per_s": rate,
        "burst_mean_batch_requests": st_burst["mean_batch_requests"],
        "offered_load": load,
        "poisson_requests": n_poisson,
        "poisson_evals_per_s": main["evals_per_s"],
        "p50_latency_s": main["p50_latency_s"],
        "p99_latency_s": main["p99_latency_s"],
        "batches": main["batches"],
        "mean_batch_requests": main["mean_batch_requests"],
        "latency_phases": main["latency_phases"],
        "poisson_by_load": by_load,
    }


def network_leg(mte, stages=False, clm=True):
    """Network inference on the benchmark's 10-node VAR (T = 10000): every
    target's greedy selection through the request loop (targets concurrent),
    S = 200, alpha = 0.05, FDR over omnibus p-values; wall time, estimates per
    second and the link statistics against the generating graph.  With
    `stages`, the kernels' HIP-event times per stage over the run (launches
    are then made directly, not from graphs; with MTE_SERVE_SLOTS=1 the
    batches run one at a time, so the stage times add up to the GPU time).
    With `clm`, also the paper's CLM network at its significance level."""
    import synth
    series, links = synth.var_network(10, N_ROWS, seed=SEED)
    stage_names = list(mte._lib.STAGES)
    if stages:
        mte.mte_kernel_timing(True)
        for st in stage_names:
            mte.mte_kernel_timing_stage(st, reset=True)
    mte.mte_serve_get_stats(reset=True)
    t = time.perf_counter()
    adj, summ = mte.mte_infer_network(series, max_lag_sources=5, alpha=0.05, alpha_fdr=0.05, S=S, seed=SEED)
    wall = time.perf_counter() - t
    sst = mte.mte_serve_get_stats(reset=True)
    stage_ms = {}
    if stages:
        for st in stage_names:
            n, ms = mte.mte_kernel_timing_stage(st, reset=True)
            if n:
                stage_ms[st] = {"launches": n, "ms": ms}
        mte.mte_kernel_timing(False)
    est = int(sum(s["n_estimates"] for s in summ))
    m = mte.mte_link_metrics(adj, synth.truth_adjacency(10, links))
    out = {"workload": "10-node VAR (config form), T=10000, all targets, S=200, alpha=0.05, BH-FDR 0.05",
           "wall_s": wall, "estimates": est, "evals_per_s": est / wall,
           "precision": m["precision"], "recall": m["recall"], "specificity": m["specificity"],
           "batches": sst["batches"], "mean_batch_requests": sst["mean_batch_requests"],
           "serve_slots": int(os.environ.get("MTE_SERVE_SLOTS") or 3)}
    if stages:
        out["stages_ms"] = stage_ms
    if not clm:
        return out
    # the paper's KSG workload: its coupled-logistic-map variant at its
    # significance level (S = 1001 > 1/alpha surrogates)
    cs, clinks = synth.paper_clm_network(10, N_ROWS, seed=1)
    t = time.perf_counter()
    cadj, csumm = mte.mte_infer_network(cs, max_lag_sources=5, alpha=0.001, alpha_fdr=0.001, S=1001, seed=1)
    cwall = time.perf_counter() - t
    cest = int(sum(s["n_estimates"] for s in csumm))
    cm = mte.mte_link_metrics(cadj, synth.truth_adjacency(10, clinks))
    clm = {"workload": "10-node CLM (paper's form), T=10000, all targets, S=1001, alpha=0.001, BH-FDR 0.001",
           "wall_s": cwall, "estimates": cest, "evals_per_s": cest / cwall, "links": int(len(clinks)),
           "precision": cm["precision"], "recall": cm["recall"], "specificity": cm["specificity"],
           "paper_accuracy": "precision, recall and specificity above 0.98 on average at T=10000"}
    out["clm"] = clm
    return out


PEAK_F64_TFLOPS = 78.6                 # MI355X fp64 (vector and matrix rates are equal)


def gauss_leg(mte, torch, dev):
    """The Gaussian estimator with its analytic null: network inference on the
    same 10-node VAR (T = 10000; one covariance matrix per target, then one
    Cholesky launch per greedy round), and the float64 Gram kernel timed with
    HIP events on its stream, at the network's shape (D = 51 variables: target,
    5 target lags, 9 sources x 5 lags; N = 9995) and at the largest covariance
    the library takes (D = 512, N = 10^6).  Gram flops: one fma (2 flops) per
    upper-triangle entry and row, D (D + 1) N."""
    import synth
    series, links = synth.var_network(10, N_ROWS, seed=SEED)
    mte.mte_infer_network(series, max_lag_sources=5, alpha=0.05, alpha_fdr=0.05, estimator="gauss")
    t = time.perf_counter()
    reps = 5
    for _ in range(reps):
        adj, summ = mte.mte_infer_network(series, max_lag_sources=5, alpha=0.05, alpha_fdr=0.05,
                                          estimator="gauss")
    wall = (time.perf_counter() - t) / reps
    est = int(sum(s["n_estimates"] for s in summ))
    m = mte.mte_link_metrics(adj, synth.truth_adjacency(10, links))
    out = {"workload": "10-node VAR, T=10000, all targets, Gaussian estimator, analytic null, alpha=0.05, "
                       "BH-FDR 0.05",
           "wall_s": wall, "estimates": est, "precision": m["precision"], "recall": m["recall"],
           "specificity": m["specificity"]}
    gram = []
    for D, n, reps in ((51, N_ROWS - 5, 20), (512, 1000000, 5)):
        g = torch.Generator(device=dev).manual_seed(SEED)
        V = torch.randn((D, n), generator=g, device=dev, dtype=torch.float32)
        cov = torch.empty((D, D), dtype=torch.float64, device=dev)
        mte.mte_gauss_covariance_dev(V, cov)
        mte.mte_kernel_timing_stage("gauss_gram", reset=True)
        mte.mte_kernel_timing(True)
        t = time.perf_counter()
        for _ in range(reps):
            mte.mte_gauss_covariance_dev(V, cov)
        call_ms = (time.perf_counter() - t) / reps * 1e3
        mte.mte_kernel_timing(False)
        launches, ms = mte.mte_kernel_timing_stage("gauss_gram", reset=True)
        k_ms = ms / max(1, launches)
        flops = float(D) * (D + 1) * n
        tf = flops / (k_ms * 1e-3) / 1e12
        gram.append({"D": D, "N": n, "kernel_ms": k_ms, "covariance_call_ms": call_ms, "tflops": tf,
                     "frac_fp64_peak": tf / PEAK_F64_TFLOPS, "hbm_bytes_read": 4 * D * n})
        del V, cov
    out["gram"] = gram
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-network", action="store_true")
    ap.add_argument("--no-gauss", action="store_true")
    ap.add_argument("--no-clm", action="store_true", help="network leg without the paper's CLM network")
    ap.add_argument("--network-stages", action="store_true",
                    help="per-stage kernel times over the network leg (direct launches)")
    ap.add_argument("--no-c1", action="store_true")
    ap.add_argument("--no-c3", action="store_true")
    ap.add_argument("--no-c5", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one elementwise copy of 1 GiB (256Mi float32 read + written) before the "
                         "timed region, as the reference for HBM byte counters")
    ap.add_argument("--write-traffic", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "SQ_DIR", "PRE_JSON"),
                    help="write profiles/traffic.json from the C2 counter runs' rocprofv3 databases and the "
                         "JSON line of the untimed run before them, then exit (no GPU needed)")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the KSG path runs on a single MI355X and no multi-GPU "
              "form is implemented; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1902_06828_amd as mte
    import synth

    dev = torch.device("cuda:0")
    X, Y, Z, meta = synth.c2_te_inputs(N_ROWS, seed=SEED)
    dX, dY, dZ = (torch.from_numpy(a).to(dev) for a in (X, Y, Z))
    E = S + 1
    out = torch.zeros(E, dtype=torch.float64, device=dev)
    host = torch.zeros(E, dtype=torch.float64).pin_memory()
    stream = torch.cuda.current_stream()

    def step():
        mte.cmi_ksg_surrogates_dev(dX, dY, dZ, K_NN, S, SEED, 0, out)
        host.copy_(out, non_blocking=True)
        stream.synchronize()
        v = host.numpy()
        return mte.mte_omnibus(float(v[0]), v[1:], 0.05)

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log("calibration copy: 1073741824 bytes read, 1073741824 bytes written (torch.neg)")
        del src, dst

    log("batched: warm-up (includes the tile autotuner)")
    for _ in range(args.warmup):
        step()
    stages = list(mte._lib.STAGES)
    mte.mte_kernel_timing(True)
    for st in stages:
        mte.mte_kernel_timing_stage(st, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        p, sig = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage_ms = {}
    for st in stages:
        launches, ms = mte.mte_kernel_timing_stage(st, reset=True)
        if launches:
            stage_ms[st] = {"launches_per_step": launches / args.steps, "ms_per_step": ms / args.steps,
                            "ms_per_launch": ms / launches}
    mte.mte_kernel_timing(False)
    dt = t1 - t0
    value = E * args.steps / dt
    # the list path's entry counts for this input (one checked call, same data)
    mte.mte_list_stats(reset=True)
    mte.mte_list_stats_enable(True)
    mte.cmi_ksg_surrogates(X, Y, Z, K_NN, S, SEED)
    mte.mte_list_stats_enable(False)
    pairs, undecided, entries = mte.mte_list_stats(reset=True, entries=True)
    def roofline_of(stage):
        k_ms = stage_ms[stage]["ms_per_launch"]
        if stage == "scan":
            # a gather kernel: HBM bytes from the counter record; the bytes
            # its lanes request (list entries and permuted X values as issued,
            # most served by L2) are reported beside them, not as the roof
            bound, unit, peak = "hbm", "GB/s", PEAK_HBM_GBS
            work = measured_traffic(stage)
            achieved = work / (k_ms * 1e-3) / 1e9 if work else None
            gather = scan_bytes(1, entries)
            extra = {"gather_bytes_per_launch": gather, "gather_gb_per_s": gather / (k_ms * 1e-3) / 1e9}
        else:
            bound, unit, peak = "alu", "TOP/s", PEAK_TOPS
            work = algorithmic_ops(N_ROWS, 1, 1, 5, E) if stage == "all_pairs" else (
                build_ops(N_ROWS, 1, 5) if stage == "build" else None)
            achieved = work / (k_ms * 1e-3) / 1e12 if work else None
            split = algorithmic_ops_split(N_ROWS, 1, 1, 5, E) if stage == "all_pairs" else (
                build_ops_split(N_ROWS, 1, 5) if stage == "build" else None)
            extra = {}
            if split and achieved:
                mp = mix_peak(*split)
                extra = {"mix_peak": mp, "frac_of_mix_peak": achieved / mp,
                         "mix_ops_128_lane_rate": split[0], "mix_ops_64_lane_rate": split[1]}
        return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak if achieved else None, "traffic": measured_traffic(stage),
                "kernel": stage, "kernel_ms": k_ms, "work_per_launch": work,
                "valu_issue_frac": valu_issue_frac(stage, k_ms), **extra, **choice_note(stage)}

    # the counter record holds the launch choices its run made; the tuner may
    # choose differently on another box (the scan's traffic depends on the
    # cooperative-finish threshold, the build's on its rows per block)
    this_choice = [c for c in mte.mte_tune_report() if c["key"] == C2_LIST_KEY]
    this_choice = this_choice[-1] if this_choice else None

    def choice_note(stage):
        rec = traffic_record()
        counted = rec.get("tuned_choice") if rec else None
        knobs = {"scan": ("coop_lanes", "scan_step", "grouped"), "build": ("build_rows",)}.get(stage)
        if not knobs:
            return {}
        same = (counted is not None and this_choice is not None and
                all(counted.get(k) == this_choice.get(k) for k in knobs))
        return {"tuned_choice": {k: this_choice.get(k) for k in knobs} if this_choice else None,
                "traffic_tuned_choice": {k: counted.get(k) for k in knobs} if counted else None,
                "traffic_choice_matches": same}

    # on the list path the permutation runs beside the build (a second stream),
    # so it is not on the step's critical path
    critical = [k for k in stage_ms if not (k == "permute" and "build" in stage_ms)]
    dominant = max(critical, key=lambda k: stage_ms[k]["ms_per_launch"] * stage_ms[k]["launches_per_step"])
    roof = roofline_of(dominant)
    # the list path's two big kernels take similar times at this size: both
    rooflines = {st: roofline_of(st) for st in ("scan", "build") if st in stage_ms}
    k_avg_ms, achieved, unit, peak = roof["kernel_ms"], roof["achieved"], roof["unit"], roof["peak"]
    equiv = algorithmic_ops(N_ROWS, 1, 1, 5, E) / (dt / args.steps) / 1e12
    log(f"batched: {value:.1f} evals/s, {dt / args.steps * 1e3:.3f} ms/step; stages (ms/step): " +
        ", ".join(f"{k} {v['ms_per_step']:.3f}" for k, v in stage_ms.items()))
    log(f"list path: {pairs} pairs, {undecided} redone over all rows, entries read {entries}")
    if achieved:
        log(f"dominant kernel: {dominant} {k_avg_ms:.3f} ms, {achieved:.2f} {unit} ({achieved / peak:.1%} of "
            f"{peak:.1f}); all-pairs-equivalent rate {equiv:.1f} TOP/s; TE p={p:.3f}")
    for st, rf in rooflines.items():
        if rf.get("mix_peak"):
            log(f"{st}: {rf['achieved']:.2f} TOP/s, {rf['frac']:.1%} of {rf['peak']:.1f} (nominal), "
                f"{rf['frac_of_mix_peak']:.1%} of {rf['mix_peak']:.1f} (its mix of 128- and 64-lane-rate operations)")
    if roof.get("mix_peak") and dominant not in rooflines:
        log(f"{dominant}: {roof['frac_of_mix_peak']:.1%} of its mix peak {roof['mix_peak']:.1f} TOP/s")

    # graph replay of the same step (timing off)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    graph_value = E * args.steps / (time.perf_counter() - t0)

    # plain form: one call per estimate (surrogate inputs permuted up front)
    plain = None
    if args.plain_steps > 0:
        perms = [np.arange(N_ROWS)] + [mte.mte_permutation(SEED, 0, s, N_ROWS).astype(np.int64) for s in range(S)]
        dXs = [torch.from_numpy(np.ascontiguousarray(X[:, pm])).to(dev) for pm in perms]
        outs = torch.zeros((E, 1), dtype=torch.float64, device=dev)

        def plain_step():
            for e in range(E):
                mte.cmi_ksg_dev(dXs[e], dY, dZ, K_NN, outs[e])
            host.copy_(outs.view(-1), non_blocking=True)
            stream.synchronize()
            v = host.numpy()
            return mte.mte_omnibus(float(v[0]), v[1:], 0.05)
        log("plain: warm-up")
        plain_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            plain_step()
        torch.cuda.synchronize()
        pt = time.perf_counter() - t0
        same = np.array_equal(outs.view(-1).cpu().numpy(), out.cpu().numpy())
        plain = {"evals_per_s": E * args.plain_steps / pt, "ms_per_step": pt / args.plain_steps * 1e3,
                 "identical_to_batched": bool(same)}
        log(f"plain: {plain['evals_per_s']:.1f} evals/s (identical results: {same})")

    # the autotuner's choices, by the leg whose calls made or read them
    seen_tuning = set()
    tuning = {}

    def note_tuning(leg):
        new = [r for r in mte.mte_tune_report() if (r["key"], r["from"]) not in seen_tuning]
        seen_tuning.update((r["key"], r["from"]) for r in new)
        tuning[leg] = new

    note_tuning("batched_and_plain")

    srv = None
    if not args.no_served:
        log("served: burst + Poisson arrivals")
        srv = served(mte, torch)
        log(f"served: {srv['saturation_evals_per_s']:.1f} evals/s saturated (first burst {srv['first_burst_evals_per_s']:.1f}); Poisson p50 "
            f"{srv['p50_latency_s'] * 1e3:.1f} ms p99 {srv['p99_latency_s'] * 1e3:.1f} ms")
        for pl in srv["poisson_by_load"]:
            ph = pl["latency_phases"]
            log(f"served at {pl['offered_load']:.2f}x saturation: {pl['evals_per_s']:.0f} evals/s, p50 "
                f"{pl['p50_latency_s'] * 1e3:.1f} ms p99 {pl['p99_latency_s'] * 1e3:.1f} ms; phases (ms): queued p50 "
                f"{ph['queue_p50_s'] * 1e3:.2f} p99 {ph['queue_p99_s'] * 1e3:.2f}, host p50 {ph['host_p50_s'] * 1e3:.2f} "
                f"p99 {ph['host_p99_s'] * 1e3:.2f}, device p50 {ph['device_p50_s'] * 1e3:.2f} p99 "
                f"{ph['device_p99_s'] * 1e3:.2f}; the {ph['tail_requests']} requests at or above p99: queued "
                f"{ph['tail_queue_s'] * 1e3:.2f}, host {ph['tail_host_s'] * 1e3:.2f}, device "
                f"{ph['tail_device_s'] * 1e3:.2f}, mean N {ph['tail_mean_n']:.0f}, batch "
                f"{ph['tail_mean_batch_requests']:.1f}")

    note_tuning("served")
    c3 = None
    if not args.no_c3:
        log("c3: one target's greedy selection")
        c3 = c3_leg(mte)
        log(f"c3: {c3['direct_s']:.3f} s direct ({c3['direct_evals_per_s']:.0f} evals/s), {c3['served_s']:.3f} s "
            f"served, {c3['estimates']} estimates, sources {c3['sources']} (true {c3['true_parents']})")

    note_tuning("c3")
    net = None
    if not args.no_network:
        log("network: all targets of the 10-node VAR")
        net = network_leg(mte, stages=args.network_stages, clm=not args.no_clm)
        log(f"network: {net['wall_s']:.2f} s, {net['evals_per_s']:.1f} evals/s, precision {net['precision']:.2f} "
            f"recall {net['recall']:.2f}")
        if "stages_ms" in net:
            tot = sum(v["ms"] for k, v in net["stages_ms"].items() if k != "permute")
            log("network: stage ms " + ", ".join(f"{k} {v['ms']:.1f}" for k, v in net["stages_ms"].items()) +
                f" (all but the permutation, which runs beside the build: {tot:.1f})")
        if "clm" in net:
            c = net["clm"]
            log(f"network: paper's CLM, {c['wall_s']:.2f} s, {c['evals_per_s']:.1f} evals/s, precision "
                f"{c['precision']:.3f} recall {c['recall']:.3f} specificity {c['specificity']:.3f}")

    note_tuning("network")
    gl = None
    if not args.no_gauss:
        log("gauss: network inference with the Gaussian estimator, Gram kernel")
        gl = gauss_leg(mte, torch, dev)
        log(f"gauss: network {gl['wall_s'] * 1e3:.1f} ms, precision {gl['precision']:.2f} recall "
            f"{gl['recall']:.2f}; gram " + ", ".join(f"D={g['D']} N={g['N']}: {g['kernel_ms']:.3f} ms "
                                                     f"{g['tflops']:.1f} TF/s" for g in gl["gram"]))

    note_tuning("gauss")
    c1 = None
    if not args.no_c1:
        log("c1: single-estimate latency, N = 1000")
        c1 = c1_leg(mte, torch, dev)
        log(f"c1: device call p50 {c1['device_call_p50_s'] * 1e3:.3f} ms, host call p50 "
            f"{c1['host_call_p50_s'] * 1e3:.3f} ms, estimate {c1['estimate']:.4f} (closed form "
            f"{c1['closed_form']:.4f})")

    note_tuning("c1")
    c5 = None
    if not args.no_c5:
        log("c5: 100 concurrent target searches under a 2 GiB budget")
        c5 = c5_leg(mte)
        log(f"c5: {c5['evals_per_s']:.0f} evals/s over {c5['requests']} requests, p50 "
            f"{c5['p50_latency_s'] * 1e3:.1f} ms p99 {c5['p99_latency_s'] * 1e3:.1f} ms, peak "
            f"{c5['peak_bytes_in_use'] >> 20} MiB, {c5['admissions_that_waited']} admissions waited")

    note_tuning("c5")
    cpu = None
    if not args.no_cpu:
        log("cpu baseline: C oracle on a bounded sample")
        cpu = cpu_baseline(X, Y, Z)
        log(f"cpu: {cpu['value']:.3f} evals/s on {cpu['cores']} threads, {cpu['single_thread_evals_per_s']:.3f} on "
            f"one ({cpu['cpu_model']})")

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "one TE test: estimate + 200 permutation surrogates, N=10000, X 1-D source lag, "
                        "Y 1-D target, Z 5-D target past (lags 1..5), 10-node linear VAR, k=4, "
                        "201 estimates in one batched launch, host significance test",
            "N": N_ROWS, "dims": [1, 1, 5], "k": K_NN, "estimates_per_step": E,
        },
        "roofline": roof,
        "rooflines": rooflines,
        "stages_ms_per_step": {k: v["ms_per_step"] for k, v in stage_ms.items()},
        "list_path": {"pairs": pairs, "redone_over_all_rows": undecided, "entries_read": entries},
        "all_pairs_equivalent_tops": equiv,
        "cpu_baseline": cpu,
        "graph_replay_evals_per_s": graph_value,
        "plain": plain,
        "served": srv,
        "network": net,
        "gauss": gl,
        "c1": c1,
        "c3": c3,
        "c5": c5,
        "tuned_choices": tuning,
        "tile_configs": [list(r) for r in mte.mte_tile_configs()],
        "tile_config_fields": ["kmax", "g", "qp", "dzm", "dym", "dxm"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
