"""ctypes binding of libmte.so: argument marshalling only.

Every computation runs in the library (HIP kernels on the GPU, C++ on the
host).  The binding raises MteError for a non-zero status and refuses to load
anything else when the library is missing.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# MTE_LIBRARY selects another build of the same library (the host-code
# sanitizer build, libmte_san.so, whose runtime must be preloaded)
LIB_PATH = os.environ.get("MTE_LIBRARY") or os.path.join(HERE, "libmte.so")

MTE_OK, MTE_EINVAL, MTE_ENOMEM, MTE_EDEVICE, MTE_ETIMEOUT, MTE_EBUSY, MTE_ECANCELED = 0, -1, -2, -3, -4, -5, -6
_NAMES = {0: "MTE_OK", -1: "MTE_EINVAL", -2: "MTE_ENOMEM", -3: "MTE_EDEVICE", -4: "MTE_ETIMEOUT",
          -5: "MTE_EBUSY", -6: "MTE_ECANCELED"}


class MteError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class mte_opts(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("S", ctypes.c_int), ("max_lag_target", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("theiler", ctypes.c_int), ("estimator", ctypes.c_int),
                ("replications", ctypes.c_int), ("standardise", ctypes.c_int)]


class mte_var(ctypes.Structure):
    _fields_ = [("node", ctypes.c_int32), ("lag", ctypes.c_int32), ("cmi", ctypes.c_double),
                ("p", ctypes.c_double)]


class mte_result(ctypes.Structure):
    _fields_ = [("target_past", ctypes.POINTER(mte_var)), ("sources", ctypes.POINTER(mte_var)),
                ("n_target_past", ctypes.c_int), ("n_sources", ctypes.c_int),
                ("n_sources_tested", ctypes.c_int), ("omnibus_te", ctypes.c_double),
                ("omnibus_p", ctypes.c_double), ("significant", ctypes.c_int),
                ("n_estimates", ctypes.c_int64), ("gpu_seconds", ctypes.c_double)]


class mte_request(ctypes.Structure):
    _fields_ = [("sid", ctypes.c_int32), ("dx", ctypes.c_int), ("dy", ctypes.c_int), ("dz", ctypes.c_int),
                ("nodes", ctypes.POINTER(ctypes.c_int32)), ("lags", ctypes.POINTER(ctypes.c_int32)),
                ("t0", ctypes.c_int64), ("N", ctypes.c_int64), ("k", ctypes.c_int), ("S", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("cand", ctypes.c_uint32), ("theiler", ctypes.c_int)]


class mte_target_summary(ctypes.Structure):
    _fields_ = [("n_target_past", ctypes.c_int), ("n_sources", ctypes.c_int), ("n_sources_tested", ctypes.c_int),
                ("omnibus_te", ctypes.c_double), ("omnibus_p", ctypes.c_double), ("significant", ctypes.c_int),
                ("fdr_kept", ctypes.c_int), ("n_estimates", ctypes.c_int64)]


class mte_serve_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("estimates", ctypes.c_int64),
                ("p50_latency_s", ctypes.c_double), ("p99_latency_s", ctypes.c_double),
                ("mean_batch_requests", ctypes.c_double), ("peak_bytes_in_use", ctypes.c_int64),
                ("budget_bytes", ctypes.c_int64), ("waited", ctypes.c_int64),
                ("queue_p50_s", ctypes.c_double), ("queue_p99_s", ctypes.c_double),
                ("host_p50_s", ctypes.c_double), ("host_p99_s", ctypes.c_double),
                ("device_p50_s", ctypes.c_double), ("device_p99_s", ctypes.c_double),
                ("tail_queue_s", ctypes.c_double), ("tail_host_s", ctypes.c_double),
                ("tail_device_s", ctypes.c_double), ("tail_mean_n", ctypes.c_double),
                ("tail_mean_batch_requests", ctypes.c_double), ("tail_requests", ctypes.c_int64)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_U32 = ctypes.c_uint32
_U64 = ctypes.c_uint64
_D = ctypes.c_double
_SZ = ctypes.c_size_t

# name -> (argtypes); every entry point returns int status
SIGNATURES = {
    "mte_abi_version": [],
    "mte_init": [_I, _SZ],
    "mte_shutdown": [],
    "cmi_ksg": [_P, _I, _P, _I, _P, _I, _I64, _I, _P],
    "cmi_ksg_surrogates": [_P, _I, _P, _I, _P, _I, _I64, _I, _I, _U64, _P, _P],
    "cmi_ksg_diag": [_P, _I, _P, _I, _P, _I, _I64, _I, _I, _U64, _U32, _P, _P, _P, _P, _P],
    "cmi_ksg_diag_ex": [_P, _I, _P, _I, _P, _I, _I64, _I, _I, _I, _U64, _U32, _P, _P, _P, _P, _P],
    "cmi_ksg_dev": [_P, _I, _P, _I, _P, _I, _I64, _I64, _I, _P, _P],
    "cmi_ksg_surrogates_dev": [_P, _I, _P, _I, _P, _I, _I64, _I64, _I, _I, _U64, _U32, _P, _P],
    "cmi_ksg_surrogates_dev_ex": [_P, _I, _P, _I, _P, _I, _I64, _I64, _I, _I, _I, _U64, _U32, _P, _P],
    "cmi_ksg_surrogates_dev_noalloc": [_P, _I, _P, _I, _P, _I, _I64, _I64, _I, _I, _U64, _U32, _P, _P],
    "mte_autocorr_decay_time": [_P, _I64, _I, _P],
    "mte_fdr_bh": [_P, _I, ctypes.c_double, _P],
    "mte_link_metrics": [_P, _P, _I, _P, _P],
    "mte_infer_network": [_P, _I, _I64, _I, ctypes.c_double, ctypes.c_double, _P, _I, _P, _P],
    "mte_permutation": [_U64, _U32, _U32, _I64, _P],
    "mte_max_statistic": [_P, _P, _I, _I, _D, _P, _P, _P],
    "mte_min_statistic": [_P, _P, _I, _I, _D, _P, _P, _P],
    "mte_omnibus": [_D, _P, _I, _D, _P, _P],
    "mte_select_sources": [_P, _I, _I64, _I, _P, _I, _I, _D, _P, _P],
    "mte_select_sources_sid": [ctypes.c_int32, _I, _P, _I, _I, _D, _P, _P],
    "mte_series_register": [_P, _I, _I64, _P],
    "mte_series_release": [ctypes.c_int32],
    "mte_submit": [_P, _P],
    "mte_wait": [_U64, _P, _P, _D],
    "mte_serve_get_stats": [_P, _I],
    "mte_serve_cancel": [ctypes.c_int32],
    "mte_tile_configs": [_P, _I, _P],
    "mte_tune_report": [_P, _SZ, _P],
    "mte_kernel_timing": [_I],
    "mte_kernel_timing_read": [_P, _P, _I],
    "mte_kernel_timing_stage": [_I, _P, _P, _I],
    "mte_list_stats": [_P, _P, _P, _I],
    "mte_list_stats_enable": [_I],
    "cmi_gauss": [_P, _I, _P, _I, _P, _I, _I64, _P, _P],
    "mte_gauss_covariance_dev": [_P, _I, _I64, _I64, _P, _P],
    "mte_gauss_cmi_sets": [_P, _I, _I, _P, _P, _P, _P],
    "mte_chi2_sf": [_D, _I, _P],
    "mte_shuffle_mode": [_I, _I, _P],
    "mte_standardise": [_P, _I, _I, _I64, _P],
    "mte_permutation_rep": [_U64, _U32, _U32, _I64, _I, _I, _P],
    "cmi_ksg_surrogates_rep": [_P, _I, _P, _I, _P, _I, _I64, _I, _I, _I, _U64, _U32, _I, _P, _P],
}

SHUFFLE = {"auto": -1, "within": 0, "replications": 1}

ESTIMATORS = {"ksg": 0, "gauss": 1}

_lib = None


def lib():
    """The loaded libmte.so (built by paper_1902_06828_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_1902_06828_amd.build.build() first")
        # One HIP runtime per process: load PyTorch's first, so that
        # libmte's libamdhip64.so.7 dependency binds to the copy PyTorch
        # already mapped (it owns the device buffers and streams we receive).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        L.mte_last_error.restype = ctypes.c_char_p
        L.mte_last_error.argtypes = []
        for name, args in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = ctypes.c_int
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != MTE_OK:
        raise MteError(rc, lib().mte_last_error().decode())


def _f32(a, name):
    if a is None:
        return None, 0, None
    a = np.asarray(a)
    if a.dtype != np.float32:
        raise TypeError(f"{name} must be float32")
    if a.ndim == 1:
        a = a[None, :]
    a = np.ascontiguousarray(a)
    return a, a.shape[0], a.shape[1]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _xyz(X, Y, Z):
    X, dx, n = _f32(X, "X")
    Y, dy, ny = _f32(Y, "Y")
    Z, dz, nz = _f32(Z, "Z")
    if ny != n or (Z is not None and nz != n):
        raise ValueError("X, Y and Z must have the same number of rows")
    return X, dx, Y, dy, Z, dz, n


# ---------------------------------------------------------------- estimator
def mte_init(device: int = 0, hbm_budget_bytes: int = 0) -> None:
    _check(lib().mte_init(device, hbm_budget_bytes))


def mte_shutdown() -> None:
    _check(lib().mte_shutdown())


def cmi_ksg(X, Y, Z=None, k: int = 4) -> float:
    X, dx, Y, dy, Z, dz, n = _xyz(X, Y, Z)
    out = ctypes.c_double()
    _check(lib().cmi_ksg(_ptr(X), dx, _ptr(Y), dy, _ptr(Z), dz, n, k, ctypes.byref(out)))
    return out.value


def cmi_ksg_surrogates(X, Y, Z=None, k: int = 4, S: int = 200, seed: int = 0):
    """Returns (estimate, surrogates[S])."""
    X, dx, Y, dy, Z, dz, n = _xyz(X, Y, Z)
    out = ctypes.c_double()
    surr = np.empty(S, np.float64)
    _check(lib().cmi_ksg_surrogates(_ptr(X), dx, _ptr(Y), dy, _ptr(Z), dz, n, k, S, seed,
                                    ctypes.byref(out), _ptr(surr)))
    return out.value, surr


def cmi_ksg_diag(X, Y, Z=None, k: int = 4, S: int = 0, seed: int = 0, cand: int = 0, theiler: int = 0):
    """Returns (cmi[1+S], eps[1+S][N], n_xz, n_yz, n_z) (counts int32 [1+S][N])."""
    X, dx, Y, dy, Z, dz, n = _xyz(X, Y, Z)
    E = S + 1
    cmi = np.empty(E, np.float64)
    eps = np.empty((E, n), np.float32)
    cx, cy, cz = (np.empty((E, n), np.int32) for _ in range(3))
    if theiler:
        _check(lib().cmi_ksg_diag_ex(_ptr(X), dx, _ptr(Y), dy, _ptr(Z), dz, n, k, theiler, S, seed, cand,
                                     _ptr(cmi), _ptr(eps), _ptr(cx), _ptr(cy), _ptr(cz)))
    else:
        _check(lib().cmi_ksg_diag(_ptr(X), dx, _ptr(Y), dy, _ptr(Z), dz, n, k, S, seed, cand, _ptr(cmi),
                                  _ptr(eps), _ptr(cx), _ptr(cy), _ptr(cz)))
    return cmi, eps, cx, cy, cz


def mte_autocorr_decay_time(x, max_lag: int) -> int:
    """Autocorrelation decay time of a float32 series (Theiler window heuristic)."""
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1)
    out = ctypes.c_int()
    _check(lib().mte_autocorr_decay_time(_ptr(x), len(x), max_lag, ctypes.byref(out)))
    return out.value


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(int(stream))


def cmi_ksg_dev(X, Y, Z, k: int, out, stream=None) -> None:
    """Device-resident estimate: X, Y, Z are float32 CUDA tensors [d][ld]
    (Z may be None), out a float64 CUDA tensor with >= 1 entry."""
    cmi_ksg_surrogates_dev(X, Y, Z, k, 0, 0, 0, out, stream)


def _dev_shape(X, Y, Z, S, out, n):
    """Checks the device-resident arguments; returns (rows, ld)."""
    import torch

    def chk(t, name):
        if t.dtype != torch.float32 or not t.is_cuda or t.dim() != 2 or t.stride(1) != 1:
            raise TypeError(f"{name} must be a float32 CUDA tensor [d][ld] with unit row stride")
    chk(X, "X")
    chk(Y, "Y")
    if Z is not None:
        chk(Z, "Z")
    if out.dtype != torch.float64 or not out.is_cuda or out.numel() < S + 1:
        raise TypeError("out must be a float64 CUDA tensor with S+1 entries")
    rows = X.shape[1] if n is None else n
    # the column stride of a one-column tensor is never used
    multi = [t.stride(0) for t in (X, Y, Z) if t is not None and t.shape[0] > 1]
    ld = multi[0] if multi else max(t.shape[1] for t in (X, Y, Z) if t is not None)
    if any(s != ld for s in multi):
        raise ValueError("X, Y and Z must share the leading dimension")
    if any(t is not None and t.shape[1] < rows for t in (X, Y, Z)) or rows > ld:
        raise ValueError("fewer columns than rows requested")
    return rows, ld


def _dev_cols(X, Y, Z):
    return (ctypes.c_void_p(X.data_ptr()), X.shape[0], ctypes.c_void_p(Y.data_ptr()), Y.shape[0],
            None if Z is None else ctypes.c_void_p(Z.data_ptr()), 0 if Z is None else Z.shape[0])


def cmi_ksg_surrogates_dev(X, Y, Z, k: int, S: int, seed: int, cand: int, out, stream=None,
                           n: int | None = None, theiler: int = 0) -> None:
    """Device-resident estimate and S surrogates into out[0..S] (float64 CUDA
    tensor), asynchronous on `stream` (torch's current stream by default)."""
    rows, ld = _dev_shape(X, Y, Z, S, out, n)
    _check(lib().cmi_ksg_surrogates_dev_ex(*_dev_cols(X, Y, Z), rows, ld, k, theiler, S, seed, cand,
                                           ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))


def cmi_ksg_surrogates_dev_noalloc(X, Y, Z, k: int, S: int, seed: int, cand: int, out, stream=None,
                                   n: int | None = None) -> None:
    """cmi_ksg_surrogates_dev with every scratch word in the library's static
    device array (no allocation); needs mte_init first."""
    rows, ld = _dev_shape(X, Y, Z, S, out, n)
    _check(lib().cmi_ksg_surrogates_dev_noalloc(*_dev_cols(X, Y, Z), rows, ld, k, S, seed, cand,
                                                ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))


def mte_permutation(seed: int, cand: int, s: int, n: int) -> np.ndarray:
    out = np.empty(n, np.uint32)
    _check(lib().mte_permutation(seed, cand, s, n, _ptr(out)))
    return out


# ---------------------------------------------------------------- tests
def _stat(fn, real, surr, alpha):
    real = np.ascontiguousarray(real, dtype=np.float64)
    surr = np.ascontiguousarray(surr, dtype=np.float64).reshape(len(real), -1)
    idx, p, sig = ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
    _check(fn(_ptr(real), _ptr(surr), len(real), surr.shape[1], alpha, ctypes.byref(idx),
              ctypes.byref(p), ctypes.byref(sig)))
    return idx.value, p.value, bool(sig.value)


def mte_max_statistic(real, surr, alpha):
    return _stat(lib().mte_max_statistic, real, surr, alpha)


def mte_min_statistic(real, surr, alpha):
    return _stat(lib().mte_min_statistic, real, surr, alpha)


def mte_omnibus(real: float, surr, alpha):
    surr = np.ascontiguousarray(surr, dtype=np.float64).ravel()
    p, sig = ctypes.c_double(), ctypes.c_int()
    _check(lib().mte_omnibus(real, _ptr(surr), len(surr), alpha, ctypes.byref(p), ctypes.byref(sig)))
    return p.value, bool(sig.value)


# ---------------------------------------------------------------- greedy
def _result_dict(res, tp, src):
    var = lambda v: (v.node, v.lag, v.cmi, v.p)
    return {
        "target_past": [var(tp[i]) for i in range(res.n_target_past)],
        "sources": [var(src[i]) for i in range(res.n_sources)],
        "sources_before_omnibus": [var(src[i]) for i in range(res.n_sources_tested)],
        "omnibus_te": res.omnibus_te,
        "omnibus_p": res.omnibus_p,
        "significant": bool(res.significant),
        "n_estimates": res.n_estimates,
        "gpu_seconds": res.gpu_seconds,
    }


def _opts(k, S, max_lag_target, seed, theiler=0, estimator="ksg", replications=1, standardise=True):
    if estimator not in ESTIMATORS:
        raise ValueError(f"estimator must be one of {sorted(ESTIMATORS)}")
    return mte_opts(k=k, S=S, max_lag_target=max_lag_target, seed=seed, theiler=theiler,
                    estimator=ESTIMATORS[estimator], replications=replications, standardise=int(bool(standardise)))


def _series(data):
    """float32 [P][T] (one replication) or [R][P][T] -> (array, R, P, T)."""
    data = np.ascontiguousarray(data)
    if data.dtype != np.float32 or data.ndim not in (2, 3):
        raise TypeError("data must be float32 [P][T] or [R][P][T]")
    if data.ndim == 2:
        return data, 1, data.shape[0], data.shape[1]
    return data, data.shape[0], data.shape[1], data.shape[2]


def mte_select_sources(data, target: int, candidates, max_lag_sources: int = 5, alpha: float = 0.05,
                       k: int = 4, S: int = 200, max_lag_target: int = 5, seed: int = 0, theiler: int = 0,
                       estimator: str = "ksg", standardise: bool = True):
    """data: float32 [P][T], or [R][P][T] for R replications."""
    data, R, P, T = _series(data)
    cands = np.ascontiguousarray(candidates, dtype=np.int32)
    tp = (mte_var * max(1, max_lag_target))()
    src = (mte_var * max(1, len(cands) * max_lag_sources))()
    res = mte_result(target_past=tp, sources=src)
    o = _opts(k, S, max_lag_target, seed, theiler, estimator, R, standardise)
    _check(lib().mte_select_sources(_ptr(data), P, T, target, _ptr(cands),
                                    len(cands), max_lag_sources, alpha, ctypes.byref(o),
                                    ctypes.byref(res)))
    return _result_dict(res, tp, src)


def mte_select_sources_sid(sid: int, target: int, candidates, max_lag_sources: int = 5,
                           alpha: float = 0.05, k: int = 4, S: int = 200, max_lag_target: int = 5,
                           seed: int = 0, theiler: int = 0, estimator: str = "ksg", standardise: bool = True):
    cands = np.ascontiguousarray(candidates, dtype=np.int32)
    tp = (mte_var * max(1, max_lag_target))()
    src = (mte_var * max(1, len(cands) * max_lag_sources))()
    res = mte_result(target_past=tp, sources=src)
    o = _opts(k, S, max_lag_target, seed, theiler, estimator, 1, standardise)
    _check(lib().mte_select_sources_sid(sid, target, _ptr(cands), len(cands), max_lag_sources, alpha,
                                        ctypes.byref(o), ctypes.byref(res)))
    return _result_dict(res, tp, src)


# ---------------------------------------------------------------- serving
def mte_series_register(data) -> int:
    data = np.ascontiguousarray(data)
    if data.dtype != np.float32 or data.ndim != 2:
        raise TypeError("data must be float32 [P][T]")
    sid = ctypes.c_int32()
    _check(lib().mte_series_register(_ptr(data), data.shape[0], data.shape[1], ctypes.byref(sid)))
    return sid.value


def mte_series_release(sid: int) -> None:
    _check(lib().mte_series_release(sid))


def mte_submit(sid: int, nodes, lags, dx: int, dy: int, dz: int, t0: int, n: int, k: int = 4,
               S: int = 0, seed: int = 0, cand: int = 0, theiler: int = 0) -> int:
    nodes = np.ascontiguousarray(nodes, dtype=np.int32)
    lags = np.ascontiguousarray(lags, dtype=np.int32)
    if len(nodes) != dx + dy + dz or len(lags) != len(nodes):
        raise ValueError("need dx+dy+dz nodes and lags")
    req = mte_request(sid=sid, dx=dx, dy=dy, dz=dz,
                      nodes=nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                      lags=lags.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                      t0=t0, N=n, k=k, S=S, seed=seed, cand=cand, theiler=theiler)
    ticket = ctypes.c_uint64()
    _check(lib().mte_submit(ctypes.byref(req), ctypes.byref(ticket)))
    return ticket.value


def mte_wait(ticket: int, S: int = 0, timeout_s: float = -1.0):
    """Returns (estimate, surrogates[S])."""
    out = ctypes.c_double()
    surr = np.empty(max(S, 0), np.float64)
    _check(lib().mte_wait(ticket, ctypes.byref(out), _ptr(surr) if S > 0 else None, timeout_s))
    return out.value, surr


def mte_serve_cancel(sid: int) -> None:
    """Cancel a series: its queued requests and any search on it end with
    MTE_ECANCELED; batches on the GPU complete."""
    _check(lib().mte_serve_cancel(sid))


def mte_serve_get_stats(reset: bool = False) -> dict:
    st = mte_serve_stats()
    _check(lib().mte_serve_get_stats(ctypes.byref(st), int(reset)))
    return {name: getattr(st, name) for name, _ in mte_serve_stats._fields_}


def mte_tile_configs():
    """Rows (kmax, g, qp, dzm, dym, dxm) of the compiled tile configurations."""
    n = ctypes.c_int()
    _check(lib().mte_tile_configs(None, 0, ctypes.byref(n)))
    buf = np.empty((n.value, 6), np.int32)
    _check(lib().mte_tile_configs(_ptr(buf), n.value, ctypes.byref(n)))
    return [tuple(int(v) for v in row) for row in buf]


def mte_tune_report():
    """The autotuner's choices made or read from the tuning file in this
    process: a list of dicts (key, variant, split, build_rows, coop_lanes,
    grouped, scan_step, perm_cu, ms, from)."""
    n = ctypes.c_size_t()
    _check(lib().mte_tune_report(None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(lib().mte_tune_report(buf, n.value + 1, ctypes.byref(n)))
    out = []
    for line in buf.value.decode().splitlines():
        key, *fields = line.split()
        rec = {"key": key}
        for f in fields:
            name, val = f.split("=", 1)
            rec[name] = val if name == "from" else (float(val) if name == "ms" else int(val))
        out.append(rec)
    return out


# ---------------------------------------------------------------- timing
def mte_kernel_timing(enable: bool) -> None:
    _check(lib().mte_kernel_timing(int(enable)))


def mte_kernel_timing_read(reset: bool = False):
    """Returns (launches, total milliseconds) of the all-pairs KSG kernel."""
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check(lib().mte_kernel_timing_read(ctypes.byref(n), ctypes.byref(ms), int(reset)))
    return n.value, ms.value


STAGES = {"all_pairs": 0, "build": 1, "scan": 2, "fallback": 3, "reduce": 4, "permute": 5, "gauss_gram": 6,
          "gauss_cmi": 7}


def mte_kernel_timing_stage(stage, reset: bool = False):
    """Returns (launches, total milliseconds) of one timed stage (name or number)."""
    st = STAGES[stage] if isinstance(stage, str) else int(stage)
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check(lib().mte_kernel_timing_stage(st, ctypes.byref(n), ctypes.byref(ms), int(reset)))
    return n.value, ms.value


def mte_list_stats_enable(enable: bool) -> None:
    _check(lib().mte_list_stats_enable(int(enable)))


def mte_list_stats(reset: bool = False, entries: bool = False):
    """Returns (pairs on the list path, pairs redone over all rows), plus the
    list entries read by the three scans when `entries` is set."""
    a, b = ctypes.c_int64(), ctypes.c_int64()
    ent = np.zeros(2, np.int64)
    _check(lib().mte_list_stats(ctypes.byref(a), ctypes.byref(b), _ptr(ent), int(reset)))
    if entries:
        return a.value, b.value, [int(v) for v in ent]
    return a.value, b.value


# ---------------------------------------------------------------- network level
def mte_fdr_bh(pvals, q: float):
    """Benjamini-Hochberg keep mask (bool array) at level q."""
    p = np.ascontiguousarray(pvals, dtype=np.float64)
    keep = np.zeros(len(p), np.uint8)
    _check(lib().mte_fdr_bh(_ptr(p), len(p), q, _ptr(keep)))
    return keep.astype(bool)


def mte_link_metrics(inferred, truth):
    a = np.ascontiguousarray(inferred, dtype=np.uint8)
    b = np.ascontiguousarray(truth, dtype=np.uint8)
    counts = np.zeros(4, np.int64)
    rates = np.zeros(4, np.float64)
    _check(lib().mte_link_metrics(_ptr(a), _ptr(b), a.shape[0], _ptr(counts), _ptr(rates)))
    return {"tp": int(counts[0]), "fp": int(counts[1]), "tn": int(counts[2]), "fn": int(counts[3]),
            "precision": float(rates[0]), "recall": float(rates[1]), "specificity": float(rates[2]),
            "fpr": float(rates[3])}


def mte_infer_network(data, max_lag_sources: int = 5, alpha: float = 0.05, alpha_fdr: float = 0.05,
                      k: int = 4, S: int = 200, max_lag_target: int = 5, seed: int = 0, theiler: int = 0,
                      n_threads: int = 0, estimator: str = "ksg", standardise: bool = True):
    """data: float32 [P][T], or [R][P][T] for R replications.  Returns
    (adjacency uint8 [P][P], per-target summaries as dicts)."""
    data, R, P, T = _series(data)
    adj = np.zeros((P, P), np.uint8)
    tgt = (mte_target_summary * P)()
    o = _opts(k, S, max_lag_target, seed, theiler, estimator, R, standardise)
    _check(lib().mte_infer_network(_ptr(data), P, T, max_lag_sources, alpha,
                                   alpha_fdr if alpha_fdr else 0.0, ctypes.byref(o), n_threads, _ptr(adj), tgt))
    summ = [{name: getattr(tgt[t], name) for name, _ in mte_target_summary._fields_} for t in range(P)]
    return adj, summ


# ---------------------------------------------------------------- Gaussian estimator
def cmi_gauss(X, Y, Z=None):
    """Gaussian I(X;Y|Z) in nats and its analytic p-value sf_{dx*dy}(2 N I)."""
    X, dx, Y, dy, Z, dz, n = _xyz(X, Y, Z)
    out, p = ctypes.c_double(), ctypes.c_double()
    _check(lib().cmi_gauss(_ptr(X), dx, _ptr(Y), dy, _ptr(Z), dz, n, ctypes.byref(out), ctypes.byref(p)))
    return out.value, p.value


def mte_gauss_covariance_dev(V, cov, n: int | None = None, stream=None) -> None:
    """Covariance of the rows of a device float32 tensor V [D][ld] (first n
    columns of each row) into the device float64 tensor cov [D][D]."""
    if V.dtype != _torch().float32 or V.dim() != 2 or V.stride(1) != 1:
        raise TypeError("V must be a float32 [D][ld] tensor with unit column stride")
    D = V.shape[0]
    if cov.dtype != _torch().float64 or tuple(cov.shape) != (D, D) or not cov.is_contiguous():
        raise TypeError("cov must be a contiguous float64 [D][D] tensor")
    rows = V.shape[1] if n is None else n
    _check(lib().mte_gauss_covariance_dev(ctypes.c_void_p(V.data_ptr()), D, rows, V.stride(0),
                                          ctypes.c_void_p(cov.data_ptr()), _stream_ptr(stream)))


def mte_gauss_cmi_sets(cov, sets, stream=None):
    """I for each (X, Y, Z) index-list triple against a device covariance."""
    if cov.dtype != _torch().float64 or cov.dim() != 2 or not cov.is_contiguous():
        raise TypeError("cov must be a contiguous float64 [D][D] tensor")
    dims, idx = [], []
    for x, y, z in sets:
        dims += [len(x), len(y), len(z)]
        idx += list(x) + list(y) + list(z)
    dims = np.ascontiguousarray(dims, dtype=np.int32)
    idx = np.ascontiguousarray(idx if idx else [0], dtype=np.int32)
    out = np.zeros(max(1, len(sets)), np.float64)
    _check(lib().mte_gauss_cmi_sets(ctypes.c_void_p(cov.data_ptr()), cov.shape[0], len(sets), _ptr(dims),
                                    _ptr(idx), _ptr(out), _stream_ptr(stream)))
    return out[:len(sets)]


def mte_chi2_sf(x: float, dof: int) -> float:
    out = ctypes.c_double()
    _check(lib().mte_chi2_sf(float(x), dof, ctypes.byref(out)))
    return out.value


# ---------------------------------------------------------------- replications
def mte_shuffle_mode(R: int, S: int) -> str:
    out = ctypes.c_int()
    _check(lib().mte_shuffle_mode(R, S, ctypes.byref(out)))
    return {v: k for k, v in SHUFFLE.items()}[out.value]


def mte_permutation_rep(seed: int, cand: int, s: int, n: int, R: int, mode: str):
    """Source row of every row of surrogate s over R replications (host)."""
    out = np.empty(n, np.uint32)
    _check(lib().mte_permutation_rep(seed, cand, s, n, R, SHUFFLE[mode], _ptr(out)))
    return out


def cmi_ksg_surrogates_rep(X, Y, Z=None, k: int = 4, S: int = 20, R: int = 1, seed: int = 0, cand: int = 0,
                           mode: str = "auto"):
    """Estimate and S surrogates over R replications of N/R rows each."""
    X, dx, Y, dy, Z, dz, n = _xyz(X, Y, Z)
    out, surr = ctypes.c_double(), np.zeros(S, np.float64)
    _check(lib().cmi_ksg_surrogates_rep(_ptr(X), dx, _ptr(Y), dy, _ptr(Z), dz, n, R, k, S, seed, cand,
                                        SHUFFLE[mode], ctypes.byref(out), _ptr(surr)))
    return out.value, surr


def mte_standardise(data):
    """Per-node z-score of float32 [P][T] or [R][P][T] data (the greedy search's
    normalisation)."""
    data, R, P, T = _series(data)
    out = np.empty_like(data)
    _check(lib().mte_standardise(_ptr(data), R, P, T, _ptr(out)))
    return out
