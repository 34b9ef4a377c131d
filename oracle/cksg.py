"""ctypes loader and build step for oracle/ksg_oracle.c.  TEST INFRASTRUCTURE ONLY."""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ksg_oracle.c")
# ORACLE_LIBRARY selects the sanitizer build (libksg_oracle_san.so)
LIB = os.environ.get("ORACLE_LIBRARY") or os.path.join(HERE, "libksg_oracle.so")
LIB_SAN = os.path.join(HERE, "libksg_oracle_san.so")
CLANG = "/opt/rocm/llvm/bin/clang"


def build() -> str:
    """Compile the C oracle (plain gcc, no fast-math, no FP contraction)."""
    out = os.path.join(HERE, "libksg_oracle.so")
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                           "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, out)
    return out


def build_sanitized() -> str:
    """The same oracle with AddressSanitizer and UndefinedBehaviorSanitizer
    (clang, whose runtime the sanitized library build also uses)."""
    omp = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(CLANG))), "lib")
    tmp = LIB_SAN + ".tmp"
    subprocess.check_call([CLANG, "-O1", "-g", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-shared", "-fPIC", "-o", tmp, SRC, "-lm",
                           "-L" + omp, "-Wl,-rpath," + omp])
    os.replace(tmp, LIB_SAN)
    return LIB_SAN


_lib = None


def lib():
    global _lib
    if _lib is None:
        if LIB == os.path.join(HERE, "libksg_oracle.so") and (
                not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build()
        L = ctypes.CDLL(LIB)
        f = L.oracle_ksg
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                      ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                      ctypes.c_void_p, ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def eps_and_counts(x, y, z, k: int, queries=None, threads: int = 0, theiler: int = 0):
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    x = x[None, :] if x.ndim == 1 else x
    y = y[None, :] if y.ndim == 1 else y
    n = x.shape[1]
    if z is not None:
        z = np.ascontiguousarray(z, dtype=np.float32)
        z = z[None, :] if z.ndim == 1 else z
    dz = 0 if z is None else z.shape[0]
    q = None if queries is None else np.ascontiguousarray(queries, dtype=np.int64)
    m = n if q is None else len(q)
    eps = np.empty(m, np.float32)
    cx, cy, cz = (np.empty(m, np.int32) for _ in range(3))
    cmi = ctypes.c_double(0.0)
    rc = lib().oracle_ksg(_ptr(x), x.shape[0], _ptr(y), y.shape[0], _ptr(z), dz, n, k, theiler, threads,
                          _ptr(q), m, _ptr(eps), _ptr(cx), _ptr(cy), _ptr(cz),
                          ctypes.byref(cmi))
    if rc != 0:
        raise ValueError("oracle_ksg rejected its arguments")
    return eps, cx, cy, cz, (cmi.value if q is None else None)


def cmi_ksg(x, y, z, k: int = 4, threads: int = 0, theiler: int = 0):
    return eps_and_counts(x, y, z, k, None, threads, theiler)[4]


def max_threads() -> int:
    return lib().oracle_max_threads()
