"""Build libmte.so (HIP for gfx950 plus the C++ host runtime) in-tree.

    python -m paper_1902_06828_amd.build        # or build() from Python

Every source is compiled by hipcc for gfx950 only, with denormals kept
(-fno-gpu-flush-denormals-to-zero) and packed FP32 instructions disabled; the
objects are linked into paper_1902_06828_amd/libmte.so.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmte.so")

SOURCES = ["kernels_k4.hip", "kernels_k8.hip", "kernels_k16.hip", "kernels.hip", "lists.hip", "gauss.hip", "noalloc.hip", "solo.hip", "runtime.cpp",
           "api.cpp", "greedy.cpp", "serve.cpp", "network.cpp", "gauss.cpp"]

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANGXX = "/opt/rocm/llvm/bin/clang++" if os.path.exists("/opt/rocm/llvm/bin/clang++") else "g++"

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-I", INCLUDE, "-I", CSRC]
# Device code: gfx950 only; denormals kept (distances are exact binary32
# differences); packed FP32 disabled; IEEE mode off with no NaNs assumed, which
# drops the quieting of max/min operands (the inputs are finite and no step
# can produce a NaN, so min, max, med3 and compares give the same results).
DEVICE = ["-x", "hip", "--offload-arch=gfx950", "-fno-gpu-flush-denormals-to-zero",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-fno-honor-nans", "-mno-amdgpu-ieee"]
HOST = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    flags = DEVICE if src.endswith(".hip") else HOST
    cmd = [HIPCC] + COMMON + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def hip_runtime() -> str:
    """The HIP runtime library to link: the copy bundled with PyTorch when it
    is installed (PyTorch owns the device buffers and streams handed to the
    library, and one process must use a single HIP runtime), else ROCm's."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec and spec.origin:
        cand = os.path.join(os.path.dirname(spec.origin), "lib", "libamdhip64.so")
        if os.path.exists(cand):
            return cand
    return "/opt/rocm/lib/libamdhip64.so"


# Host-code sanitizer build: the host C++ sources (and the host side of the
# allocation-free entry point) with AddressSanitizer and UndefinedBehavior-
# Sanitizer, linked with the same device objects into libmte_san.so.  It is
# loaded through MTE_LIBRARY with the sanitizer runtime preloaded
# (sanitizer_env()); device code is never instrumented.
LIB_SAN = os.path.join(PKG, "libmte_san.so")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
SAN_SOURCES = [s for s in SOURCES if s.endswith(".cpp")] + ["noalloc.hip"]


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime to preload into a process that
    loads a sanitized library."""
    r = subprocess.run([CLANGXX, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


def sanitizer_env(env=None) -> dict:
    """Environment for a Python process that loads libmte_san.so."""
    e = dict(os.environ if env is None else env)
    e["MTE_LIBRARY"] = LIB_SAN
    # the sanitizer runtime must come first; anything already preloaded stays
    e["LD_PRELOAD"] = ":".join(x for x in (asan_runtime(), e.get("LD_PRELOAD", "")) if x)
    e["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    e["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return e


def _compile_san(src: str) -> str:
    d = os.path.join(BUILD, "san")
    obj = os.path.join(d, os.path.basename(src) + ".o")
    if src.endswith(".hip"):
        flags = DEVICE + [x for f in SAN for x in ("-Xarch_host", f)]
    else:
        flags = HOST + SAN
    cmd = [HIPCC] + COMMON + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build_sanitized(verbose: bool = False) -> str:
    """libmte_san.so (after build(): the device objects come from it)."""
    os.makedirs(os.path.join(BUILD, "san"), exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SAN_SOURCES))) as ex:
        san = dict(zip(SAN_SOURCES, ex.map(_compile_san, SAN_SOURCES)))
    objs = [san.get(s, os.path.join(BUILD, os.path.basename(s) + ".o")) for s in SOURCES]
    tmp = LIB_SAN + ".tmp"
    rt = hip_runtime()
    cmd = [CLANGXX, "-shared", "-fPIC", "-fsanitize=address,undefined", "-o", tmp] + objs + [
        rt, "-Wl,-rpath," + os.path.dirname(rt), "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB_SAN)
    if verbose:
        print("built", LIB_SAN)
    return LIB_SAN


# The VALU issue-rate probe (a program of its own, not part of the library):
# the measurement behind the ALU peaks the benchmark prices kernels against.
PROBE = os.path.join(PKG, "valu_issue_probe")


def build_probe(verbose: bool = False) -> str:
    cmd = [HIPCC, "-O3", "-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", os.path.join(CSRC, "valu_issue_probe.hip"), "-o", PROBE + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(PROBE + ".tmp", PROBE)
    if verbose:
        print("built", PROBE)
    return PROBE


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    rt = hip_runtime()
    # plain link (no hipcc driver), so the only HIP runtime dependency is `rt`
    cmd = [CLANGXX, "-shared", "-fPIC", "-o", tmp] + objs + [
        rt, "-Wl,-rpath," + os.path.dirname(rt), "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    build_probe(verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    if "--sanitize" in sys.argv:
        build_sanitized(verbose=True)
    sys.exit(0)
