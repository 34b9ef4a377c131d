"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The library's host C++ (validation, layouts, the request loop, the greedy
search, the tests, network statistics) and the C oracle are rebuilt with both
sanitizers (libmte_san.so, libksg_oracle_san.so; device code is not
instrumented) and the whole CPU suite (this file aside) runs in a
subprocess that loads them, with the sanitizer runtime preloaded.  Any report
aborts that process."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import cksg  # noqa: E402
from paper_1902_06828_amd import build as B  # noqa: E402


def test_host_code_under_sanitizers():
    if not (os.path.exists(B.LIB_SAN) and os.path.exists(cksg.LIB_SAN)):
        pytest.skip("sanitizer builds missing: run __graft_entry__.build()")
    env = B.sanitizer_env()
    env["ORACLE_LIBRARY"] = cksg.LIB_SAN
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests", "--deselect", "tests/test_sanitized_host.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail


def test_sanitized_builds_are_the_ones_loaded():
    if not (os.path.exists(B.LIB_SAN) and os.path.exists(cksg.LIB_SAN)):
        pytest.skip("sanitizer builds missing: run __graft_entry__.build()")
    env = B.sanitizer_env()
    env["ORACLE_LIBRARY"] = cksg.LIB_SAN
    probe = ("import paper_1902_06828_amd as m\n"
             "from oracle import cksg\n"
             "m.lib(); cksg.lib()\n"
             "maps = open('/proc/self/maps').read()\n"
             "print('mte', 'libmte_san.so' in maps, 'oracle', 'libksg_oracle_san.so' in maps,\n"
             "      'asan', 'libclang_rt.asan' in maps)\n")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "mte True oracle True asan True" in r.stdout, r.stdout
