"""ASan/UBSan builds of the host-side C and C++ code (no GPU).

- The library's host-only CSR helpers (kh_csr.cpp: kh_validate_csr, the
  canonicalisation behind KH_CANONICALIZE, kh_buffer_size, kh_status_str) are
  built with the driver in tests/sanitize/ and run over valid, malformed and
  hostile inputs.
- The C oracle is built with the same sanitizers and loaded (KH_ORACLE_LIB)
  into a child Python that runs every oracle entry point on small graphs.
Any sanitizer report aborts the child and fails the test.  The device code is
not covered: GPU sanitizers are not available here."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="gcc/g++ not available")


def runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_csr_helpers_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "csr_driver")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "paper_2112_06154_amd", "csrc"),
                           os.path.join(ROOT, "tests", "sanitize", "csr_driver.cpp"),
                           os.path.join(ROOT, "paper_2112_06154_amd", "csrc", "kh_csr.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert "csr helpers ok" in r.stdout


CHILD = r"""
import numpy as np
import graphgen as gg
import oracle
g = gg.chung_lu(300, 1200, 2.1, seed=5)
e = gg.erdos_renyi(40, 90, seed=2)
r = oracle.ranks(g.n, 3)
for h in (1, 2, 3):
    oracle.hdeg(g, h, with_te=True)
    oracle.hdeg_list(g, h, np.arange(0, g.n, 7), with_te=True)
    c = oracle.exact_core(g, h)
    cs = oracle.sampled_core(g, h, r, 40)
    oracle.sampled_core(g, h, r, 40, early_stop=True)
    oracle.estimate_all(g, h, r, 40)
    oracle.dense(g, c, h)
    oracle.dense(g, cs, h, mode="sampled", r=oracle.ranks(g.n, 3, 1), M=60, prune=True)
    order, core, rnd = oracle.bulk_order(g, h, "sampled", r, 40)
    oracle.dense_suffix(g, order, h, "sampled", oracle.ranks(g.n, 3, 1), 60)
    oracle.exact_core_sweep(e, h)
for i in (1, 2, 3):
    oracle.sampled_lists(g, i, r, 40)
oracle.exact_core(gg.empty(1), 2)
print("oracle ok")
"""


def test_oracle_under_asan_ubsan(tmp_path):
    asan, ubsan = runtime("libasan.so"), runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("sanitizer runtimes not found")
    so = str(tmp_path / "libkhoracle_san.so")
    subprocess.check_call(["gcc", "-std=c11", "-fPIC", "-shared", *SAN, "-o", so,
                           os.path.join(ROOT, "oracle", "khoracle.c"), "-lm"])
    env = {**os.environ, "KH_ORACLE_LIB": so, "LD_PRELOAD": f"{asan}:{ubsan}",
           # the Python interpreter itself is not built for leak checking
           "ASAN_OPTIONS": "detect_leaks=0", "UBSAN_OPTIONS": "print_stacktrace=1",
           "PYTHONPATH": ROOT}
    r = subprocess.run([sys.executable, "-c", CHILD], capture_output=True, text=True, timeout=600, env=env, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "oracle ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
