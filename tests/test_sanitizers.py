"""Host sanitizer runs (CPU only): AddressSanitizer and UndefinedBehaviorSanitizer
over the library's host-side setup code and over the oracle.

* ``csrc/host_setup.cpp`` (operator tables, interaction lists, level layout,
  M2L work items, boundary strips) is built with clang++
  ``-fsanitize=address,undefined -fno-sanitize-recover=all`` together with
  ``tests/sanitize/host_setup_check.cpp``, which builds every table for
  p = 2..20, six near sets and three grid sizes, and the work lists of trees
  with 0..9 levels, and checks their properties.
* ``oracle/fmm_oracle.c`` is built with gcc and the same sanitizers, and the
  whole ``-m "not gpu"`` suite runs against that build (through
  ``FMM_ORACLE_LIB``, with the ASan runtime preloaded into Python).

The GPU-side code and the HIP runtime calls are not covered (no GPU sanitizer
runs on this hardware's pool); the library's own host code that drives the
kernels runs under the GPU tests.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1308_3339_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g",
       "-O1"]

pytestmark = pytest.mark.skipif(os.environ.get("FMM_SANITIZER_RUN") == "1",
                                reason="already inside a sanitizer run")


def _have(cmd):
    return shutil.which(cmd) is not None or os.path.exists(cmd)


@pytest.mark.timeout(300)
def test_host_setup_under_asan_and_ubsan(tmp_path):
    if not _have(CLANG):
        pytest.skip("clang++ not found")
    exe = str(tmp_path / "host_setup_check")
    subprocess.check_call([CLANG, "-std=c++17", *SAN, "-I", CSRC,
                           os.path.join(CSRC, "host_setup.cpp"),
                           os.path.join(ROOT, "tests", "sanitize", "host_setup_check.cpp"),
                           "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=240)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0
    assert "host setup check ok" in r.stdout
    assert "0 failures" in r.stdout


@pytest.mark.timeout(600)
def test_cpu_suite_against_sanitized_oracle(tmp_path):
    if not _have("gcc"):
        pytest.skip("gcc not found")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not asan or not os.path.exists(asan):
        pytest.skip("libasan not found")
    lib = str(tmp_path / "libfmm_oracle_asan.so")
    subprocess.check_call(["gcc", "-std=gnu99", *SAN, "-fopenmp", "-fPIC", "-shared", "-o", lib,
                           os.path.join(ROOT, "oracle", "fmm_oracle.c"), "-lm"])
    env = dict(os.environ)
    env.update({"FMM_ORACLE_LIB": lib, "LD_PRELOAD": asan, "FMM_SANITIZER_RUN": "1",
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", os.path.join(ROOT, "tests")],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=540)
    tail = r.stdout[-3000:] + r.stderr[-3000:]
    print(tail)
    assert r.returncode == 0, tail
    assert "passed" in r.stdout
    assert "AddressSanitizer" not in tail and "runtime error" not in tail
