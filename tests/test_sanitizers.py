"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds the oracle (g++) and the C-ABI library's host code (hipcc, sanitizers
on the host side only: -Xarch_host before each -fsanitize) with both
sanitizers, and runs tests/sanitizer_driver.py against them in a child process
with the sanitizer runtime preloaded.  Any report aborts the child (UBSan
without recovery), which fails the test.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "sanitizer_driver.py")

pytestmark = pytest.mark.slow


def _run(kind, lib, runtime, tmp_path):
    env = dict(os.environ, LD_PRELOAD=runtime, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, DRIVER, kind, lib, ROOT], env=env, capture_output=True, text=True,
                       timeout=600, cwd=str(tmp_path))
    assert r.returncode == 0 and "sanitized run ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


def test_oracle_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                    "-ffp-contract=off", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-o", lib, os.path.join(ROOT, "oracle", "chem_oracle.cpp")],
                   check=True)
    runtime = ":".join(subprocess.check_output(["gcc", f"-print-file-name={n}"], text=True).strip()
                       for n in ("libasan.so", "libubsan.so"))
    _run("oracle", lib, runtime, tmp_path)


def test_library_host_code_under_asan_ubsan(tmp_path):
    rts = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rts or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("no ROCm clang sanitizer runtime")
    lib = str(tmp_path / "libchem_san.so")
    subprocess.run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-fno-fast-math",
                    "-ffp-contract=fast", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                    "-w", "-I", os.path.join(ROOT, "include"), "-o", lib,
                    os.path.join(ROOT, "paper_2105_12070_amd", "csrc", "chem.hip")], check=True,
                   capture_output=True)
    _run("library", lib, rts[0], tmp_path)
