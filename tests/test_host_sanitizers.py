"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU): the library is
rebuilt with the sanitizers on its host side only (each -fsanitize after -Xarch_host; the
device code is built as usual and never runs here), and the plain C consumer of the ABI
(tests/c/abi_consumer.c) drives the calls that need no GPU: options, shape and option
validation, memory accounting, autotuner argument checks and error reporting.  Any
sanitizer report fails the test."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1802_08938_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
SOURCES = ["did_engine.hip", "did_kernels.hip", "did_thin.hip", "did_batch.hip", "did_static.hip"]


def test_host_code_clean_under_asan_and_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    lib = str(tmp_path / "libdid.so")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", *san,
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
                    *[os.path.join(CSRC, s) for s in SOURCES], "-o", lib],
                   check=True, capture_output=True, timeout=900)
    exe = str(tmp_path / "abi_consumer")
    subprocess.run([CLANG, "-std=c99", "-g", "-fsanitize=address,undefined", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c", "abi_consumer.c"), "-L", str(tmp_path), "-ldid",
                    "-Wl,-rpath," + str(tmp_path), "-o", exe], check=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "AddressSanitizer" not in out.stderr and "runtime error" not in out.stderr, out.stderr
    assert "FAIL" not in out.stdout
