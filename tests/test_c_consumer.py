"""The boundary from C: a plain C program (tests/c/abi_consumer.c) compiled with gcc
against include/did.h and linked to the in-tree libdid.so runs the calls that need no
GPU.  This checks that the header is C (not only C++ behind ctypes) and that every call
it makes links."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_DIR = os.path.join(ROOT, "paper_1802_08938_amd")


def test_c_program_builds_links_and_runs(tmp_path):
    if not os.path.exists(os.path.join(LIB_DIR, "libdid.so")):
        pytest.skip("libdid.so is not built")
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = str(tmp_path / "abi_consumer")
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c", "abi_consumer.c"), "-L", LIB_DIR, "-ldid",
                    "-Wl,-rpath," + LIB_DIR, "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "FAIL" not in out.stdout
