"""The GPU path driven from C: tests/c/abi_gpu.c, compiled with gcc against include/did.h
and linked to the in-tree libdid.so, runs a planted instance alone and in a batch through
the ABI only (host X in, factors and objectives out) and checks monotone objective,
nonnegative factors and batch = alone bit for bit.  The same instance run through the
Python binding must give the same objective history bit for bit."""

import os
import shutil
import subprocess

import numpy as np
import pytest

import paper_1802_08938_amd as did
from tests._gpu import announce, require_gpu

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_DIR = os.path.join(ROOT, "paper_1802_08938_amd")


def _lcg_planted(M, N, K, state):
    """The C program's planted X: its linear congruential sequence, B0 then C0, and
    X = B0 C0 summed over k in ascending order in float64, rounded to float32."""
    mask = (1 << 64) - 1

    def draws(n):
        nonlocal state
        out = np.empty(n, np.float32)
        for i in range(n):
            state = (state * 6364136223846793005 + 1442695040888963407) & mask
            out[i] = np.float32(((state >> 40) & 0xFFFFFF) / 16777216.0)
        return out

    B0 = draws(M * K).reshape(K, M).T.astype(np.float64)  # column-major M x K
    C0 = draws(K * N).reshape(N, K).T.astype(np.float64)  # column-major K x N
    X = np.zeros((M, N))
    for k in range(K):
        X += B0[:, k:k + 1] * C0[k:k + 1, :]
    return X.astype(np.float32), state


def test_c_program_runs_the_gpu_path(tmp_path):
    torch = require_gpu()
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    announce("C consumer of the ABI on the GPU")
    exe = str(tmp_path / "abi_gpu")
    subprocess.run([cc, "-std=c99", "-Wall", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c", "abi_gpu.c"), "-L", LIB_DIR, "-ldid",
                    "-Wl,-rpath," + LIB_DIR, "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "FAIL" not in out.stdout
    hist_c = [float(v) for v in next(l for l in out.stdout.splitlines() if l.startswith("history")).split()[1:]]
    # the same instance through the Python binding: the C program's first planted X
    X, _ = _lcg_planted(300, 2000, 12, 12345)
    h = did.did_init(np.asfortranarray(X), 300, 2000, 12, 7)
    try:
        did.did_iterate(h, 20)
        hist_py = did.did_history(h)
    finally:
        did.did_free(h)
    assert len(hist_c) == 20
    assert hist_py == hist_c
