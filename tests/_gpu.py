"""Helpers for GPU tests: run the HIP path through the C ABI and compare with the oracle."""

from __future__ import annotations

import sys

import numpy as np
import pytest

import paper_1802_08938_amd as did


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    try:
        did.lib()
    except did.DidLibraryMissing as e:  # a GPU without the library is a failure, not a skip
        raise AssertionError(str(e))
    return torch


def announce(msg):
    print(f"\n[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def device_x(torch, X32):
    """Column-major float32 X (M x N) on the device: a (N, M) row-major tensor."""
    Xc = np.ascontiguousarray(np.asarray(X32, dtype=np.float32).T)
    Xd = torch.from_numpy(Xc).to("cuda")
    torch.cuda.synchronize()  # the engine reads X on its own stream
    return Xd


def read_factors(h, M, N, K):
    Bt = np.empty((K, M), dtype=np.float32)
    Ct = np.empty((N, K), dtype=np.float32)
    did.did_factors(h, Bt, Ct)
    return Bt.T.astype(np.float64), Ct.T.astype(np.float64)


def run_gpu(torch, X32, K, seed=12345, iters=(1,), opts=None, B0=None, C0=None):
    """Run the GPU path; returns dict with initial factors, factors after each requested
    cumulative iteration count, the objective history and the final objective."""
    M, N = X32.shape
    Xd = device_x(torch, X32)
    if B0 is not None:
        Bd = torch.from_numpy(np.ascontiguousarray(np.asarray(B0, np.float32).T)).to("cuda")
        Cd = torch.from_numpy(np.ascontiguousarray(np.asarray(C0, np.float32).T)).to("cuda")
        torch.cuda.synchronize()
        h = did.did_init_from_factors(Xd, M, N, K, Bd, Cd, opts)
    else:
        h = did.did_init_ex(Xd, M, N, K, seed, opts)
    try:
        out = {"init": read_factors(h, M, N, K)}
        done = 0
        for n in iters:
            did.did_iterate(h, n - done)
            done = n
            out[n] = read_factors(h, M, N, K)
        out["hist"] = np.array(did.did_history(h))
        out["f"] = did.did_objective(h)
    finally:
        did.did_free(h)
    return out


def rel_fro(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
