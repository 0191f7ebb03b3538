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


GOLDEN_DIR = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def worst_line(a, o, axis=1, floor_frac=1e-2):
    """Largest relative error of one row (axis=1: rows of B) or one column (axis=0: columns
    of C) of a against the oracle's o.  A line whose oracle norm is below floor_frac of the
    root-mean-square line norm is measured against that floor: such a line carries less
    than floor_frac^2 of an average line's weight, and a projection [z]_+ flipping at z ~ 0
    there moves it by rounding only."""
    a = np.asarray(a, np.float64)
    o = np.asarray(o, np.float64)
    d = np.linalg.norm(a - o, axis=axis)
    n = np.linalg.norm(o, axis=axis)
    rms = float(np.sqrt(np.mean(n * n))) if n.size else 0.0
    den = np.maximum(n, floor_frac * rms)
    den = np.where(den > 0, den, 1.0)
    return float(np.max(d / den)) if d.size else 0.0


def check_factors(B, Bo, C, Co, tol=1e-5, tol_line=1e-4, label=""):
    """Normwise bars (relative Frobenius error of B and of C) and per-line bars (worst row
    of B, worst column of C); prints the four numbers and returns them."""
    eb, ec = rel_fro(B, Bo), rel_fro(C, Co)
    lb, lc = worst_line(B, Bo, axis=1), worst_line(C, Co, axis=0)
    print(f"[factors] {label} B {eb:.2e} C {ec:.2e} worst row of B {lb:.2e} worst column of C {lc:.2e}", flush=True)
    assert eb <= tol, (label, "B normwise", eb)
    assert ec <= tol, (label, "C normwise", ec)
    assert lb <= tol_line, (label, "worst row of B", lb)
    assert lc <= tol_line, (label, "worst column of C", lc)
    return eb, ec, lb, lc


def check_trajectory(fg, fo, tol=1e-4, label=""):
    """max_t |f_gpu[t] - f_oracle[t]| / f_oracle[t] over the common length."""
    fg = np.asarray(fg, np.float64)
    fo = np.asarray(fo, np.float64)
    assert fg.shape == fo.shape, (label, fg.shape, fo.shape)
    err = float(np.max(np.abs(fg - fo) / fo))
    print(f"[trajectory] {label} {len(fo) - 1} iterations: max relative error {err:.2e}", flush=True)
    assert err <= tol, (label, err)
    return err


def load_golden(case):
    """Oracle trajectory written by tests/golden/make_trajectories.py (calls only oracle/)."""
    import json
    import os

    path = os.path.join(GOLDEN_DIR, f"traj_{case}.json")
    if not os.path.exists(path):
        pytest.fail(f"missing {path}: run python tests/golden/make_trajectories.py {case}")
    with open(path) as fh:
        return json.load(fh)
