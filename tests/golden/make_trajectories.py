"""Write the oracle's objective trajectories (and, for the largest case, sampled factors
after one iteration) that the GPU parity tests compare against.

Each case runs ``oracle.did_run`` (Alg. 3 in float64) on seeded synthetic data from
``workloads`` and initial factors from ``workloads.uniform_init`` rounded to float32 (the
values the GPU is given).  Nothing here touches the GPU path.  Usage:

    python tests/golden/make_trajectories.py CASE [CASE ...]   # or: all

Output: tests/golden/traj_<case>.json with the recipe, f[0..T] and a checksum of the
float32 data (sum and sum of squares in float64).
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import (as_oracle_input, image_like, large_halfnormal, round_to_bf16, serving_x,  # noqa: E402
                       to_f32_colmajor, uniform_init)

INIT_SEED = 12345


def _x_image():
    return image_like(784, 70000, 16, seed=2)[0]


def _x_large(blocks):
    return large_halfnormal(5000, 1_000_000, 50, seed=3, n_blocks=64, take_blocks=blocks)[0]


# name -> (data builder, K, P, T, bf16 storage, sampled columns/rows after one iteration)
CASES = {
    "image_like_p4": (_x_image, 16, 4, 50, False, False),
    "large_slice_b1": (lambda: _x_large(1), 50, 1, 50, False, False),
    "large_slice_b4": (lambda: _x_large(4), 50, 4, 50, False, True),
    "large_slice_b1_bf16": (lambda: _x_large(1), 50, 1, 50, True, False),
    "serving_1868x40000_k60": (lambda: serving_x(1868, 40000, 60, seed=7), 60, 1, 5, False, False),
    "serving_3809x2248_k49": (lambda: serving_x(3809, 2248, 49, seed=6), 49, 1, 5, False, False),
}


def sample_indices(n, count, seed):
    """Sorted sample of indices, always including the first and last two and tile edges."""
    r = np.random.default_rng(seed)
    s = set(r.choice(n, count, replace=False).tolist()) | {0, 1, 31, 32, n - 33, n - 2, n - 1}
    return sorted(i for i in s if 0 <= i < n)


def initial_factors(M, N, K):
    B0, C0 = uniform_init(M, N, K, INIT_SEED)
    return B0.astype(np.float32).astype(np.float64), C0.astype(np.float32).astype(np.float64)


def data(case):
    build, K, P, T, bf16, sampled = CASES[case]
    X32 = to_f32_colmajor(build())
    Xo = round_to_bf16(X32) if bf16 else as_oracle_input(X32)
    return X32, Xo, K, P, T, bf16, sampled


def run(case):
    X32, Xo, K, P, T, bf16, sampled = data(case)
    M, N = Xo.shape
    B0, C0 = initial_factors(M, N, K)
    t0 = time.perf_counter()
    out = {"case": case, "M": M, "N": N, "K": K, "P": P, "T": T, "x_storage": "bf16" if bf16 else "f32",
           "init": f"workloads.uniform_init(M, N, K, {INIT_SEED}) rounded to float32",
           "x_sum": float(np.sum(Xo)), "x_sumsq": float(np.sum(Xo * Xo))}
    if sampled:
        B1, C1, f1 = oracle.did_run(Xo, B0, C0, 1, P=P)
        cols = sample_indices(N, 64, 11)
        rows = sample_indices(M, 24, 12)
        out["sample_cols"] = cols
        out["sample_rows"] = rows
        out["C1_cols"] = C1[:, cols].T.tolist()  # one list per sampled column
        out["B1_rows"] = B1[rows].tolist()
        _, _, ft = oracle.did_run(Xo, B1, C1, T - 1, P=P)
        f = np.concatenate([f1, ft[1:]])
    else:
        _, _, f = oracle.did_run(Xo, B0, C0, T, P=P)
    out["f"] = [float(v) for v in f]
    out["oracle_seconds"] = round(time.perf_counter() - t0, 1)
    path = os.path.join(HERE, f"traj_{case}.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"{case}: T={T} f[0]={f[0]:.6e} f[T]={f[-1]:.6e} ({out['oracle_seconds']} s) -> {path}", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or ["all"]
    if names == ["all"]:
        names = list(CASES)
    for n in names:
        run(n)
