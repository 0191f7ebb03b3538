"""Parity at the benchmark's full sizes, in the launch configuration bench.py times.

The oracle cannot run a whole iteration at these sizes, but each half of Alg. 3 splits
into independent pieces it can check one by one:

* C half: column j of C after the sweep depends only on x_j, B^t and c_j^t (eq. sol:c_ij
  with the running residual of eq. up:c).  Sampled columns, including the ragged last
  tile, are recomputed by ``oracle.c_half``.
* B half: row m of B^{t+1} depends only on row m of B^t, row m of W = E' C'^T and
  V = tril(C' C'^T) (eqs. W_j, V_j and the delta-b rule).  With C' taken from the GPU,
  W's sampled rows and V are formed in float64 on the host and ``oracle.b_half`` gives
  the expected rows.
"""

import numpy as np
import pytest

import oracle
import paper_1802_08938_amd as did
from tests._gpu import announce, read_factors, rel_fro, require_gpu

pytestmark = pytest.mark.gpu

TOL_FACTORS = 1e-5


def _run_one_iteration(torch, Xt, M, N, K, n_blocks, tiled=0, x_dtype=did.DID_F32):
    o = did.did_default_opts()
    o.n_blocks = n_blocks
    o.borrow_x = 1
    o.x_tiled = tiled
    o.x_dtype = x_dtype
    h = did.did_init_ex(Xt, M, N, K, 12345, o)
    try:
        B0, C0 = read_factors(h, M, N, K)
        did.did_iterate(h, 1)
        B1, C1 = read_factors(h, M, N, K)
    finally:
        did.did_free(h)
    return B0, C0, B1, C1


def _check_c_columns(Xt, B0, C0, C1, cols):
    Xc = Xt[cols].double().cpu().numpy().T  # M x len(cols)
    Cs = C0[:, cols].copy()
    E = Xc - B0 @ Cs
    oracle.c_half(B0, Cs, E)
    err = rel_fro(C1[:, cols], Cs)
    assert err <= TOL_FACTORS, err
    return err


def _check_b_rows_chunked(Xt, B0, C1, rows, chunk):
    """Rows of B^{t+1} from W's rows and V accumulated over column chunks (float64)."""
    N = C1.shape[1]
    K = C1.shape[0]
    W = np.zeros((len(rows), K))
    V = np.zeros((K, K))
    Br = B0[rows]
    for a in range(0, N, chunk):
        b = min(N, a + chunk)
        Xr = Xt[a:b, rows].double().cpu().numpy().T  # len(rows) x (b - a)
        Cc = C1[:, a:b]
        W += (Xr - Br @ Cc) @ Cc.T
        V += Cc @ Cc.T
    Bexp = Br.copy()
    oracle.b_half(Bexp, W, np.tril(V))
    return Bexp


def test_large_workload_full_size_sampled():
    """M = 5000, N = 10^6, K = 50, 64 column blocks, X kept in tile order: the benchmark's
    workload and launch configuration.  Sampled columns of C and rows of B against the
    oracle; the whole of B and C bitwise against the same iteration on X read as given."""
    from workloads import large_halfnormal_device

    torch = require_gpu()
    M, N, K = 5000, 1_000_000, 50
    announce("full-size large workload, one iteration")
    Xt = large_halfnormal_device(torch, M=M, N=N, K=K, seed=3, n_blocks=64)
    torch.cuda.synchronize()
    B0, C0, B1, C1 = _run_one_iteration(torch, Xt, M, N, K, 64, tiled=1)
    B0g, C0g, B1g, C1g = _run_one_iteration(torch, Xt, M, N, K, 64, tiled=0)
    np.testing.assert_array_equal(B0, B0g)
    np.testing.assert_array_equal(C0, C0g)
    np.testing.assert_array_equal(B1, B1g)
    np.testing.assert_array_equal(C1, C1g)
    del B0g, C0g, B1g, C1g
    rng = np.random.default_rng(8)
    cols = sorted(set(rng.choice(N, 96, replace=False).tolist()) | {0, 1, 31, 32, 15624, 15625, N - 33, N - 1})
    ec = _check_c_columns(Xt, B0, C0, C1, cols)
    rows = sorted(set(rng.choice(M, 12, replace=False).tolist()) | {0, 31, 32, 4991, M - 1})
    Bexp = _check_b_rows_chunked(Xt, B0, C1, rows, 200_000)
    eb = rel_fro(B1[rows], Bexp)
    print(f"full-size large: sampled C columns rel err {ec:.2e}, sampled B rows rel err {eb:.2e}")
    assert eb <= TOL_FACTORS, eb
    del Xt
    torch.cuda.empty_cache()


def test_large_workload_full_size_bf16_sampled():
    """The precision form at full size: the large workload with X stored as bf16 (two
    tiled copies), one iteration, sampled columns of C and rows of B against the oracle's
    halves on bf16(X) (round to nearest even, as the engine stores it)."""
    from workloads import large_halfnormal_device

    torch = require_gpu()
    M, N, K = 5000, 1_000_000, 50
    announce("full-size large workload, X stored as bf16, one iteration")
    Xt = large_halfnormal_device(torch, M=M, N=N, K=K, seed=3, n_blocks=64)
    torch.cuda.synchronize()
    B0, C0, B1, C1 = _run_one_iteration(torch, Xt, M, N, K, 64, x_dtype=did.DID_BF16)
    Xb = Xt.to(torch.bfloat16)  # the values the engine iterates on
    del Xt
    torch.cuda.synchronize()
    rng = np.random.default_rng(10)
    cols = sorted(set(rng.choice(N, 96, replace=False).tolist()) | {0, 31, 32, N - 33, N - 1})
    ec = _check_c_columns(Xb, B0, C0, C1, cols)
    rows = sorted(set(rng.choice(M, 12, replace=False).tolist()) | {0, 31, 32, M - 1})
    Bexp = _check_b_rows_chunked(Xb, B0, C1, rows, 200_000)
    eb = rel_fro(B1[rows], Bexp)
    print(f"full-size large, bf16 X: sampled C columns rel err {ec:.2e}, sampled B rows rel err {eb:.2e}")
    assert eb <= TOL_FACTORS, eb
    del Xb
    torch.cuda.empty_cache()


def test_paper_shape_full_size():
    """M = 5, K = 3, N = 10^8 on the thin-matrix path: sampled columns of C, and all of B
    (M = 5 rows) from W and V accumulated over the whole of X in float64."""
    from workloads import paper_synthetic_device

    torch = require_gpu()
    M, N, K = 5, 100_000_000, 3
    announce("full-size experiments' shape, one iteration")
    Xt = paper_synthetic_device(torch, N, M=M, K=K, seed=4)
    torch.cuda.synchronize()
    B0, C0, B1, C1 = _run_one_iteration(torch, Xt, M, N, K, 16)
    rng = np.random.default_rng(9)
    cols = sorted(set(rng.choice(N, 256, replace=False).tolist()) | {0, 255, 256, N - 257, N - 1})
    ec = _check_c_columns(Xt, B0, C0, C1, cols)
    Bexp = _check_b_rows_chunked(Xt, B0, C1, list(range(M)), 10_000_000)
    eb = rel_fro(B1, Bexp)
    print(f"full-size paper shape: sampled C columns rel err {ec:.2e}, B rel err {eb:.2e}")
    assert eb <= TOL_FACTORS, eb
    del Xt
    torch.cuda.empty_cache()
