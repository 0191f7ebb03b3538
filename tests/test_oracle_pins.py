"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these tests re-types the oracle's own formulas: each compares it with something
independent of it -- hand-derived exact rationals, a brute-force 1-D minimiser, the
textbook sequential BCD written from scratch in exact arithmetic or with fresh residuals,
SVD / NNLS library routines, closed-form special cases and the paper's own invariants.
"""

import json
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.optimize import nnls

import oracle
from oracle import bcd
from workloads import identifiable_plant, planted_lowrank, uniform_init

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def _mat(rows):
    return np.array([[float(Fraction(v)) for v in r] for r in rows], dtype=np.float64)


def _load(name):
    with open(GOLDEN) as fh:
        return json.load(fh)[name]


# ---------------------------------------------------------------- P1 / P2 worked examples
@pytest.mark.parametrize("name", ["k1", "k2_clipping"])
def test_worked_example_one_iteration(name):
    g = _load(name)
    X, B0, C0 = _mat(g["X"]), _mat(g["B0"]), _mat(g["C0"])
    assert oracle.objective(X, B0, C0) == pytest.approx(float(Fraction(g["f0"])), rel=1e-15)
    B, C = B0.copy(), C0.copy()
    E = oracle.residual(X, B, C)
    oracle.c_half(B, C, E)
    np.testing.assert_allclose(C, _mat(g["C1"]), rtol=0, atol=1e-14)
    if "f_after_C_half" in g:
        assert 0.5 * np.sum(E * E) == pytest.approx(float(Fraction(g["f_after_C_half"])), rel=1e-14)
    W, V = oracle.messages(E, C, oracle.column_blocks(X.shape[1], 1))
    np.testing.assert_allclose(W, _mat(g["W"]), rtol=0, atol=1e-13)
    np.testing.assert_allclose(V, _mat(g["V"]), rtol=0, atol=1e-13)
    dB = oracle.b_half(B, W, V)
    E -= dB @ C
    np.testing.assert_allclose(B, _mat(g["B1"]), rtol=0, atol=1e-14)
    if "E1" in g:
        np.testing.assert_allclose(E, _mat(g["E1"]), rtol=0, atol=1e-14)
    f1 = float(Fraction(g["f1"]))
    assert 0.5 * np.sum(E * E) == pytest.approx(f1, rel=1e-13)
    # the same through the whole iteration (did_run)
    Bd, Cd, f = oracle.did_run(X, B0, C0, 1, check=True)
    assert f[1] == pytest.approx(f1, rel=1e-13)


def _naive_bcd_exact(X, B, C, T):
    """Sequential BCD in exact rationals: eq. sol:c_ij and eq. sol:b_i 2 from scratch."""
    M, N, K = len(X), len(X[0]), len(B[0])
    pos = lambda z: z if z > 0 else Fraction(0)  # noqa: E731
    for _ in range(T):
        for j in range(N):
            for i in range(K):
                nb = sum(B[m][i] ** 2 for m in range(M))
                if nb <= 0:
                    continue
                a = [X[m][j] - sum(B[m][k] * C[k][j] for k in range(K) if k != i) for m in range(M)]
                C[i][j] = pos(sum(B[m][i] * a[m] for m in range(M)) / nb)
        for i in range(K):
            z = sum(C[i][j] ** 2 for j in range(N))
            if z <= 0:
                continue
            for m in range(M):
                y = sum((X[m][j] - sum(B[m][k] * C[k][j] for k in range(K) if k != i)) * C[i][j]
                        for j in range(N))
                B[m][i] = pos(y / z)
    return B, C


@pytest.mark.parametrize("name", ["k1", "k2_clipping"])
def test_worked_example_equals_exact_sequential_bcd(name):
    """The golden values are one exact sequential-BCD iteration (the paper's 'Correctness')."""
    g = _load(name)
    X = [[Fraction(v) for v in r] for r in g["X"]]
    B = [[Fraction(v) for v in r] for r in g["B0"]]
    C = [[Fraction(v) for v in r] for r in g["C0"]]
    B, C = _naive_bcd_exact(X, B, C, 1)
    assert B == [[Fraction(v) for v in r] for r in g["B1"]]
    assert C == [[Fraction(v) for v in r] for r in g["C1"]]


def test_exact_bcd_vs_oracle_several_iterations_rational_inputs():
    """Three iterations on a small integer instance: oracle (FP64) vs exact rationals."""
    rng = np.random.default_rng(11)
    M, N, K = 4, 5, 2
    Xi = rng.integers(0, 6, size=(M, N))
    Bi = rng.integers(0, 3, size=(M, K)) + np.eye(M, K, dtype=int)
    Ci = rng.integers(0, 3, size=(K, N)) + np.eye(K, N, dtype=int)
    Xf = [[Fraction(int(v)) for v in r] for r in Xi]
    Bf = [[Fraction(int(v)) for v in r] for r in Bi]
    Cf = [[Fraction(int(v)) for v in r] for r in Ci]
    Bf, Cf = _naive_bcd_exact(Xf, Bf, Cf, 3)
    B, C, _ = oracle.did_run(Xi.astype(float), Bi.astype(float), Ci.astype(float), 3, check=True)
    np.testing.assert_allclose(B, np.array(Bf, dtype=float), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(C, np.array(Cf, dtype=float), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- P3 brute-force 1-D minimiser
def _argmin_1d_nonneg(a, b):
    """argmin_{t >= 0} 1/2 ||a - b t||^2 by a dense grid and golden-section refinement."""
    phi = lambda t: 0.5 * float(np.sum((a - b * t) ** 2))  # noqa: E731
    hi = 1.0
    while phi(hi) < phi(hi / 2) or hi < 1.0:
        hi *= 2.0
        if hi > 1e8:
            break
    grid = np.linspace(0.0, hi, 4001)
    vals = [phi(t) for t in grid]
    k = int(np.argmin(vals))
    lo, up = grid[max(k - 1, 0)], grid[min(k + 1, len(grid) - 1)]
    gr = (np.sqrt(5) - 1) / 2
    x1, x2 = up - gr * (up - lo), lo + gr * (up - lo)
    for _ in range(200):
        if phi(x1) < phi(x2):
            up, x2 = x2, x1
            x1 = up - gr * (up - lo)
        else:
            lo, x1 = x1, x2
            x2 = lo + gr * (up - lo)
    t = 0.5 * (lo + up)
    return 0.0 if phi(0.0) <= phi(t) else t


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_each_coordinate_is_the_1d_minimiser(seed):
    rng = np.random.default_rng(seed)
    M, N, K = 5, 4, 3
    X = rng.random((M, N)) * 2.0
    B0, C0 = rng.random((M, K)), rng.random((K, N)) * 1.5
    # C half: coordinates of each column in ascending order, each the 1-D minimiser
    Bb, Cb = B0.copy(), C0.copy()
    for j in range(N):
        for i in range(K):
            a = X[:, j] - Bb @ Cb[:, j] + Bb[:, i] * Cb[i, j]
            Cb[i, j] = _argmin_1d_nonneg(a, Bb[:, i])
    B, C = B0.copy(), C0.copy()
    E = oracle.residual(X, B, C)
    oracle.c_half(B, C, E)
    # a derivative-free search resolves a quadratic's minimiser to ~sqrt(eps) only
    np.testing.assert_allclose(C, Cb, rtol=0, atol=1e-7)
    # B half: separable by rows m; within a row, entries i ascending
    for m in range(M):
        for i in range(K):
            a = X[m, :] - Bb[m, :] @ Cb + Bb[m, i] * Cb[i, :]
            Bb[m, i] = _argmin_1d_nonneg(a, Cb[i, :])
    W, V = oracle.messages(E, C, oracle.column_blocks(N, 2))
    oracle.b_half(B, W, V)
    np.testing.assert_allclose(B, Bb, rtol=0, atol=1e-7)


# ---------------------------------------------------------------- P4 DID == sequential BCD
@pytest.mark.parametrize("shape", [(6, 8, 3), (8, 5, 4), (3, 7, 1), (7, 7, 2)])
def test_did_equals_naive_sequential_bcd(shape):
    M, N, K = shape
    rng = np.random.default_rng(M * 100 + N * 10 + K)
    X = rng.random((M, N)) * 3.0
    B0, C0 = rng.random((M, K)), rng.random((K, N))
    B, C, f = oracle.did_run(X, B0, C0, 20, P=3, check=True)
    Bn, Cn, fn, _ = bcd.naive_bcd_run(X, B0, C0, 20)
    np.testing.assert_allclose(B, Bn, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(C, Cn, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(f, fn, rtol=1e-11, atol=1e-13)


def test_dbcd_equals_did():
    rng = np.random.default_rng(5)
    M, N, K = 7, 9, 3
    X = rng.random((M, N))
    B0, C0 = rng.random((M, K)), rng.random((K, N))
    B, C, _ = oracle.did_run(X, B0, C0, 10, P=2)
    Bd, Cd = B0.copy(), C0.copy()
    for _ in range(10):
        bcd.dbcd_iteration(X, Bd, Cd, oracle.column_blocks(N, 2))
    np.testing.assert_allclose(B, Bd, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(C, Cd, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- P5 invariants
def test_invariants_planted_c1_shape():
    X, _, _ = planted_lowrank(M=500, N=2000, K=10, seed=1)
    B0, C0 = uniform_init(500, 2000, 10, seed=12345)
    B, C, f = oracle.did_run(X, B0, C0, 20, P=4, check=True)
    assert np.all(np.diff(f) <= 1e-12 * f[:-1])
    assert f[-1] < 0.1 * f[0]


def test_invariants_badly_scaled_start_with_clipping():
    rng = np.random.default_rng(3)
    X = rng.random((30, 40))
    B0, C0 = 3.0 * rng.random((30, 5)), 3.0 * rng.random((5, 40))  # E starts strictly negative
    B, C, f = oracle.did_run(X, B0, C0, 15, P=4, check=True)
    assert np.all(B >= 0) and np.all(C >= 0)


# ---------------------------------------------------------------- P6 K = 1 is power iteration
def test_rank_one_reaches_svd_optimum():
    rng = np.random.default_rng(7)
    X = 0.2 + rng.random((12, 20))
    B0, C0 = 0.5 + rng.random((12, 1)), 0.5 + rng.random((1, 20))
    B, C, f = oracle.did_run(X, B0, C0, 200, check=True)
    s = np.linalg.svd(X, compute_uv=False)
    assert f[-1] == pytest.approx(0.5 * (np.sum(X * X) - s[0] ** 2), rel=1e-9)
    assert np.all(B > 0) and np.all(C > 0)  # Perron-Frobenius: no clipping


# ---------------------------------------------------------------- P7 NNLS limits
def test_repeated_c_half_converges_to_columnwise_nnls():
    rng = np.random.default_rng(8)
    M, N, K = 10, 6, 4
    X = rng.random((M, N))
    B = rng.random((M, K))
    C = rng.random((K, N))
    E = oracle.residual(X, B, C)
    for _ in range(3000):
        oracle.c_half(B, C, E)
    for j in range(N):
        ref, _ = nnls(B, X[:, j])
        np.testing.assert_allclose(C[:, j], ref, rtol=1e-6, atol=1e-8)


def test_repeated_b_half_converges_to_rowwise_nnls():
    rng = np.random.default_rng(9)
    M, N, K = 6, 12, 4
    X = rng.random((M, N))
    B = rng.random((M, K))
    C = rng.random((K, N))
    blocks = oracle.column_blocks(N, 3)
    E = oracle.residual(X, B, C)
    for _ in range(3000):
        W, V = oracle.messages(E, C, blocks)
        dB = oracle.b_half(B, W, V)
        E -= dB @ C
    for m in range(M):
        ref, _ = nnls(C.T, X[m, :])
        np.testing.assert_allclose(B[m, :], ref, rtol=1e-6, atol=1e-8)


# ---------------------------------------------------------------- P8 X = 0
def test_zero_data_zeroes_c_and_keeps_b():
    """X = 0: every c-update is <= 0 in exact arithmetic, so C = 0, then v_ii = 0 for all i
    and the zero-denominator guard keeps B.  Small-integer factors keep every product and
    sum exact in FP64, so the exact-arithmetic result must come out exactly."""
    rng = np.random.default_rng(10)
    X = np.zeros((6, 9))
    B0 = rng.integers(0, 4, size=(6, 3)).astype(float) + np.eye(6, 3)
    C0 = rng.integers(0, 4, size=(3, 9)).astype(float)
    B, C, f = oracle.did_run(X, B0, C0, 1, check=True)
    assert np.all(C == 0.0)
    np.testing.assert_array_equal(B, B0)  # v_ii = 0 guard: B untouched
    assert f[1] == 0.0


def test_zero_data_generic_factors_to_rounding():
    rng = np.random.default_rng(10)
    X = np.zeros((6, 9))
    B0, C0 = rng.random((6, 3)), rng.random((3, 9))
    B = B0.copy()
    C = C0.copy()
    E = oracle.residual(X, B, C)
    oracle.c_half(B, C, E)
    assert np.max(C) <= 1e-14 and np.all(C >= 0)


def test_zero_column_of_b_is_skipped():
    rng = np.random.default_rng(12)
    X = rng.random((8, 10))
    B0, C0 = rng.random((8, 3)), rng.random((3, 10))
    B0[:, 1] = 0.0
    B, C, f = oracle.did_run(X, B0, C0, 1, check=True)
    np.testing.assert_array_equal(C[1], C0[1])  # coordinate with b_1^T b_1 = 0 untouched


# ---------------------------------------------------------------- P9 shard invariance
def test_shard_count_does_not_change_iterates():
    X, _, _ = planted_lowrank(M=40, N=640, K=5, seed=21)
    B0, C0 = uniform_init(40, 640, 5, seed=22)
    ref = oracle.did_run(X, B0, C0, 10, P=1)
    for P in (4, 64):
        B, C, f = oracle.did_run(X, B0, C0, 10, P=P)
        np.testing.assert_allclose(B, ref[0], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(C, ref[1], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(f, ref[2], rtol=1e-12)


def test_column_blocks_partition():
    for N, P in [(10, 3), (64, 64), (5, 9), (1_000_000, 64)]:
        bl = oracle.column_blocks(N, P)
        assert bl[0][0] == 0 and bl[-1][1] == N
        assert all(a < b for a, b in bl)
        assert all(bl[i][1] == bl[i + 1][0] for i in range(len(bl) - 1))


# ---------------------------------------------------------------- P10 planted product
def test_noiseless_plant_reaches_paper_tolerance():
    X, _, _ = planted_lowrank(M=60, N=200, K=4, seed=31)
    B0, C0 = uniform_init(60, 200, 4, seed=32)
    t, f = oracle.iterations_to_tolerance(X, B0, C0, eps=1e-6, max_iter=5000)
    assert f[-1] <= 1e-6 * f[0], (t, f[-1] / f[0])


def test_identifiable_plant_recovers_factors():
    X, B0, C0 = identifiable_plant(M=20, N=40, K=3, seed=41)
    Bi, Ci = uniform_init(20, 40, 3, seed=42)
    B, C, f = oracle.did_run(X, Bi, Ci, 4000)
    assert f[-1] <= 1e-10 * f[0]
    # match columns of B to B0 up to permutation and scaling (normalised cosine)
    Bn = B / np.linalg.norm(B, axis=0)
    B0n = B0 / np.linalg.norm(B0, axis=0)
    cos = np.abs(Bn.T @ B0n)
    assert np.all(np.max(cos, axis=0) > 1 - 1e-4)


# ---------------------------------------------------------------- P11 iteration-count parity
def test_iteration_count_matches_sequential_bcd():
    X, _, _ = planted_lowrank(M=6, N=8, K=2, seed=51)
    B0, C0 = uniform_init(6, 8, 2, seed=52)
    t_did, f_did = oracle.iterations_to_tolerance(X, B0, C0, eps=1e-6, max_iter=3000, P=4)
    _, _, f_bcd, t_bcd = bcd.naive_bcd_run(X, B0, C0, 3000, eps=1e-6)
    assert t_did == t_bcd
    np.testing.assert_allclose(f_did, f_bcd, rtol=1e-9, atol=1e-14)
