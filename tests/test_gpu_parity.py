"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same inputs.

Tolerances (FP32 engine vs FP64 oracle), normwise as the projection [z]_+ can flip at
z ~ 0 under a different summation order:
  factors after one iteration   ||B_gpu - B_or||_F / ||B_or||_F <= 1e-5, same for C;
  objective trajectory          max_t |f_gpu[t] - f_or[t]| / f_or[t] <= 1e-4;
  exact worked examples         1e-6 relative.
"""

from fractions import Fraction
import json
import os

import numpy as np
import pytest

import oracle
import paper_1802_08938_amd as did
from workloads import as_oracle_input, image_like, large_halfnormal, planted_lowrank, round_to_bf16, to_f32_colmajor

from _gpu import (announce, check_factors, check_trajectory, device_x, load_golden, read_factors, rel_fro,
                  require_gpu, run_gpu, worst_line)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")
TOL_FACTORS = 1e-5
TOL_OBJ = 1e-4
TOL_UNSTRUCTURED_CAP = 1e-3  # ceiling of the data-derived bar on ill-conditioned inputs


def _mat(rows):
    return np.array([[float(Fraction(v)) for v in r] for r in rows])


def _oracle_from(X32, B0, C0, T, P=1):
    return oracle.did_run(as_oracle_input(X32), B0, C0, T, P=P)


@pytest.mark.parametrize("name", ["k1", "k2_clipping"])
def test_worked_examples_on_gpu(name):
    torch = require_gpu()
    g = json.load(open(GOLDEN))[name]
    X, B0, C0 = _mat(g["X"]), _mat(g["B0"]), _mat(g["C0"])
    announce(f"worked example {name}")
    out = run_gpu(torch, to_f32_colmajor(X), B0.shape[1], iters=(1,), B0=B0, C0=C0)
    B1, C1 = out[1]
    np.testing.assert_allclose(C1, _mat(g["C1"]), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(B1, _mat(g["B1"]), rtol=1e-6, atol=1e-6)
    assert out["hist"][0] == pytest.approx(float(Fraction(g["f0"])), rel=1e-6)
    assert out["f"] == pytest.approx(float(Fraction(g["f1"])), rel=1e-6)


def test_planted_500x2000_k10_parity_50_iterations():
    torch = require_gpu()
    X, _, _ = planted_lowrank(500, 2000, 10, seed=1)
    X32 = to_f32_colmajor(X)
    announce("planted 500x2000 K=10, 50 iterations")
    out = run_gpu(torch, X32, 10, iters=(1, 50))
    B0, C0 = out["init"]
    B1o, C1o, _ = _oracle_from(X32, B0, C0, 1)
    check_factors(out[1][0], B1o, out[1][1], C1o, label="planted, 1 iteration")
    _, _, fo = _oracle_from(X32, B0, C0, 50)
    check_trajectory(np.append(out["hist"], out["f"]), fo, label="planted")
    assert np.all(out[50][0] >= 0) and np.all(out[50][1] >= 0)


def _golden_case(case):
    from tests.golden.make_trajectories import data, initial_factors

    g = load_golden(case)
    X32, Xo, K, P, T, bf16, _ = data(case)
    assert (g["M"], g["N"], g["K"], g["P"], g["T"]) == (X32.shape[0], X32.shape[1], K, P, T)
    if abs(float(np.sum(Xo)) - g["x_sum"]) > 1e-9 * abs(g["x_sum"]):
        print(f"[golden] {case}: data checksum differs from the golden's (host BLAS rounding); "
              "the trajectory bar still applies", flush=True)
    B0, C0 = initial_factors(X32.shape[0], X32.shape[1], K)
    return g, X32, Xo, K, P, T, bf16, B0, C0


def _sampled_golden_factors(g, out):
    """Sampled columns of C and rows of B after one iteration against the golden's."""
    cols, rows = g["sample_cols"], g["sample_rows"]
    C1o = np.array(g["C1_cols"]).T
    B1o = np.array(g["B1_rows"])
    check_factors(out[1][0][rows], B1o, out[1][1][:, cols], C1o, label=f"{g['case']}, sampled, 1 iteration")


@pytest.mark.parametrize("case,cw", [("image_like_p4", 4), ("image_like_p4", 8), ("large_slice_b1", 4),
                                     ("large_slice_b1", 8), ("large_slice_b4", 4)])
def test_named_workloads_parity_50_iterations(case, cw):
    """The image-like workload (784 x 70000, K = 16, 4 blocks) and slices of the large one
    (5000 x 15625 and 5000 x 62500, K = 50, 1 and 4 blocks) from the same initial factors as
    the oracle: factors after one iteration (all of them, or for the 4-block slice sampled
    columns and rows the oracle recorded) and the objective over 50 iterations, with both
    column-pass tiles (4 and 8 waves per block)."""
    torch = require_gpu()
    g, X32, Xo, K, P, T, _, B0, C0 = _golden_case(case)
    o = did.did_default_opts()
    o.n_blocks = P
    o.col_waves = cw
    announce(f"{case}: {X32.shape[0]}x{X32.shape[1]} K={K} P={P} col_waves={cw}, {T} iterations")
    out = run_gpu(torch, X32, K, iters=(1, T), opts=o, B0=B0.astype(np.float32), C0=C0.astype(np.float32))
    np.testing.assert_array_equal(out["init"][0], B0)
    if "sample_cols" in g:
        _sampled_golden_factors(g, out)
    else:
        B1o, C1o, _ = oracle.did_run(Xo, B0, C0, 1, P=P)
        check_factors(out[1][0], B1o, out[1][1], C1o, label=f"{case}, 1 iteration")
    check_trajectory(np.append(out["hist"], out["f"]), g["f"], label=case)


@pytest.mark.parametrize("M,N,K", [
    (37, 45, 3),     # ragged rows and columns, odd K
    (31, 33, 1),     # K = 1, below one tile in rows
    (100, 300, 32),  # K exactly one output tile
    (70, 129, 33),   # K just above one tile (padded to 64)
    (130, 260, 64),  # largest supported K
    (64, 200, 7),    # M % 4 == 0 (vector loads) with a tail tile of columns
    (5, 1000, 3),    # the experiments' shape, tiny M
])
def test_edge_shapes_parity(M, N, K):
    """Shapes that exercise ragged tiles and K padding, on planted low-rank data with
    half-normal noise (conditioned like the named workloads)."""
    torch = require_gpu()
    rng = np.random.default_rng(M * 7 + N + K)
    X = rng.random((M, K)) @ rng.random((K, N)) + np.abs(0.01 * rng.standard_normal((M, N)))
    X32 = to_f32_colmajor(X)
    announce(f"edge shape M={M} N={N} K={K}")
    out = run_gpu(torch, X32, K, iters=(1, 5))
    B0, C0 = out["init"]
    B1o, C1o, _ = _oracle_from(X32, B0, C0, 1)
    check_factors(out[1][0], B1o, out[1][1], C1o, label=f"edge {M}x{N} K={K}")
    _, _, fo = _oracle_from(X32, B0, C0, 5)
    check_trajectory(np.append(out["hist"], out["f"]), fo, label=f"edge {M}x{N} K={K}")


@pytest.mark.parametrize("M,N,K", [
    (40, 1, 1),     # a single column of X (one partial tile); an exact fit after one iteration
    (20, 20, 20),   # K = M = N
    (64, 100, 64),  # K = M at the largest supported K
    (100, 33, 33),  # K = N, just above one tile of columns
])
def test_degenerate_shapes_parity(M, N, K):
    """K as large as min(M, N) allows (the engine rejects more), on planted data.  Factors
    after one iteration to the usual bars; the objective to 1e-4 relative over 5
    iterations, plus, where the oracle fits X exactly (f -> 0), an absolute floor of
    M N (eps32 max|X|)^2: float32 rounding of the residual, which the oracle (float64)
    does not have."""
    torch = require_gpu()
    rng = np.random.default_rng(M * 7 + N + K)
    X = rng.random((M, K)) @ rng.random((K, N)) + np.abs(0.01 * rng.standard_normal((M, N)))
    X32 = to_f32_colmajor(X)
    announce(f"degenerate shape M={M} N={N} K={K}")
    out = run_gpu(torch, X32, K, iters=(1, 5))
    B0, C0 = out["init"]
    B1o, C1o, _ = _oracle_from(X32, B0, C0, 1)
    check_factors(out[1][0], B1o, out[1][1], C1o, label=f"degenerate {M}x{N} K={K}")
    _, _, fo = _oracle_from(X32, B0, C0, 5)
    fg = np.append(out["hist"], out["f"])
    floor = M * N * (np.finfo(np.float32).eps * float(np.max(X32))) ** 2
    excess = np.abs(fg - fo) - 1e-4 * fo
    print(f"[trajectory] degenerate {M}x{N} K={K}: f oracle {fo[-1]:.3e} gpu {fg[-1]:.3e}, "
          f"largest excess over 1e-4 relative {float(np.max(excess)):.2e} (floor {floor:.2e})", flush=True)
    assert np.all(excess <= floor), (fg, fo, floor)


def _fp32_sensitivity(X32, B0, C0, draws=3):
    """How far the oracle's one-iteration factors move when X is perturbed at the scale of
    float32 rounding of the residual, eps32 * max|B0 C0|: the floor any float32 engine
    faces on this input, whatever its summation order."""
    X = as_oracle_input(X32)
    B1, C1, _ = oracle.did_run(X, B0, C0, 1)
    scale = np.finfo(np.float32).eps * float(np.max(np.abs(B0 @ C0)))
    worst = 0.0
    for d in range(draws):
        r = np.random.default_rng(1000 + d)
        Bp, Cp, _ = oracle.did_run(X + scale * r.standard_normal(X.shape), B0, C0, 1)
        worst = max(worst, rel_fro(Bp, B1), rel_fro(Cp, C1))
    return worst


@pytest.mark.parametrize("M,N,K", [(100, 300, 32), (130, 260, 64), (70, 129, 33)])
def test_unstructured_data_within_fp32_conditioning(M, N, K):
    """Dense U[0,2] data with K close to M/3 is ill-conditioned for NMF: the tolerance is
    max(1e-5, 10 x the oracle's own movement under float32-sized perturbations of X), capped
    at 1e-3; the test prints the bar it used."""
    torch = require_gpu()
    rng = np.random.default_rng(M * 7 + N + K)
    X32 = to_f32_colmajor(rng.random((M, N)) * 2.0)
    announce(f"unstructured data M={M} N={N} K={K}")
    out = run_gpu(torch, X32, K, iters=(1,))
    B0, C0 = out["init"]
    sens = _fp32_sensitivity(X32, B0, C0)
    tol = min(TOL_UNSTRUCTURED_CAP, max(TOL_FACTORS, 10.0 * sens))
    B1o, C1o, _ = _oracle_from(X32, B0, C0, 1)
    eb, ec = rel_fro(out[1][0], B1o), rel_fro(out[1][1], C1o)
    print(f"[unstructured] {M}x{N} K={K}: oracle float32 sensitivity {sens:.2e}, bar {tol:.2e}, "
          f"B {eb:.2e} C {ec:.2e}", flush=True)
    assert eb <= tol and ec <= tol


def _badly_scaled(M, N, K, seed):
    """Planted X whose rows and columns span 1e-2 .. 1e2, and factors whose components are
    imbalanced by 1e3 each way between B and C (the same X, with very uneven factors);
    initial factors are the planted ones perturbed by up to 10 %."""
    r = np.random.default_rng(seed)
    rs = 10.0 ** r.uniform(-2, 2, M)
    cs = 10.0 ** r.uniform(-2, 2, N)
    comp = 10.0 ** np.linspace(-3, 3, K)
    Bp = (rs[:, None] * (0.2 + r.random((M, K)))) * comp[None, :]
    Cp = ((0.2 + r.random((K, N))) * cs[None, :]) / comp[:, None]
    X32 = to_f32_colmajor(Bp @ Cp)
    B0 = (Bp * (1 + 0.1 * r.random((M, K)))).astype(np.float32)
    C0 = (Cp * (1 + 0.1 * r.random((K, N)))).astype(np.float32)
    return X32, B0, C0


def _relative_sensitivity(X32, B0, C0, draws=3):
    """Movement of the oracle's one-iteration factors under elementwise relative
    perturbations of X, B0 and C0 at float32 rounding size: normwise for B and C, and for
    the worst single row of B and column of C."""
    X = as_oracle_input(X32)
    B1, C1, _ = oracle.did_run(X, B0, C0, 1)
    e = np.finfo(np.float32).eps
    worst = np.zeros(4)
    for d in range(draws):
        q = np.random.default_rng(100 + d)
        B2, C2, _ = oracle.did_run(X * (1 + e * q.standard_normal(X.shape)), B0 * (1 + e * q.standard_normal(B0.shape)),
                                   C0 * (1 + e * q.standard_normal(C0.shape)), 1)
        worst = np.maximum(worst, [rel_fro(B2, B1), rel_fro(C2, C1), _worst_row(B2, B1), _worst_row(C2.T, C1.T)])
    return worst


def _worst_row(a, b):
    nb = np.linalg.norm(b, axis=1)
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.where(nb > 0, nb, 1.0)))


@pytest.mark.parametrize("M,N,K,seed", [(150, 700, 6, 1), (130, 500, 40, 2)])
def test_badly_scaled_data_and_components(M, N, K, seed):
    """The MFMA products split each operand into two fp16 pieces under a power-of-two scale
    per row, column or chunk; rows and columns of very different magnitude, and components
    imbalanced by 1e6 between B and C, must keep float32 accuracy row by row and column by
    column, not only normwise.  Bars: max(1e-5, 10 x the oracle's own sensitivity)
    normwise and max(1e-4, 10 x sensitivity) per row of B and column of C."""
    torch = require_gpu()
    X32, B0, C0 = _badly_scaled(M, N, K, seed)
    announce(f"badly scaled data M={M} N={N} K={K}")
    out = run_gpu(torch, X32, K, iters=(1,), B0=B0, C0=C0)
    Bi, Ci = out["init"]
    sens = _relative_sensitivity(X32, Bi, Ci)
    B1o, C1o, _ = _oracle_from(X32, Bi, Ci, 1)
    B1, C1 = out[1]
    assert rel_fro(B1, B1o) <= max(TOL_FACTORS, 10 * sens[0])
    assert rel_fro(C1, C1o) <= max(TOL_FACTORS, 10 * sens[1])
    assert _worst_row(B1, B1o) <= max(1e-4, 10 * sens[2])
    assert _worst_row(C1.T, C1o.T) <= max(1e-4, 10 * sens[3])


def test_zero_data_and_guard_on_gpu():
    """X = 0 with small-integer factors: C becomes exactly 0, every v_ii = 0 keeps B."""
    torch = require_gpu()
    rng = np.random.default_rng(10)
    M, N, K = 40, 50, 3
    B0 = rng.integers(0, 4, size=(M, K)).astype(float) + np.eye(M, K)
    C0 = rng.integers(0, 4, size=(K, N)).astype(float)
    announce("zero data")
    out = run_gpu(torch, to_f32_colmajor(np.zeros((M, N))), K, iters=(1,), B0=B0, C0=C0)
    B1, C1 = out[1]
    assert np.all(C1 == 0.0)
    np.testing.assert_array_equal(B1, B0)
    assert out["f"] == 0.0


def test_zero_column_of_b_is_skipped_on_gpu():
    torch = require_gpu()
    rng = np.random.default_rng(12)
    M, N, K = 48, 70, 4
    X32 = to_f32_colmajor(rng.random((M, N)))
    B0, C0 = rng.random((M, K)), rng.random((K, N))
    B0[:, 2] = 0.0
    announce("zero column of B")
    out = run_gpu(torch, X32, K, iters=(1,), B0=B0.astype(np.float32), C0=C0.astype(np.float32))
    np.testing.assert_array_equal(out[1][1][2], C0.astype(np.float32)[2].astype(np.float64))
    B1o, C1o, _ = _oracle_from(X32, out["init"][0], out["init"][1], 1)
    check_factors(out[1][0], B1o, out[1][1], C1o, label="zero column of B")


@pytest.mark.parametrize("K", [8, 9, 16, 17, 24, 25, 40, 41, 48, 49, 56, 57])
def test_every_k_class_parity(K):
    """K on both sides of each multiple of 8: the B update's coordinate loops are bounded by K
    rounded up to a multiple of 8 (a compile-time bound chosen per call), so each class runs
    its own code; every one matches the oracle."""
    torch = require_gpu()
    M, N = 90, 200
    rng = np.random.default_rng(500 + K)
    X = rng.random((M, K)) @ rng.random((K, N)) + np.abs(0.01 * rng.standard_normal((M, N)))
    X32 = to_f32_colmajor(X)
    announce(f"K class: M={M} N={N} K={K}")
    out = run_gpu(torch, X32, K, iters=(1, 3))
    B0, C0 = out["init"]
    B1o, C1o, _ = _oracle_from(X32, B0, C0, 1)
    check_factors(out[1][0], B1o, out[1][1], C1o, label=f"K={K}, 1 iteration")
    B3o, C3o, fo = _oracle_from(X32, B0, C0, 3)
    check_factors(out[3][0], B3o, out[3][1], C3o, tol=1e-4, tol_line=1e-3, label=f"K={K}, 3 iterations")
    check_trajectory(np.append(out["hist"], out["f"]), fo, label=f"K={K}")


@pytest.mark.parametrize("K", [4, 40])
def test_zero_row_of_c_keeps_b_column_mid_order(K):
    """A zero column of B and the matching zero row of C at coordinate 2: the sweep skips
    c_2 (n_2 = 0) and the B update skips b_2 (v_22 = 0) while the coordinates after it
    still move; B's column 2 and C's row 2 stay zero and the rest matches the oracle."""
    torch = require_gpu()
    rng = np.random.default_rng(14 + K)
    M, N = 60, 90
    X32 = to_f32_colmajor(rng.random((M, K)) @ rng.random((K, N)))
    B0, C0 = rng.random((M, K)), rng.random((K, N))
    B0[:, 2] = 0.0
    C0[2, :] = 0.0
    announce(f"zero row of C, K={K}")
    out = run_gpu(torch, X32, K, iters=(1, 2), B0=B0.astype(np.float32), C0=C0.astype(np.float32))
    for t in (1, 2):
        assert np.all(out[t][0][:, 2] == 0.0) and np.all(out[t][1][2] == 0.0)
    B2o, C2o, fo = _oracle_from(X32, out["init"][0], out["init"][1], 2)
    check_factors(out[2][0], B2o, out[2][1], C2o, label=f"zero row of C, K={K}")
    check_trajectory(np.append(out["hist"], out["f"]), fo, label=f"zero row of C, K={K}")


def test_rejects_negative_and_nonfinite_x():
    torch = require_gpu()
    for bad in (-1.0, np.nan, np.inf):
        X = np.ones((40, 40), dtype=np.float32)
        X[3, 7] = bad
        announce(f"invalid X entry {bad}")
        with pytest.raises(did.DidError) as ei:
            did.did_init(device_x(torch, X), 40, 40, 2, 1)
        assert ei.value.code == did.DID_EINVAL


@pytest.mark.parametrize("storage", ["f32", "f32-tiled", "bf16"])
def test_host_pointer_x_matches_device_pointer(storage):
    """X in host memory is uploaded (and, for the tiled storages, tiled from a temporary
    upload); the iterates equal those from the same X on the device."""
    torch = require_gpu()
    rng = np.random.default_rng(4)
    X32 = to_f32_colmajor(rng.random((64, 96)))
    o = did.did_default_opts()
    o.x_tiled = 1 if storage == "f32-tiled" else 0
    o.x_dtype = did.DID_BF16 if storage == "bf16" else did.DID_F32
    announce(f"host vs device X ({storage})")
    hd = did.did_init_ex(device_x(torch, X32), 64, 96, 5, 7, o)
    Xh = np.ascontiguousarray(X32.T)  # host memory, column-major X
    hh = did.did_init_ex(Xh, 64, 96, 5, 7, o)
    try:
        did.did_iterate(hd, 3)
        did.did_iterate(hh, 3)
        a = read_factors(hd, 64, 96, 5)
        b = read_factors(hh, 64, 96, 5)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
    finally:
        did.did_free(hd)
        did.did_free(hh)


def test_deterministic_bitwise():
    torch = require_gpu()
    X, _, _ = planted_lowrank(300, 5000, 12, seed=9)
    X32 = to_f32_colmajor(X)
    announce("determinism")
    a = run_gpu(torch, X32, 12, iters=(7,))
    b = run_gpu(torch, X32, 12, iters=(7,))
    np.testing.assert_array_equal(a[7][0], b[7][0])
    np.testing.assert_array_equal(a[7][1], b[7][1])
    np.testing.assert_array_equal(a["hist"], b["hist"])


@pytest.mark.parametrize("M,N,K,storage", [(300, 1000, 10, "f32"), (130, 777, 40, "tiled"), (97, 1234, 64, "bf16"),
                                            (64, 200, 7, "f32"), (40, 300, 33, "f32")])
def test_column_tile_choice_keeps_factors_bitwise(M, N, K, storage):
    """Each wave of the column pass owns one 32-column tile whatever the block size, so
    B, C (and H) are the same bit for bit with 4 or 8 waves per block; only the objective's
    summation order changes (ragged N: 1000, 777, 1234, 200 and 300 columns are not
    multiples of 256)."""
    torch = require_gpu()
    X, _, _ = planted_lowrank(M, N, K, seed=21)
    X32 = to_f32_colmajor(X)
    res = []
    for cw in (4, 8):
        o = did.did_default_opts()
        o.x_dtype = did.DID_BF16 if storage == "bf16" else did.DID_F32
        o.x_tiled = 1 if storage == "tiled" else 0
        o.col_waves = cw
        announce(f"{M}x{N} K={K} {storage} col_waves={cw}")
        res.append(run_gpu(torch, X32, K, iters=(1, 6), opts=o))
    for t in (1, 6):
        np.testing.assert_array_equal(res[0][t][0], res[1][t][0])
        np.testing.assert_array_equal(res[0][t][1], res[1][t][1])
    np.testing.assert_allclose(res[1]["hist"], res[0]["hist"], rtol=1e-12)
    assert res[1]["f"] == pytest.approx(res[0]["f"], rel=1e-12)


@pytest.mark.parametrize("spread", [3.0, 10.0, 1e3])
def test_shared_scale_groups_parity(spread):
    """Rows of B and columns of C whose magnitudes vary by a factor `spread` inside each
    32-row chunk / 32-column tile: within a factor 4 they share one fp16 scale per group
    (one multiplier per tile in the passes), beyond it each keeps its own.  Both ways the
    factors after one and five iterations match the oracle, normwise and line by line."""
    torch = require_gpu()
    M, N, K = 200, 1500, 12
    rng = np.random.default_rng(int(spread) + 5)
    rs = spread ** (np.arange(M) % 2)           # alternate rows 1 and `spread` within chunks
    cs = spread ** ((np.arange(N) // 3) % 2)    # runs of three columns at 1 and `spread`
    B0p = rs[:, None] * (0.2 + rng.random((M, K)))
    C0p = (0.2 + rng.random((K, N))) * cs[None, :]
    X32 = to_f32_colmajor(B0p @ C0p + np.abs(0.01 * rng.standard_normal((M, N))))
    B0 = (B0p * (1 + 0.1 * rng.random((M, K)))).astype(np.float32)
    C0 = (C0p * (1 + 0.1 * rng.random((K, N)))).astype(np.float32)
    announce(f"shared scale groups, spread {spread}")
    out = run_gpu(torch, X32, K, iters=(1, 5), B0=B0, C0=C0)
    Bi, Ci = out["init"]
    B1o, C1o, _ = _oracle_from(X32, Bi, Ci, 1)
    check_factors(out[1][0], B1o, out[1][1], C1o, label=f"spread {spread}, 1 iteration")
    B5o, C5o, fo = _oracle_from(X32, Bi, Ci, 5)
    check_factors(out[5][0], B5o, out[5][1], C5o, tol=1e-4, tol_line=1e-3, label=f"spread {spread}, 5 iterations")
    check_trajectory(np.append(out["hist"], out["f"]), fo, label=f"spread {spread}")


def test_block_count_only_changes_rounding():
    torch = require_gpu()
    X, _, _ = planted_lowrank(200, 6400, 8, seed=13)
    X32 = to_f32_colmajor(X)
    res = []
    for P in (1, 4, 64):
        o = did.did_default_opts()
        o.n_blocks = P
        announce(f"n_blocks={P}")
        res.append(run_gpu(torch, X32, 8, iters=(5,), opts=o))
    for r in res[1:]:
        assert rel_fro(r[5][0], res[0][5][0]) <= 1e-5
        assert rel_fro(r[5][1], res[0][5][1]) <= 1e-5


@pytest.mark.parametrize("tiled", [0, 1])
def test_resume_from_factors_equals_uninterrupted(tiled):
    torch = require_gpu()
    X, _, _ = planted_lowrank(150, 900, 6, seed=17)
    X32 = to_f32_colmajor(X)
    announce(f"resume (x_tiled={tiled})")
    o = did.did_default_opts()
    o.x_tiled = tiled
    full = run_gpu(torch, X32, 6, iters=(4, 8), opts=o)
    B4, C4 = full[4]
    resumed = run_gpu(torch, X32, 6, iters=(4,), opts=o, B0=B4.astype(np.float32), C0=C4.astype(np.float32))
    np.testing.assert_array_equal(resumed[4][0], full[8][0])
    np.testing.assert_array_equal(resumed[4][1], full[8][1])


def test_init_scale_minimises_common_scale():
    torch = require_gpu()
    X, _, _ = image_like(100, 700, 5, seed=3)
    X32 = to_f32_colmajor(X)
    announce("init_scale")
    o = did.did_default_opts()
    o.init_scale = 1
    sc = run_gpu(torch, X32, 5, iters=(0,), opts=o)
    un = run_gpu(torch, X32, 5, iters=(0,))
    Bs, Cs = sc["init"]
    Bu, Cu = un["init"]
    Xo = as_oracle_input(X32)
    P = Bu @ Cu
    alpha = float(np.sum(Xo * P) / np.sum(P * P))
    np.testing.assert_allclose(Bs @ Cs, alpha * P, rtol=1e-4)
    assert sc["f"] < un["f"]


@pytest.mark.parametrize("M,N,K", [(500, 2000, 10), (130, 260, 64), (37, 45, 3)])
def test_bf16_storage_form_matches_oracle_on_rounded_x(M, N, K):
    """x_dtype = DID_BF16: the engine solves the problem for bf16(X) with float32-accurate
    arithmetic, so it meets the float32 tolerances against the oracle run on bf16(X)."""
    torch = require_gpu()
    rng = np.random.default_rng(M + N + K)
    X = rng.random((M, K)) @ rng.random((K, N)) + np.abs(0.01 * rng.standard_normal((M, N)))
    X32 = to_f32_colmajor(X)
    Xr = round_to_bf16(X32)
    o = did.did_default_opts()
    o.x_dtype = did.DID_BF16
    announce(f"bf16 storage M={M} N={N} K={K}")
    out = run_gpu(torch, X32, K, iters=(1, 10), opts=o)
    B0, C0 = out["init"]
    B1o, C1o, _ = oracle.did_run(Xr, B0, C0, 1)
    check_factors(out[1][0], B1o, out[1][1], C1o, label=f"bf16 {M}x{N} K={K}")
    _, _, fo = oracle.did_run(Xr, B0, C0, 10)
    check_trajectory(np.append(out["hist"], out["f"]), fo, label=f"bf16 {M}x{N} K={K}")


@pytest.mark.parametrize("M,N,K", [(500, 2000, 10), (130, 777, 64), (97, 1234, 33), (64, 4001, 7)])
def test_bf16_storage_equals_float32_form_on_rounded_x_bitwise(M, N, K):
    """The bf16 form reads X from two tiled copies (one per pass) and the float32 form
    reads the column-major X, but both feed the same values to the same arithmetic: run
    on X and on bf16(X) respectively, their iterates agree bit for bit.  Ragged M and N
    (zero padding of the tiles) and a column-pass wave past the last tile (N = 777, 4001)
    are covered."""
    torch = require_gpu()
    rng = np.random.default_rng(7 * M + N + K)
    X32 = to_f32_colmajor(rng.random((M, K)) @ rng.random((K, N)) + np.abs(0.01 * rng.standard_normal((M, N))))
    Xr = to_f32_colmajor(round_to_bf16(X32))
    ob = did.did_default_opts()
    ob.x_dtype = did.DID_BF16
    announce(f"bf16 tiled vs float32 on rounded X, M={M} N={N} K={K}")
    a = run_gpu(torch, X32, K, iters=(1, 6), opts=ob)
    b = run_gpu(torch, Xr, K, iters=(1, 6), opts=did.did_default_opts())
    for n in (1, 6):
        np.testing.assert_array_equal(a[n][0], b[n][0])
        np.testing.assert_array_equal(a[n][1], b[n][1])
    np.testing.assert_array_equal(a["hist"], b["hist"])
    assert a["f"] == b["f"]


@pytest.mark.parametrize("M,N,K", [(500, 2000, 10), (130, 777, 64), (97, 1234, 33), (5000, 3001, 50)])
def test_tiled_float32_x_equals_column_major_bitwise(M, N, K):
    """x_tiled = 1 keeps X as two float32 copies in tile order; the passes load the same
    values, so the iterates equal those of the column-major form bit for bit."""
    torch = require_gpu()
    rng = np.random.default_rng(3 * M + N + K)
    X32 = to_f32_colmajor(rng.random((M, K)) @ rng.random((K, N)) + np.abs(0.01 * rng.standard_normal((M, N))))
    ot = did.did_default_opts()
    ot.x_tiled = 1
    announce(f"tiled float32 X vs column-major, M={M} N={N} K={K}")
    a = run_gpu(torch, X32, K, iters=(1, 6), opts=ot)
    b = run_gpu(torch, X32, K, iters=(1, 6), opts=did.did_default_opts())
    for n in (1, 6):
        np.testing.assert_array_equal(a[n][0], b[n][0])
        np.testing.assert_array_equal(a[n][1], b[n][1])
    np.testing.assert_array_equal(a["hist"], b["hist"])
    assert a["f"] == b["f"]


def test_tiled_x_rejected_on_thin_shapes_and_bad_values():
    torch = require_gpu()
    announce("x_tiled rejections")
    ot = did.did_default_opts()
    ot.x_tiled = 1
    Xt = torch.rand((1000, 5), device="cuda")
    torch.cuda.synchronize()
    with pytest.raises(did.DidError) as ei:
        did.did_init_ex(Xt, 5, 1000, 3, 1, ot)
    assert ei.value.code == did.DID_EINVAL
    ot.x_tiled = 2
    X = torch.rand((1000, 100), device="cuda")
    torch.cuda.synchronize()
    with pytest.raises(did.DidError) as ei:
        did.did_init_ex(X, 100, 1000, 8, 1, ot)
    assert ei.value.code == did.DID_EINVAL


def test_bf16_storage_rejects_bad_x_and_borrow_is_ignored():
    torch = require_gpu()
    X = np.ones((40, 40), dtype=np.float32)
    X[1, 1] = -2.0
    o = did.did_default_opts()
    o.x_dtype = did.DID_BF16
    o.borrow_x = 1
    announce("bf16 storage invalid X")
    with pytest.raises(did.DidError) as ei:
        did.did_init_ex(device_x(torch, X), 40, 40, 2, 1, o)
    assert ei.value.code == did.DID_EINVAL
    X[1, 1] = 2.0
    Xd = device_x(torch, X)
    h = did.did_init_ex(Xd, 40, 40, 2, 1, o)
    try:
        Xd.zero_()  # the engine holds its own bf16 copy: changing the caller's X has no effect
        did.did_iterate(h, 2)
        assert did.did_objective(h) > 0.0
    finally:
        did.did_free(h)


@pytest.mark.parametrize("M,N,K", [(5, 4000, 3), (16, 700, 4), (8, 700, 8), (7, 333, 5), (1, 100, 1), (8, 257, 4),
                                   (5, 100_003, 3), (16, 700, 8)])
def test_thin_path_parity(M, N, K):
    """M <= 16, K <= 8 (M <= 8 or K <= 4) runs the fused single-pass thin-matrix path;
    (16, 700, 8) lies just outside it and runs the MFMA passes."""
    torch = require_gpu()
    rng = np.random.default_rng(M * 31 + N + K)
    X = rng.random((M, K)) @ rng.random((K, N)) + np.abs(0.01 * rng.standard_normal((M, N)))
    X32 = to_f32_colmajor(X)
    announce(f"thin path M={M} N={N} K={K}")
    out = run_gpu(torch, X32, K, iters=(1, 20))
    B0, C0 = out["init"]
    B1o, C1o, _ = _oracle_from(X32, B0, C0, 1)
    check_factors(out[1][0], B1o, out[1][1], C1o, label=f"thin {M}x{N} K={K}")
    _, _, fo = _oracle_from(X32, B0, C0, 20)
    fg = np.append(out["hist"], out["f"])
    # M = 1, K = 1 factors exactly, so f falls to its float32 rounding floor (about
    # 1e-14 f^0); relative error is measured against max(f, 1e-8 f^0).
    assert np.max(np.abs(fg - fo) / np.maximum(fo, 1e-8 * fo[0])) <= TOL_OBJ


@pytest.mark.parametrize("M,N,K", [(5, 3000, 3), (12, 2000, 4)])
def test_dbcd_ablation_follows_the_same_iterates(M, N, K):
    """Alg. 2 (DBCD, K reductions per iteration) and Alg. 3 (DID, one) give the same
    iterates; the GPU's DBCD also matches the oracle's DBCD."""
    from oracle import bcd

    torch = require_gpu()
    rng = np.random.default_rng(77)
    X = rng.random((M, K)) @ rng.random((K, N))
    X32 = to_f32_colmajor(X)
    o = did.did_default_opts()
    o.algorithm = did.DID_ALG_DBCD
    announce(f"DBCD vs DID M={M} N={N} K={K}")
    dbcd_run = run_gpu(torch, X32, K, iters=(1, 10), opts=o)
    did_run = run_gpu(torch, X32, K, iters=(1, 10))
    for n in (1, 10):
        assert rel_fro(dbcd_run[n][0], did_run[n][0]) <= TOL_FACTORS
        assert rel_fro(dbcd_run[n][1], did_run[n][1]) <= TOL_FACTORS
    B0, C0 = dbcd_run["init"]
    Bo, Co = B0.copy(), C0.copy()
    Xo = as_oracle_input(X32)
    for _ in range(10):
        bcd.dbcd_iteration(Xo, Bo, Co, oracle.column_blocks(N, 4))
    assert rel_fro(dbcd_run[10][0], Bo) <= 1e-4
    assert rel_fro(dbcd_run[10][1], Co) <= 1e-4


def test_dbcd_needs_the_thin_path():
    torch = require_gpu()
    o = did.did_default_opts()
    o.algorithm = did.DID_ALG_DBCD
    X = np.ones((40, 50), dtype=np.float32)
    announce("DBCD on a wide shape")
    with pytest.raises(did.DidError) as ei:
        did.did_init_ex(device_x(torch, X), 40, 50, 3, 1, o)
    assert ei.value.code == did.DID_EINVAL


def test_stopping_rule_iteration_count_matches_oracle():
    """The experiments' stopping rule ||E^t||^2 <= 1e-6 ||E^0||^2 on the experiments' shape
    (M = 5, K = 3): the GPU stops at the oracle's iteration (within one, for float32
    rounding at the threshold), and DID and DBCD stop together (the paper's Correctness
    paragraph)."""
    from workloads import paper_synthetic

    torch = require_gpu()
    X, _, _ = paper_synthetic(20000, seed=4)
    X32 = to_f32_colmajor(X)

    def gpu_count(alg):
        o = did.did_default_opts()
        o.algorithm = alg
        h = did.did_init_ex(device_x(torch, X32), 5, 20000, 3, 2024, o)
        try:
            Bt = np.empty((3, 5), np.float32)
            Ct = np.empty((20000, 3), np.float32)
            did.did_factors(h, Bt, Ct)
            did.did_iterate(h, 3000)
            f = np.append(did.did_history(h), did.did_objective(h))
        finally:
            did.did_free(h)
        hit = np.nonzero(f <= 1e-6 * f[0])[0]
        return (int(hit[0]) if hit.size else None), Bt.T.astype(np.float64), Ct.T.astype(np.float64)

    announce("stopping rule on the experiments' shape")
    t_did, B0, C0 = gpu_count(did.DID_ALG_DID)
    t_dbcd, _, _ = gpu_count(did.DID_ALG_DBCD)
    t_or, _ = oracle.iterations_to_tolerance(as_oracle_input(X32), B0, C0, eps=1e-6, max_iter=3000)
    assert t_did is not None and t_dbcd is not None
    assert abs(t_did - t_dbcd) <= 1
    assert abs(t_did - t_or) <= 1, (t_did, t_or)


def test_injected_fault_is_sticky():
    """A faked device error (host-side flag, no device fault) makes the handle
    sticky-failed: every later call returns DID_EDEVICE and did_free still releases it."""
    torch = require_gpu()
    rng = np.random.default_rng(21)
    X32 = to_f32_colmajor(rng.random((64, 200)))
    announce("injected sticky fault")
    h = did.did_init(device_x(torch, X32), 64, 200, 4, 3)
    try:
        did.did_iterate(h, 1)
        did.did_debug_inject_fault(h)
        with pytest.raises(did.DidError) as ei:
            did.did_iterate(h, 1)
        assert ei.value.code == did.DID_EDEVICE and "injected" in str(ei.value)
        for call in (lambda: did.did_iterate(h, 1), lambda: did.did_objective(h), lambda: read_factors(h, 64, 200, 4),
                     lambda: did.did_history(h), lambda: did.did_sync(h), lambda: did.did_iterations(h)):
            with pytest.raises(did.DidError) as ei:
                call()
            assert ei.value.code == did.DID_EDEVICE
    finally:
        did.did_free(h)



# ---------------------------------------------------------------- carried residual (a7)
# refresh_every = r > 1 keeps R = X - BC resident and carries it (the C sweep's
# r_j -= b_i delta c_ij and E := E - delta b_i c_i^r of Section 4), refreshing it from X
# every r-th iteration.  In exact arithmetic the iterates are those of Alg. 3, so the
# oracle (which carries its own float64 residual) is the reference at the same bars.

@pytest.mark.parametrize("M,N,K,storage,r", [(300, 2000, 10, "f32", 3), (130, 777, 64, "f32", 10),
                                             (97, 1234, 33, "bf16", 10), (200, 3001, 20, "f32-tiled", 4),
                                             (37, 45, 3, "f32", 2)])
def test_carried_residual_matches_oracle(M, N, K, storage, r):
    torch = require_gpu()
    rng = np.random.default_rng(11 * M + N + K)
    X32 = to_f32_colmajor(rng.random((M, K)) @ rng.random((K, N)) + np.abs(0.01 * rng.standard_normal((M, N))))
    Xo = round_to_bf16(X32) if storage == "bf16" else as_oracle_input(X32)
    o = did.did_default_opts()
    o.refresh_every = r
    o.x_dtype = did.DID_BF16 if storage == "bf16" else did.DID_F32
    o.x_tiled = 1 if storage == "f32-tiled" else 0
    T = 3 * r + 2  # several refresh cycles and carried stretches
    announce(f"carried residual {M}x{N} K={K} {storage} refresh_every={r}, {T} iterations")
    out = run_gpu(torch, X32, K, iters=(1, T), opts=o)
    B0, C0 = out["init"]
    B1o, C1o, _ = oracle.did_run(Xo, B0, C0, 1)
    check_factors(out[1][0], B1o, out[1][1], C1o, label=f"carried r={r} {M}x{N} K={K}, 1 iteration")
    BTo, CTo, fo = oracle.did_run(Xo, B0, C0, T)
    check_trajectory(np.append(out["hist"], out["f"]), fo, label=f"carried r={r} {M}x{N} K={K}")
    check_factors(out[T][0], BTo, out[T][1], CTo, tol=1e-4, tol_line=1e-3,
                  label=f"carried r={r} {M}x{N} K={K}, {T} iterations")


@pytest.mark.parametrize("r", [1, 10])
def test_bf16_large_slice_refresh_every_parity_50_iterations(r):
    """The precision form on the large workload's first column block (5000 x 15625, K = 50,
    X stored as bf16), refreshing the residual every iteration or carrying it with a
    refresh every 10 iterations: the objective over 50 iterations against the oracle run
    on bf16(X) (which carries its float64 residual throughout)."""
    torch = require_gpu()
    g, X32, Xo, K, P, T, bf16, B0, C0 = _golden_case("large_slice_b1_bf16")
    assert bf16
    o = did.did_default_opts()
    o.x_dtype = did.DID_BF16
    o.refresh_every = r
    announce(f"bf16 large slice, refresh_every={r}, {T} iterations")
    out = run_gpu(torch, X32, K, iters=(T,), opts=o, B0=B0.astype(np.float32), C0=C0.astype(np.float32))
    check_trajectory(np.append(out["hist"], out["f"]), g["f"], label=f"bf16 slice refresh_every={r}")


def test_carried_residual_rejections():
    torch = require_gpu()
    announce("carried residual rejections")
    X = device_x(torch, np.ones((5, 300), np.float32))
    o = did.did_default_opts()
    o.refresh_every = 2
    with pytest.raises(did.DidError) as ei:  # thin-matrix shape
        did.did_init_ex(X, 5, 300, 3, 1, o)
    assert ei.value.code == did.DID_EINVAL
    o.refresh_every = 0
    X2 = device_x(torch, np.ones((64, 300), np.float32))
    with pytest.raises(did.DidError) as ei:
        did.did_init_ex(X2, 64, 300, 3, 1, o)
    assert ei.value.code == did.DID_EINVAL


def test_graph_replays_equal_eager_iterations():
    """did_iterate(h, n >= 2) replays one captured iteration (a hipGraph); did_iterate(h, 1)
    launches the kernels directly.  With eager work and synchronisations between the
    replays (objective passes, factor reads), every replay's result equals the eager one
    bit for bit."""
    torch = require_gpu()
    rng = np.random.default_rng(23)
    M, N, K = 300, 2500, 24
    X32 = to_f32_colmajor(rng.random((M, K)) @ rng.random((K, N)) + np.abs(0.01 * rng.standard_normal((M, N))))
    announce("graph replays vs eager iterations")
    Xd = device_x(torch, X32)
    he = did.did_init(Xd, M, N, K, 99)
    hg = did.did_init(Xd, M, N, K, 99)
    try:
        for step in range(4):
            for _ in range(3):
                did.did_iterate(he, 1)
            did.did_iterate(hg, 3)
            fe, fg = did.did_objective(he), did.did_objective(hg)
            a, b = read_factors(he, M, N, K), read_factors(hg, M, N, K)
            np.testing.assert_array_equal(a[0], b[0])
            np.testing.assert_array_equal(a[1], b[1])
            assert fe == fg
        np.testing.assert_array_equal(np.array(did.did_history(he)), np.array(did.did_history(hg)))
        assert did.did_iterations(hg) == 12
    finally:
        did.did_free(he)
        did.did_free(hg)
