"""The allocation-free entry point did_iterate_static against did_init_from_factors +
did_iterate on the same inputs: the same kernels and the same column ranges, so B, C and
the objective history must agree bit for bit.  Two calls in a row share the library's
static workspace, the second with a smaller instance (its leftovers must not leak into the
second result); the first is also checked against the FP64 oracle after one iteration."""

import numpy as np
import pytest

import oracle
import paper_1802_08938_amd as did
from tests._gpu import announce, read_factors, rel_fro, require_gpu
from workloads import as_oracle_input, serving_x, to_f32_colmajor, uniform_init

pytestmark = pytest.mark.gpu


def _dev(torch, a):
    """Column-major float32 (rows x cols) array as a device tensor of its transpose."""
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32).T)).to("cuda")
    torch.cuda.synchronize()
    return t


def _case(torch, M, N, K, n, n_blocks, seed, col_waves=0):
    X32 = to_f32_colmajor(serving_x(M, N, K, seed=seed))
    B0, C0 = uniform_init(M, N, K, seed + 1)
    B0 = B0.astype(np.float32)
    C0 = C0.astype(np.float32)
    Xd = _dev(torch, X32)
    o = did.did_default_opts()
    o.n_blocks = n_blocks
    o.col_waves = col_waves
    # the existing entry points
    h = did.did_init_from_factors(Xd, M, N, K, _dev(torch, B0), _dev(torch, C0), o)
    try:
        did.did_iterate(h, n)
        Bref, Cref = read_factors(h, M, N, K)
        href = np.array(did.did_history(h))
    finally:
        did.did_free(h)
    # the allocation-free entry point on the null stream (torch's current stream)
    Bd, Cd = _dev(torch, B0), _dev(torch, C0)
    fd = torch.zeros(n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    did.did_iterate_static(Xd, M, N, K, Bd, Cd, n, o, fd)
    torch.cuda.synchronize()
    Bs = Bd.cpu().numpy().T.astype(np.float64)
    Cs = Cd.cpu().numpy().T.astype(np.float64)
    fs = fd.cpu().numpy()
    return X32, B0, C0, (Bref, Cref, href), (Bs, Cs, fs)


def test_static_entry_equals_allocating_path_twice():
    torch = require_gpu()
    # second call: smaller; third: the column pass with 8 waves per block
    cases = [(600, 9000, 40, 6, 4, 31, 0), (300, 2500, 12, 4, 0, 32, 0), (500, 3000, 20, 3, 0, 33, 8)]
    for i, (M, N, K, n, P, seed, cw) in enumerate(cases):
        announce(f"did_iterate_static call {i + 1}: M={M} N={N} K={K} n={n} col_waves={cw}")
        X32, B0, C0, ref, got = _case(torch, M, N, K, n, P, seed, cw)
        np.testing.assert_array_equal(got[0], ref[0])
        np.testing.assert_array_equal(got[1], ref[1])
        np.testing.assert_array_equal(got[2], ref[2])
        if i == 0:  # and against the oracle: one iteration from the same factors
            _, _, ref1, got1 = _case(torch, M, N, K, 1, P, seed)[1:]
            Bo, Co, fo = oracle.did_run(as_oracle_input(X32), B0.astype(np.float64), C0.astype(np.float64), 1, P=max(P, 1))
            assert rel_fro(got1[0], Bo) <= 1e-5 and rel_fro(got1[1], Co) <= 1e-5
            assert abs(got1[2][0] - fo[0]) <= 1e-6 * fo[0]


def test_static_entry_rejections():
    torch = require_gpu()
    announce("did_iterate_static rejections")
    X = torch.ones((100, 5), device="cuda")
    B = torch.ones((3, 5), device="cuda")
    C = torch.ones((100, 3), device="cuda")
    torch.cuda.synchronize()
    with pytest.raises(did.DidError) as ei:  # thin-matrix shape
        did.did_iterate_static(X, 5, 100, 3, B, C, 1)
    assert ei.value.code == did.DID_EINVAL
    M, N, K = 4000, 400_000, 64  # needs more than the static workspace: refused before any work
    with pytest.raises(did.DidError) as ei:
        did.did_iterate_static(X, M, N, K, B, C, 1)
    assert ei.value.code == did.DID_EINVAL and "workspace" in str(ei.value)
    o = did.did_default_opts()
    o.x_tiled = 1
    with pytest.raises(did.DidError) as ei:
        did.did_iterate_static(X, 100, 100, 8, B, C, 1, o)
    assert ei.value.code == did.DID_EINVAL
