"""Guard zones: every path writes only inside its own buffers.

A handle made with DID_DEBUG_GUARD_ZONES=1 carves a patterned zone after each of its device
buffers (they all come from one allocation, back to back), and did_debug_check_guards
counts the zone bytes that changed.  Each case below runs one path of the engine (eager and
replayed iterations, the tiled and bf16 storage forms, the carried residual, the thin-path
instances, the DBCD ablation, resumed factors, per-stage profiling, the batched form) and
checks that no buffer was written past its end."""

import os

import numpy as np
import pytest

import paper_1802_08938_amd as did
from _gpu import announce, device_x, require_gpu
from workloads import serving_x, to_f32_colmajor

pytestmark = pytest.mark.gpu


@pytest.fixture
def guards():
    old = os.environ.get("DID_DEBUG_GUARD_ZONES")
    os.environ["DID_DEBUG_GUARD_ZONES"] = "1"
    yield
    if old is None:
        del os.environ["DID_DEBUG_GUARD_ZONES"]
    else:
        os.environ["DID_DEBUG_GUARD_ZONES"] = old


def _x(torch, M, N, K, seed):
    return device_x(torch, to_f32_colmajor(serving_x(M, N, K, seed=seed)))


def _check_clean(h, label):
    bad, zones = did.did_debug_check_guards(h)
    assert zones > 0, f"{label}: no guard zones (the handle was made without them)"
    assert bad == 0, f"{label}: {bad} guard bytes overwritten: {did.did_last_error()}"


@pytest.mark.parametrize("M,N,K,xd,tiled,refresh,alg", [
    (300, 2000, 10, did.DID_F32, 0, 1, did.DID_ALG_DID),    # K <= 32, X as given
    (130, 777, 40, did.DID_F32, 1, 1, did.DID_ALG_DID),     # K > 32, tile order, ragged tiles
    (130, 777, 64, did.DID_BF16, 0, 1, did.DID_ALG_DID),    # bf16 storage, largest K
    (300, 2000, 10, did.DID_F32, 0, 3, did.DID_ALG_DID),    # carried residual
    (97, 1234, 33, did.DID_BF16, 0, 4, did.DID_ALG_DID),    # carried residual, bf16, K just above 32
    (5, 4000, 3, did.DID_F32, 0, 1, did.DID_ALG_DID),       # thin 5 x 3
    (7, 700, 4, did.DID_F32, 0, 1, did.DID_ALG_DID),        # thin 8 x 4
    (8, 700, 8, did.DID_F32, 0, 1, did.DID_ALG_DID),        # thin 8 x 8
    (16, 700, 4, did.DID_F32, 0, 1, did.DID_ALG_DID),       # thin 16 x 4
    (5, 1000, 3, did.DID_F32, 0, 1, did.DID_ALG_DBCD),      # DBCD ablation
    (40, 1, 1, did.DID_F32, 0, 1, did.DID_ALG_DID),         # a single column of X
    (20, 20, 20, did.DID_F32, 1, 1, did.DID_ALG_DID),       # K = M = N, tile order
])
def test_paths_stay_inside_their_buffers(guards, M, N, K, xd, tiled, refresh, alg):
    torch = require_gpu()
    announce(f"guard zones {M}x{N} K={K} x_dtype={xd} tiled={tiled} refresh={refresh} alg={alg}")
    X = _x(torch, M, N, K, seed=M + N + K)
    o = did.did_default_opts()
    o.x_dtype = xd
    o.x_tiled = tiled
    o.refresh_every = refresh
    o.algorithm = alg
    h = did.did_init_ex(X, M, N, K, 7, o)
    try:
        _check_clean(h, "after init")
        did.did_iterate(h, 1)                # eager
        did.did_iterate(h, 2 * refresh + 1)  # replayed where the form allows it
        did.did_objective(h)
        Bt = np.empty((K, M), np.float32)
        Ct = np.empty((N, K), np.float32)
        did.did_factors(h, Bt, Ct)
        _check_clean(h, "after iterations")
    finally:
        did.did_free(h)


def test_resumed_and_profiled_handles_stay_inside_their_buffers(guards):
    torch = require_gpu()
    M, N, K = 260, 3000, 24
    announce("guard zones: resumed factors, profiled iterations")
    X = _x(torch, M, N, K, seed=3)
    rng = np.random.default_rng(3)
    B0 = torch.from_numpy(np.ascontiguousarray(rng.random((M, K)).astype(np.float32).T)).to("cuda")
    C0 = torch.from_numpy(np.ascontiguousarray(rng.random((K, N)).astype(np.float32).T)).to("cuda")
    torch.cuda.synchronize()
    h = did.did_init_from_factors(X, M, N, K, B0, C0, None)
    try:
        did.did_profile(h, 1)
        did.did_iterate(h, 3)
        did.did_profile_read(h)
        did.did_sync(h)
        _check_clean(h, "resumed, profiled")
    finally:
        did.did_free(h)


def test_batched_members_stay_inside_their_buffers(guards):
    torch = require_gpu()
    shapes = [(300, 2000, 10), (130, 777, 40), (97, 1234, 33)]
    announce("guard zones: batched members")
    Xs = [_x(torch, M, N, K, seed=20 + i) for i, (M, N, K) in enumerate(shapes)]
    o = did.did_default_opts()
    o.borrow_x = 1
    hs = [did.did_init_ex(Xs[i], M, N, K, 11 + i, o) for i, (M, N, K) in enumerate(shapes)]
    b = did.did_batch_create()
    try:
        for h in hs:
            did.did_batch_add(b, h)
        did.did_batch_iterate(b, 4)
        did.did_batch_sync(b)
        for i, h in enumerate(hs):
            _check_clean(h, f"batch member {i}")
        for h in hs:
            did.did_batch_remove(b, h)
    finally:
        did.did_batch_free(b)
        for h in hs:
            did.did_free(h)
