"""GPU tests of the batched and serving forms, the row-pass autotuner and the memory
accounting, all through the C ABI.

A batch member runs exactly the blocks of its own single-instance launch (through the
grouped persistent kernels and a replayed hipGraph), so its iterates must equal those of
the same instance run alone: the tests compare factors and objective histories bitwise,
after every replay and across membership changes.  The served results must equal the
same jobs run alone for the same number of iterations (bitwise as well)."""

import numpy as np
import pytest

import paper_1802_08938_amd as did
from tests._gpu import announce, device_x, read_factors, require_gpu
from workloads import serving_x, to_f32_colmajor

pytestmark = pytest.mark.gpu

TILED = "f32-tiled"  # float32 X kept in tile order (x_tiled = 1)

# (M, N, K, X storage): both K classes (K <= 32 and K > 32), all three storages, ragged sizes
SHAPES = [(300, 2000, 10, did.DID_F32), (777, 1500, 40, did.DID_F32), (130, 5000, 64, did.DID_F32),
          (64, 999, 7, did.DID_F32), (250, 3000, 20, did.DID_BF16), (97, 1234, 33, did.DID_BF16),
          (3809, 2248, 49, did.DID_F32), (1868, 40000, 60, did.DID_F32), (500, 2500, 12, TILED),
          (611, 3333, 50, TILED)]


def _make(torch, M, N, K, xd, seed):
    X = to_f32_colmajor(serving_x(M, N, K, seed=seed))
    Xd = device_x(torch, X)
    o = did.did_default_opts()
    o.x_dtype = did.DID_BF16 if xd == did.DID_BF16 else did.DID_F32
    o.x_tiled = 1 if xd == TILED else 0
    o.borrow_x = 1 if xd == did.DID_F32 else 0
    h = did.did_init_ex(Xd, M, N, K, 1000 + seed, o)
    return h, Xd


def _alone(torch, M, N, K, xd, seed, iters):
    h, Xd = _make(torch, M, N, K, xd, seed)
    try:
        did.did_iterate(h, iters)
        B, C = read_factors(h, M, N, K)
        hist = np.array(did.did_history(h))
    finally:
        did.did_free(h)
    del Xd
    return B, C, hist


def test_batch_equals_alone_bitwise_every_replay():
    torch = require_gpu()
    T = 5
    announce(f"batch of {len(SHAPES)} vs alone")
    ref = [_alone(torch, M, N, K, xd, i, T) for i, (M, N, K, xd) in enumerate(SHAPES)]
    made = [_make(torch, M, N, K, xd, i) for i, (M, N, K, xd) in enumerate(SHAPES)]
    b = did.did_batch_create()
    try:
        for h, _ in made:
            did.did_batch_add(b, h)
        assert did.did_batch_size(b) == len(SHAPES)
        for t in range(T):
            did.did_batch_iterate(b, 1)
            f = did.did_batch_objectives(b)  # synchronises between replays
            for i in range(len(SHAPES)):
                assert f[i] == ref[i][2][t], (i, t)  # f of the iterate replay t started from
        for i, ((h, _), (M, N, K, _)) in enumerate(zip(made, SHAPES)):
            did.did_batch_remove(b, h)
            B, C = read_factors(h, M, N, K)
            assert did.did_iterations(h) == T
            np.testing.assert_array_equal(B, ref[i][0])
            np.testing.assert_array_equal(C, ref[i][1])
            np.testing.assert_array_equal(np.array(did.did_history(h)), ref[i][2])
    finally:
        did.did_batch_free(b)
        for h, _ in made:
            did.did_free(h)


def test_batch_membership_changes():
    """A joins, runs 3 iterations, B joins, 2 more, A leaves, B runs 2 more and then 1
    alone: A has 5 iterations and B 5, each equal to its solo run."""
    torch = require_gpu()
    sa, sb = (400, 2500, 16, did.DID_F32), (200, 1800, 50, did.DID_F32)
    announce("batch membership changes")
    ra = _alone(torch, *sa, 11, 5)
    rb = _alone(torch, *sb, 12, 5)
    ha, xa = _make(torch, *sa, 11)
    hb, xb = _make(torch, *sb, 12)
    b = did.did_batch_create()
    try:
        did.did_batch_add(b, ha)
        did.did_batch_iterate(b, 3)
        did.did_batch_add(b, hb)
        did.did_batch_iterate(b, 2)
        did.did_batch_remove(b, ha)
        did.did_batch_iterate(b, 2)
        did.did_batch_remove(b, hb)
        did.did_iterate(hb, 1)  # the same handle continues alone
        for h, s, r in ((ha, sa, ra), (hb, sb, rb)):
            M, N, K, _ = s
            B, C = read_factors(h, M, N, K)
            np.testing.assert_array_equal(B, r[0])
            np.testing.assert_array_equal(C, r[1])
            np.testing.assert_array_equal(np.array(did.did_history(h)), r[2])
    finally:
        did.did_batch_free(b)
        did.did_free(ha)
        did.did_free(hb)


def test_batch_rejections():
    torch = require_gpu()
    announce("batch rejections")
    b = did.did_batch_create()
    thin, xt = _make(torch, 5, 500, 3, did.DID_F32, 3)
    h, xh = _make(torch, 100, 500, 8, did.DID_F32, 4)
    try:
        with pytest.raises(did.DidError) as ei:
            did.did_batch_add(b, thin)
        assert ei.value.code == did.DID_EINVAL
        did.did_batch_add(b, h)
        with pytest.raises(did.DidError) as ei:
            did.did_batch_add(b, h)
        assert ei.value.code == did.DID_ESTATE
        for call in (lambda: did.did_iterate(h, 1), lambda: did.did_objective(h), lambda: did.did_free(h)):
            with pytest.raises(did.DidError) as ei:
                call()
            assert ei.value.code == did.DID_ESTATE
        with pytest.raises(did.DidError) as ei:
            did.did_batch_remove(b, thin)
        assert ei.value.code == did.DID_EINVAL
        did.did_batch_remove(b, h)
        did.did_iterate(h, 1)
    finally:
        did.did_batch_free(b)
        did.did_free(thin)
        did.did_free(h)


@pytest.mark.parametrize("tiled", [0, 1])
def test_server_results_equal_alone_and_budget_holds(tiled):
    """Jobs of uneven shape arrive over several steps; the budget admits about two at a
    time, so later jobs queue and are admitted as earlier ones retire and are released.
    Every result equals the same job run alone (X column-major) for the same number of
    iterations, also when the server keeps X in tile order; the charged memory never
    exceeds the budget, and jobs are admitted first-in first-out."""
    torch = require_gpu()
    jobs = [(300, 2000, 10), (500, 1200, 40), (200, 4000, 64), (640, 900, 5), (128, 3000, 33), (350, 2500, 20)]
    o0 = did.did_default_opts()
    o0.borrow_x = 1
    o0.x_tiled = tiled
    fp = [did.did_mem_estimate(M, N, K, o0) + 4 * M * N for M, N, K in jobs]
    so = did.did_server_default_opts()
    so.x_tiled = tiled
    so.hbm_budget = int(max(fp) + sorted(fp)[-2])
    so.max_active = 4
    so.max_iter = 30
    so.rel_tol = 1e-3
    announce(f"server, budget {so.hbm_budget} bytes")
    s = did.did_server_create(so)
    X = {}
    ids = []
    res = {}
    admit_order = []
    try:
        submitted = 0
        steps = 0
        peak_running = 0
        while len(res) < len(jobs):
            if submitted < len(jobs) and (submitted < 3 or steps in (2, 4, 6)):  # later arrivals
                i = submitted
                M, N, K = jobs[i]
                X[i] = device_x(torch, to_f32_colmajor(serving_x(M, N, K, seed=50 + i)))
                ids.append(did.did_server_submit(s, X[i], M, N, K, 700 + i))
                submitted += 1
                if submitted < 3:
                    continue
            running, queued, _ = did.did_server_step(s)
            steps += 1
            peak_running = max(peak_running, running)
            assert did.did_server_memory(s)[0] <= so.hbm_budget
            for i, j in enumerate(ids):
                if i in res:
                    continue
                st, it, f, lat, qs = did.did_server_poll(s, j)
                if st != did.DID_JOB_QUEUED and i not in admit_order:
                    admit_order.append(i)
                if st == did.DID_JOB_DONE:
                    assert 1 <= it <= so.max_iter and lat >= qs >= 0.0
                    M, N, K = jobs[i]
                    Bt = np.empty((K, M), np.float32)
                    Ct = np.empty((N, K), np.float32)
                    did.did_server_result(s, j, Bt, Ct)
                    res[i] = (it, Bt.T.copy(), Ct.T.copy())
                    did.did_server_release(s, j)
                assert st != did.DID_JOB_FAILED
            assert steps < 2000
        used, peak = did.did_server_memory(s)
        assert used == 0 and 0 < peak <= so.hbm_budget
        assert peak_running <= so.max_active
        assert admit_order == sorted(admit_order)  # first in, first out
    finally:
        did.did_server_free(s)
    for i, (M, N, K) in enumerate(jobs):
        it, B, C = res[i]
        o = did.did_default_opts()
        o.borrow_x = 1
        h = did.did_init_ex(X[i], M, N, K, 700 + i, o)
        try:
            did.did_iterate(h, it)
            Bt = np.empty((K, M), np.float32)
            Ct = np.empty((N, K), np.float32)
            did.did_factors(h, Bt, Ct)
        finally:
            did.did_free(h)
        np.testing.assert_array_equal(B, Bt.T)
        np.testing.assert_array_equal(C, Ct.T)


def test_server_rejects_oversized_and_thin_jobs():
    torch = require_gpu()
    bad = did.did_server_default_opts()
    bad.x_tiled = 2
    with pytest.raises(did.DidError) as ei:
        did.did_server_create(bad)
    assert ei.value.code == did.DID_EINVAL
    so = did.did_server_default_opts()
    so.hbm_budget = 1 << 20
    s = did.did_server_create(so)
    X = torch.ones((1000, 300), device="cuda")
    torch.cuda.synchronize()
    announce("server rejections")
    try:
        with pytest.raises(did.DidError) as ei:
            did.did_server_submit(s, X, 300, 1000, 10, 1)
        assert ei.value.code == did.DID_ENOMEM
        with pytest.raises(did.DidError) as ei:
            did.did_server_submit(s, X, 5, 1000, 3, 1)
        assert ei.value.code == did.DID_EINVAL
    finally:
        did.did_server_free(s)


def test_autotune_records_and_applies():
    torch = require_gpu()
    M, N, K = 700, 20000, 24
    announce("autotune")
    did.did_autotune_clear()
    try:
        o = did.did_default_opts()
        o.borrow_x = 1
        before = did.did_mem_estimate(M, N, K, o)
        rb, ms = did.did_autotune(M, N, K)
        assert rb in (512, 1024, 2048, 4096, 8192) and ms > 0.0
        o2 = did.did_default_opts()
        o2.borrow_x = 1
        o2.row_blocks = rb
        # instances created afterwards with row_blocks = 0 take the tuned value (their
        # footprint includes the W partials of its column ranges)
        assert did.did_mem_estimate(M, N, K, o) == did.did_mem_estimate(M, N, K, o2)
        assert before > 0
        X = torch.rand((N, M), device="cuda")
        torch.cuda.synchronize()  # the engine reads X on its own stream
        h = did.did_init_ex(X, M, N, K, 5, o)
        try:
            assert did.did_mem_bytes(h) == did.did_mem_estimate(M, N, K, o)
        finally:
            did.did_free(h)
    finally:
        did.did_autotune_clear()


@pytest.mark.parametrize("M,N,K,xd,borrow,tiled", [(300, 2000, 10, did.DID_F32, 1, 0), (300, 2000, 10, did.DID_F32, 0, 0),
                                                   (130, 777, 64, did.DID_BF16, 0, 0), (5, 1000, 3, did.DID_F32, 1, 0),
                                                   (16, 4000, 8, did.DID_F32, 0, 0), (130, 777, 40, did.DID_F32, 1, 1)])
def test_memory_estimate_matches_allocation(M, N, K, xd, borrow, tiled):
    torch = require_gpu()
    announce(f"memory estimate {M}x{N} K={K}")
    o = did.did_default_opts()
    o.x_dtype = xd
    o.borrow_x = borrow
    o.x_tiled = tiled
    X = torch.rand((N, M), device="cuda")
    torch.cuda.synchronize()  # the engine reads X on its own stream
    h = did.did_init_ex(X, M, N, K, 5, o)
    try:
        assert did.did_mem_bytes(h) == did.did_mem_estimate(M, N, K, o, x_on_device=True)
    finally:
        did.did_free(h)
