"""GPU tests of the batched and serving forms, the tile autotuner and the memory
accounting, all through the C ABI.

A batch member runs exactly the blocks of its own single-instance launch (through the
grouped persistent kernels and a replayed hipGraph), so its iterates must equal those of
the same instance run alone: the tests compare factors and objective histories bitwise,
after every replay and across membership changes.  The served results must equal the
same jobs run alone for the same number of iterations (bitwise as well).

Every batch member and every served job is also compared with the FP64 oracle from the
same initial factors (Alg. 3): factors after one iteration within 1e-5 normwise and 1e-4
per row of B and column of C, objectives within 1e-4 relative over the iterations run,
and a served job's factors at retirement within TOL_SERVED_FACTORS of the oracle's after
the same number of iterations."""

import numpy as np
import pytest

import oracle
import paper_1802_08938_amd as did
from tests._gpu import (announce, check_factors, check_trajectory, device_x, load_golden, read_factors, rel_fro,
                        require_gpu, worst_line)
from workloads import as_oracle_input, round_to_bf16, serving_x, to_f32_colmajor, uniform_init

# Served jobs retire after up to 30 iterations; their factors then differ from the oracle's
# by float32 rounding propagated through that many iterations (normwise, and per line).
TOL_SERVED_FACTORS = 1e-4
TOL_SERVED_LINE = 1e-3

pytestmark = pytest.mark.gpu

TILED = "f32-tiled"  # float32 X kept in tile order (x_tiled = 1)

# (M, N, K, X storage): both K classes (K <= 32 and K > 32), all three storages, ragged sizes
SHAPES = [(300, 2000, 10, did.DID_F32), (777, 1500, 40, did.DID_F32), (130, 5000, 64, did.DID_F32),
          (64, 999, 7, did.DID_F32), (250, 3000, 20, did.DID_BF16), (97, 1234, 33, did.DID_BF16),
          (3809, 2248, 49, did.DID_F32), (1868, 40000, 60, did.DID_F32), (500, 2500, 12, TILED),
          (611, 3333, 50, TILED)]


def _make(torch, M, N, K, xd, seed, cw=4):
    X = to_f32_colmajor(serving_x(M, N, K, seed=seed))
    Xd = device_x(torch, X)
    o = did.did_default_opts()
    o.x_dtype = did.DID_BF16 if xd == did.DID_BF16 else did.DID_F32
    o.x_tiled = 1 if xd == TILED else 0
    o.borrow_x = 1 if xd == did.DID_F32 else 0
    o.col_waves = cw
    h = did.did_init_ex(Xd, M, N, K, 1000 + seed, o)
    return h, Xd


def _alone(torch, M, N, K, xd, seed, iters, cw=4):
    h, Xd = _make(torch, M, N, K, xd, seed, cw)
    try:
        did.did_iterate(h, iters)
        B, C = read_factors(h, M, N, K)
        hist = np.array(did.did_history(h))
    finally:
        did.did_free(h)
    del Xd
    return B, C, hist


def test_batch_equals_alone_bitwise_every_replay():
    """Every other member runs the column pass with 8 waves per block, so each (K class,
    X storage) pair is split over two groups of different column tiles."""
    torch = require_gpu()
    T = 5
    announce(f"batch of {len(SHAPES)} vs alone")
    cws = [8 if i % 2 else 4 for i in range(len(SHAPES))]
    ref = [_alone(torch, M, N, K, xd, i, T, cws[i]) for i, (M, N, K, xd) in enumerate(SHAPES)]
    made = [_make(torch, M, N, K, xd, i, cws[i]) for i, (M, N, K, xd) in enumerate(SHAPES)]
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


@pytest.mark.parametrize("tiled,reserve", [(0, 0), (1, 0), (1, 1)])
def test_server_results_equal_alone_and_budget_holds(tiled, reserve):
    """Jobs of uneven shape arrive over several steps; the budget admits about two at a
    time, so later jobs queue and are admitted as earlier ones retire and are released.
    Every result equals the same job run alone (X column-major) for the same number of
    iterations, also when the server keeps X in tile order, and when it carves the jobs'
    buffers from a reserve (released out of order, ranges merged and carved again); the
    charged memory never exceeds the budget, and jobs are admitted first-in first-out."""
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
    so.arena_reserve_gib = reserve
    announce(f"server, budget {so.hbm_budget} bytes, reserve {reserve} GiB")
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
                    res[i] = (it, Bt.T.copy(), Ct.T.copy(), f)
                    did.did_server_release(s, j)
                assert st != did.DID_JOB_FAILED
            assert steps < 2000
        used, peak = did.did_server_memory(s)
        assert used == 0 and 0 < peak <= so.hbm_budget
        assert peak_running <= so.max_active
        if reserve:  # every job carved from the reserve
            assert did.did_server_arena_stats(s)[:3] == (0, len(jobs), 0)
        assert admit_order == sorted(admit_order)  # first in, first out
    finally:
        did.did_server_free(s)
    for i, (M, N, K) in enumerate(jobs):
        it, B, C, _ = res[i]
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
        _served_vs_oracle(X[i], M, N, K, 700 + i, it, B.astype(np.float64), C.astype(np.float64), res[i][3], 0)


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
        ot = did.did_default_opts()
        ot.x_tiled = 1
        tiled_before = did.did_mem_estimate(M, N, K, ot)
        rb, cw, ms = did.did_autotune(M, N, K)
        assert rb in (512, 1024, 2048, 4096, 8192) and cw in (4, 8) and ms > 0.0
        o2 = did.did_default_opts()
        o2.borrow_x = 1
        o2.row_blocks = rb
        o2.col_waves = cw
        # instances created afterwards with row_blocks = 0 take the tuned value (their
        # footprint includes the W partials of its column ranges)
        assert did.did_mem_estimate(M, N, K, o) == did.did_mem_estimate(M, N, K, o2)
        assert before > 0
        # the tiled float32 storage is a shape class of its own: still the defaults
        assert did.did_mem_estimate(M, N, K, ot) == tiled_before
        X = torch.rand((N, M), device="cuda")
        torch.cuda.synchronize()  # the engine reads X on its own stream
        h = did.did_init_ex(X, M, N, K, 5, o)
        try:
            assert did.did_mem_bytes(h) == did.did_mem_estimate(M, N, K, o)
        finally:
            did.did_free(h)
    finally:
        did.did_autotune_clear()


def test_free_returns_device_memory_after_graph_replays():
    """did_free gives back all of an instance's device memory after replayed iterations (a
    captured hipGraph), alone and after membership of a batch: three create / iterate /
    free cycles of a 3.2 GB (tiled X) instance leave the device's free memory where it was."""
    torch = require_gpu()
    M, N, K = 2000, 200_000, 20
    announce("device memory after free, graph replays")
    X = torch.rand((N, M), device="cuda")
    torch.cuda.synchronize()
    o = did.did_default_opts()
    o.borrow_x = 1
    o.x_tiled = 1
    need = did.did_mem_estimate(M, N, K, o)
    base = torch.cuda.mem_get_info()[0]
    for cycle in range(3):
        h = did.did_init_ex(X, M, N, K, 3 + cycle, o)
        did.did_iterate(h, 3)
        did.did_sync(h)
        did.did_free(h)
        torch.cuda.synchronize()
        held = base - torch.cuda.mem_get_info()[0]
        assert held < need / 4, (cycle, held, need)
    for cycle in range(2):
        hs = [did.did_init_ex(X, M, N, K, 10 + i, o) for i in range(2)]
        b = did.did_batch_create()
        try:
            for h in hs:
                did.did_batch_add(b, h)
            did.did_batch_iterate(b, 3)
            for h in hs:
                did.did_batch_remove(b, h)
        finally:
            did.did_batch_free(b)
            for h in hs:
                did.did_free(h)
        torch.cuda.synchronize()
        held = base - torch.cuda.mem_get_info()[0]
        assert held < need / 4, ("batch", cycle, held, need)


def test_server_fails_a_job_whose_x_is_invalid():
    """X is checked on the device while the batch iterates and read at the next step: a
    job whose X holds a negative entry fails, the jobs around it run to completion."""
    torch = require_gpu()
    jobs = [(300, 2000, 10), (260, 1500, 12), (300, 2000, 10)]
    Xs = [device_x(torch, to_f32_colmajor(serving_x(M, N, K, seed=60 + i))) for i, (M, N, K) in enumerate(jobs)]
    Xs[1][7, 3] = -1.0  # column 7, row 3 of the second job's X
    torch.cuda.synchronize()
    announce("server: invalid X fails its job")
    so = did.did_server_default_opts()
    so.max_iter = 4
    s = did.did_server_create(so)
    try:
        ids = [did.did_server_submit(s, Xs[i], M, N, K, 60 + i) for i, (M, N, K) in enumerate(jobs)]
        states = {}
        steps = 0
        while len(states) < len(ids):
            did.did_server_step(s)
            steps += 1
            for i, j in enumerate(ids):
                st = did.did_server_poll(s, j)[0]
                if st in (did.DID_JOB_DONE, did.DID_JOB_FAILED) and i not in states:
                    states[i] = st
            assert steps < 100
        assert states == {0: did.DID_JOB_DONE, 1: did.DID_JOB_FAILED, 2: did.DID_JOB_DONE}
        assert did.did_server_poll(s, ids[0])[1] == 4
        with pytest.raises(did.DidError) as err:  # the failed job's reason
            did.did_server_result(s, ids[1])
        assert err.value.code == did.DID_ESTATE and "finite and nonnegative" in str(err.value)
    finally:
        did.did_server_free(s)


def test_server_released_jobs_return_device_memory():
    """A released job's charge drops at the release itself; its handle is released at the
    server's next step (after the iteration in flight has ended), its device memory kept
    for later admissions, and freed with the server: device free memory then comes back to
    where it was."""
    torch = require_gpu()
    jobs = [(1500, 60000, 20), (900, 40000, 40), (1200, 50000, 12)]
    X = [device_x(torch, to_f32_colmajor(serving_x(M, N, K, seed=90 + i))) for i, (M, N, K) in enumerate(jobs)]
    torch.cuda.synchronize()
    announce("server release returns device memory")
    base = torch.cuda.mem_get_info()[0]
    so = did.did_server_default_opts()
    so.max_iter = 3
    s = did.did_server_create(so)
    try:
        ids = [did.did_server_submit(s, X[i], M, N, K, 90 + i) for i, (M, N, K) in enumerate(jobs)]
        done = set()
        steps = 0
        while len(done) < len(ids):
            did.did_server_step(s)
            steps += 1
            for j in ids:
                if j not in done and did.did_server_poll(s, j)[0] == did.DID_JOB_DONE:
                    did.did_server_release(s, j)
                    done.add(j)
            assert steps < 100
        assert did.did_server_memory(s)[0] == 0
        did.did_server_step(s)  # releases the handles released since the last step
        torch.cuda.synchronize()
        o = did.did_default_opts()
        o.borrow_x = 1  # the server adopts each job's X
        need = sum(did.did_mem_estimate(M, N, K, o, x_on_device=True) for M, N, K in jobs)
        held = base - torch.cuda.mem_get_info()[0]
        assert held < 2 * need, (held, need)  # at most the pooled arenas of these jobs
    finally:
        did.did_server_free(s)
    torch.cuda.synchronize()
    assert base - torch.cuda.mem_get_info()[0] < need / 4


@pytest.mark.parametrize("tiled,reserve", [(0, 0), (1, 0), (1, 1)])
def test_server_reused_arenas_give_the_same_results(tiled, reserve):
    """One job at a time, two shapes in turn, the second a little smaller: from the third
    job on, each admission takes the device memory a released job left behind (still
    holding that job's values), so every buffer must be set before it is read.  Each result
    equals the same job run alone, bitwise, and the server holds about two jobs' memory at
    the end instead of one per job.  With a reserve (1 GiB), every job is carved from it:
    no allocation at all, and the freed ranges are merged and carved again."""
    torch = require_gpu()
    shapes = [(400, 3000, 40), (380, 2900, 36)] * 4
    X = [device_x(torch, to_f32_colmajor(serving_x(M, N, K, seed=120 + i))) for i, (M, N, K) in enumerate(shapes)]
    torch.cuda.synchronize()
    announce(f"server arena reuse, tiled={tiled}")
    base = torch.cuda.mem_get_info()[0]
    so = did.did_server_default_opts()
    so.x_tiled = tiled
    so.max_active = 1
    so.max_iter = 3
    so.rel_tol = 0.0
    so.arena_reserve_gib = reserve
    s = did.did_server_create(so)
    res = {}
    try:
        ids = [did.did_server_submit(s, X[i], M, N, K, 130 + i) for i, (M, N, K) in enumerate(shapes)]
        steps = 0
        while len(res) < len(ids):
            did.did_server_step(s)
            steps += 1
            for i, j in enumerate(ids):
                if i in res:
                    continue
                st, it, _, _, _ = did.did_server_poll(s, j)
                assert st != did.DID_JOB_FAILED, did.did_last_error()
                if st == did.DID_JOB_DONE:
                    M, N, K = shapes[i]
                    Bt = np.empty((K, M), np.float32)
                    Ct = np.empty((N, K), np.float32)
                    did.did_server_result(s, j, Bt, Ct)
                    res[i] = (it, Bt, Ct)
                    did.did_server_release(s, j)
            assert steps < 200
        did.did_server_step(s)  # releases the last job's handle into the pool
        torch.cuda.synchronize()
        o = did.did_default_opts()
        o.borrow_x = 1
        o.x_tiled = tiled
        need = max(did.did_mem_estimate(M, N, K, o, x_on_device=True) for M, N, K in shapes)
        held = base - torch.cuda.mem_get_info()[0]
        allocs, reuses, frees, pooled = did.did_server_arena_stats(s)
        if reserve:
            assert (allocs, reuses, frees, pooled) == (0, len(shapes), 0, 0)
            assert held < (reserve << 30) + 3 * need, (held, need)
        else:
            assert held < 3 * need, (held, need)  # eight jobs, about two arenas
            assert allocs + reuses == len(shapes) and reuses >= len(shapes) - 3 and frees == 0, (allocs, reuses,
                                                                                                  frees)
            assert 0 < pooled < held
    finally:
        did.did_server_free(s)
    for i, (M, N, K) in enumerate(shapes):
        it, Bs, Cs = res[i]
        assert it == so.max_iter
        o = did.did_default_opts()
        o.borrow_x = 1
        h = did.did_init_ex(X[i], M, N, K, 130 + i, o)
        try:
            did.did_iterate(h, it)
            Bt = np.empty((K, M), np.float32)
            Ct = np.empty((N, K), np.float32)
            did.did_factors(h, Bt, Ct)
        finally:
            did.did_free(h)
        np.testing.assert_array_equal(Bs, Bt)
        np.testing.assert_array_equal(Cs, Ct)


@pytest.mark.parametrize("M,N,K,xd,borrow,tiled,refresh", [
    (300, 2000, 10, did.DID_F32, 1, 0, 1), (300, 2000, 10, did.DID_F32, 0, 0, 1),
    (130, 777, 64, did.DID_BF16, 0, 0, 1), (5, 1000, 3, did.DID_F32, 1, 0, 1),
    (16, 4000, 8, did.DID_F32, 0, 0, 1), (130, 777, 40, did.DID_F32, 1, 1, 1),
    (130, 777, 40, did.DID_BF16, 0, 0, 10), (300, 2000, 10, did.DID_F32, 1, 0, 3)])
def test_memory_estimate_matches_allocation(M, N, K, xd, borrow, tiled, refresh):
    torch = require_gpu()
    announce(f"memory estimate {M}x{N} K={K} refresh_every={refresh}")
    o = did.did_default_opts()
    o.x_dtype = xd
    o.borrow_x = borrow
    o.x_tiled = tiled
    o.refresh_every = refresh
    X = torch.rand((N, M), device="cuda")
    torch.cuda.synchronize()  # the engine reads X on its own stream
    h = did.did_init_ex(X, M, N, K, 5, o)
    try:
        assert did.did_mem_bytes(h) == did.did_mem_estimate(M, N, K, o, x_on_device=True)
    finally:
        did.did_free(h)


# members whose 5-iteration oracle trajectory is taken from tests/golden (make_trajectories.py)
GOLDEN_MEMBERS = {(3809, 2248, 49): "serving_3809x2248_k49", (1868, 40000, 60): "serving_1868x40000_k60"}


def _init_factors(M, N, K):
    B0, C0 = uniform_init(M, N, K, 12345)
    return B0.astype(np.float32), C0.astype(np.float32)


def _make_from_factors(torch, M, N, K, xd, seed):
    X32 = to_f32_colmajor(serving_x(M, N, K, seed=seed))
    Xd = device_x(torch, X32)
    B0, C0 = _init_factors(M, N, K)
    o = did.did_default_opts()
    o.x_dtype = did.DID_BF16 if xd == did.DID_BF16 else did.DID_F32
    o.x_tiled = 1 if xd == TILED else 0
    o.borrow_x = 1 if xd == did.DID_F32 else 0
    Bd = torch.from_numpy(np.ascontiguousarray(B0.T)).to("cuda")
    Cd = torch.from_numpy(np.ascontiguousarray(C0.T)).to("cuda")
    torch.cuda.synchronize()
    h = did.did_init_from_factors(Xd, M, N, K, Bd, Cd, o)
    Xo = round_to_bf16(X32) if xd == did.DID_BF16 else as_oracle_input(X32)
    return h, Xd, Xo, B0.astype(np.float64), C0.astype(np.float64)


def test_batch_members_match_oracle():
    """Every member of a mixed batch (both K classes, all X storages, the two largest
    shapes included) against the oracle from the same initial factors: all factors after
    one batched iteration, and the objective over five."""
    torch = require_gpu()
    T = 5
    announce(f"batch of {len(SHAPES)} vs the oracle")
    made = [_make_from_factors(torch, M, N, K, xd, i) for i, (M, N, K, xd) in enumerate(SHAPES)]
    b = did.did_batch_create()
    try:
        for m in made:
            did.did_batch_add(b, m[0])
        did.did_batch_iterate(b, 1)
        for m in made:
            did.did_batch_remove(b, m[0])
        for i, ((h, _, Xo, B0, C0), (M, N, K, xd)) in enumerate(zip(made, SHAPES)):
            B1, C1 = read_factors(h, M, N, K)
            B1o, C1o, _ = oracle.did_run(Xo, B0, C0, 1)
            check_factors(B1, B1o, C1, C1o, label=f"batch member {i} {M}x{N} K={K} {xd}")
        for m in made:  # the same members continue in the batch
            did.did_batch_add(b, m[0])
        did.did_batch_iterate(b, T - 1)
        for m in made:
            did.did_batch_remove(b, m[0])
        for i, ((h, _, Xo, B0, C0), (M, N, K, xd)) in enumerate(zip(made, SHAPES)):
            fg = np.append(did.did_history(h), did.did_objective(h))
            key = GOLDEN_MEMBERS.get((M, N, K))
            if key is not None:
                g = load_golden(key)
                assert g["T"] == T and g["x_storage"] == "f32"
                fo = np.array(g["f"])
            else:
                _, _, fo = oracle.did_run(Xo, B0, C0, T)
            check_trajectory(fg, fo, label=f"batch member {i} {M}x{N} K={K} {xd}")
    finally:
        did.did_batch_free(b)
        for m in made:
            did.did_free(m[0])


def _served_vs_oracle(X32, M, N, K, seed, it, B, C, f_last, tiled, bf16=False):
    """A served job's result against the oracle after the same number of iterations from
    the job's initial factors (read from a solo instance with the same seed); a job whose X
    is stored as bf16 against the oracle on bf16(X)."""
    torch = require_gpu()
    o = did.did_default_opts()
    o.borrow_x = 1
    o.x_tiled = tiled
    h = did.did_init_ex(X32, M, N, K, seed, o)
    try:
        B0, C0 = read_factors(h, M, N, K)
    finally:
        did.did_free(h)
    Xh = X32.cpu().numpy().T
    Xo = round_to_bf16(Xh) if bf16 else as_oracle_input(Xh)
    Bo, Co, fo = oracle.did_run(Xo, B0, C0, it)
    eb, ec = rel_fro(B, Bo), rel_fro(C, Co)
    lb, lc = worst_line(B, Bo, axis=1), worst_line(C, Co, axis=0)
    ef = abs(f_last - fo[it - 1]) / fo[it - 1]
    print(f"[served] {M}x{N} K={K} after {it} iterations: B {eb:.2e} C {ec:.2e} rows {lb:.2e} cols {lc:.2e} "
          f"f {ef:.2e}", flush=True)
    tol, tol_line = (1e-5, 1e-4) if it == 1 else (TOL_SERVED_FACTORS, TOL_SERVED_LINE)
    assert eb <= tol and ec <= tol, (eb, ec)
    assert lb <= tol_line and lc <= tol_line, (lb, lc)
    assert ef <= 1e-4, ef
    return fo


def test_server_early_stop_matches_oracle():
    """A loose stopping tolerance makes jobs retire mid-mix at different iterations; each
    retired job's factors and last objective equal the oracle's after that many
    iterations, and the stopping rule holds on the oracle's own trajectory (up to the
    float32 rounding of the objective near the threshold)."""
    torch = require_gpu()
    jobs = [(300, 2000, 10), (500, 1200, 40), (200, 4000, 64), (640, 900, 5), (128, 3000, 33), (350, 2500, 20),
            (420, 1500, 16), (256, 3100, 48)]
    so = did.did_server_default_opts()
    so.max_active = 6
    so.max_iter = 40
    so.rel_tol = 1e-1
    announce(f"server early stop, rel_tol {so.rel_tol}")
    s = did.did_server_create(so)
    X, ids, res = {}, [], {}
    try:
        for i, (M, N, K) in enumerate(jobs):
            X[i] = device_x(torch, to_f32_colmajor(serving_x(M, N, K, seed=90 + i)))
        steps = 0
        submitted = 0
        while len(res) < len(jobs):
            if submitted < len(jobs) and steps % 2 == 0:  # arrivals while others run
                M, N, K = jobs[submitted]
                ids.append(did.did_server_submit(s, X[submitted], M, N, K, 800 + submitted))
                submitted += 1
            did.did_server_step(s)
            steps += 1
            for i, j in enumerate(ids):
                if i in res:
                    continue
                st, it, f, lat, qs = did.did_server_poll(s, j)
                assert st != did.DID_JOB_FAILED
                if st == did.DID_JOB_DONE:
                    M, N, K = jobs[i]
                    Bt = np.empty((K, M), np.float32)
                    Ct = np.empty((N, K), np.float32)
                    did.did_server_result(s, j, Bt, Ct)
                    res[i] = (it, Bt.T.astype(np.float64), Ct.T.astype(np.float64), f)
                    did.did_server_release(s, j)
            assert steps < 1000
    finally:
        did.did_server_free(s)
    its = [res[i][0] for i in range(len(jobs))]
    print(f"[served] retirement iterations {its}", flush=True)
    assert len(set(its)) > 1 and max(its) < so.max_iter  # stopped early, at different iterations
    for i, (M, N, K) in enumerate(jobs):
        it, B, C, f = res[i]
        fo = _served_vs_oracle(X[i], M, N, K, 800 + i, it, B, C, f, 0)
        if it >= 2:  # the oracle's relative change at the retirement iteration is near the tolerance
            assert abs(fo[it - 2] - fo[it - 1]) <= 1.01 * so.rel_tol * fo[it - 1]


def test_server_mixed_storage_jobs_match_solo_and_oracle():
    """Jobs with X stored as float32 and as bf16 served together (they fall in different
    batch groups): each equals its solo run with the same storage bit for bit, and the
    oracle (on X, or on bf16(X)) after the same number of iterations."""
    torch = require_gpu()
    jobs = [(300, 2000, 10, did.DID_F32), (500, 1200, 40, did.DID_BF16), (200, 3000, 24, did.DID_BF16),
            (350, 2500, 48, did.DID_F32), (128, 1800, 12, did.DID_BF16)]
    so = did.did_server_default_opts()
    so.max_active = 8
    so.max_iter = 6
    so.rel_tol = 0.0
    announce("server, float32 and bf16 jobs together")
    s = did.did_server_create(so)
    X, ids, res = {}, [], {}
    try:
        for i, (M, N, K, xd) in enumerate(jobs):
            X[i] = device_x(torch, to_f32_colmajor(serving_x(M, N, K, seed=120 + i)))
            ids.append(did.did_server_submit(s, X[i], M, N, K, 900 + i, xd))
        steps = 0
        while len(res) < len(jobs):
            did.did_server_step(s)
            steps += 1
            for i, j in enumerate(ids):
                if i in res:
                    continue
                st, it, f, _, _ = did.did_server_poll(s, j)
                assert st != did.DID_JOB_FAILED
                if st == did.DID_JOB_DONE:
                    M, N, K, _ = jobs[i]
                    Bt = np.empty((K, M), np.float32)
                    Ct = np.empty((N, K), np.float32)
                    did.did_server_result(s, j, Bt, Ct)
                    res[i] = (it, Bt.T.copy(), Ct.T.copy(), f)
                    did.did_server_release(s, j)
            assert steps < 200
    finally:
        did.did_server_free(s)
    for i, (M, N, K, xd) in enumerate(jobs):
        it, B, C, f = res[i]
        assert it == so.max_iter
        o = did.did_default_opts()
        o.borrow_x = 1
        o.x_dtype = xd
        h = did.did_init_ex(X[i], M, N, K, 900 + i, o)
        try:
            did.did_iterate(h, it)
            Bs, Cs = read_factors(h, M, N, K)
        finally:
            did.did_free(h)
        np.testing.assert_array_equal(B, Bs)
        np.testing.assert_array_equal(C, Cs)
        _served_vs_oracle(X[i], M, N, K, 900 + i, it, B.astype(np.float64), C.astype(np.float64), f, 0,
                          bf16=xd == did.DID_BF16)


def test_batch_rejects_carried_residual_form():
    torch = require_gpu()
    announce("batch rejects refresh_every > 1")
    X = device_x(torch, to_f32_colmajor(serving_x(120, 900, 6, seed=3)))
    o = did.did_default_opts()
    o.borrow_x = 1
    o.refresh_every = 4
    h = did.did_init_ex(X, 120, 900, 6, 5, o)
    b = did.did_batch_create()
    try:
        with pytest.raises(did.DidError) as ei:
            did.did_batch_add(b, h)
        assert ei.value.code == did.DID_EINVAL
    finally:
        did.did_batch_free(b)
        did.did_free(h)
