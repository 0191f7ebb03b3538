"""Host-side checks of the C ABI: the library loads, exports every symbol include/did.h
declares, and rejects bad arguments before touching a device (no compute calls here)."""

import ctypes
import os
import re

import pytest

import paper_1802_08938_amd as did

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "did.h")


def _lib_or_skip():
    try:
        return did.lib()
    except did.DidLibraryMissing:
        pytest.skip("libdid.so not built (run __graft_entry__.build())")


def header_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(did_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_names():
    assert set(header_symbols()) == set(did.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = _lib_or_skip()
    for name in header_symbols():
        assert hasattr(L, name), name


def test_default_opts_and_struct_layout():
    _lib_or_skip()
    o = did.did_default_opts()
    assert (o.n_blocks, o.x_dtype, o.refresh_every, o.init_scale, o.borrow_x) == (0, did.DID_F32, 1, 0, 0)
    assert (o.algorithm, o.row_blocks, o.x_tiled, o.col_waves) == (did.DID_ALG_DID, 0, 0, 0)
    assert o.stream is None
    assert ctypes.sizeof(did.did_opts) == 48
    so = did.did_server_default_opts()
    assert (so.hbm_budget, so.max_active, so.max_iter, so.rel_tol) == (200 << 30, 64, 50, 1e-4)
    assert (so.x_tiled, so.arena_reserve_gib) == (0, 0) and so.stream is None
    assert ctypes.sizeof(did.did_server_opts) == 40
    assert did.did_server_opts.arena_reserve_gib.offset == 28 and did.did_server_opts.stream.offset == 32


@pytest.mark.parametrize("M,N,K,msg", [
    (0, 10, 1, "M, N and K"),
    (10, 0, 1, "M, N and K"),
    (10, 10, 0, "M, N and K"),
    (100, 100, 65, "K > 64"),
    (5, 100, 6, "min(M, N)"),
    (100, 5, 6, "min(M, N)"),
])
def test_shape_validation_without_device(M, N, K, msg):
    L = _lib_or_skip()
    h = ctypes.c_void_p(12345)
    dummy = (ctypes.c_float * 4)()
    rc = L.did_init(ctypes.cast(dummy, ctypes.c_void_p), M, N, K, 1, ctypes.byref(h))
    assert rc == did.DID_EINVAL
    assert h.value is None
    assert msg in did.did_last_error()


def test_null_arguments():
    L = _lib_or_skip()
    h = ctypes.c_void_p()
    assert L.did_init(None, 4, 4, 1, 1, ctypes.byref(h)) == did.DID_EINVAL
    dummy = (ctypes.c_float * 4)()
    assert L.did_init(ctypes.cast(dummy, ctypes.c_void_p), 2, 2, 1, 1, None) == did.DID_EINVAL
    assert L.did_iterate(None, 1) == did.DID_EINVAL
    f = ctypes.c_double()
    assert L.did_objective(None, ctypes.byref(f)) == did.DID_EINVAL
    assert L.did_factors(None, None, None) == did.DID_EINVAL
    assert L.did_free(None) == did.DID_OK
    assert L.did_default_opts(None) == did.DID_EINVAL
    with pytest.raises(did.DidError) as ei:
        did.did_iterate(None, 1)
    assert ei.value.code == did.DID_EINVAL


def test_binding_raises_when_library_missing(monkeypatch, tmp_path):
    monkeypatch.setenv("DID_LIBRARY", str(tmp_path / "nope.so"))
    monkeypatch.setattr(did, "_lib", None)
    with pytest.raises(did.DidLibraryMissing):
        did.lib()


def test_bf16_rounding_helper_matches_torch():
    """workloads.round_to_bf16 (used to build the oracle's input for the bf16 storage form)
    agrees with torch's own float32 -> bfloat16 conversion (round to nearest even)."""
    import numpy as np
    import torch

    from workloads import round_to_bf16

    rng = np.random.default_rng(0)
    x = np.concatenate([rng.random(5000) * 20.0, rng.random(5000) * 1e-3, np.array([0.0, 1.0, 3.0e38])])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_to_bf16(x), ref)


def test_memory_estimate_host_logic():
    """did_mem_estimate is pure host arithmetic for MFMA-path shapes: a copied float32 X
    adds exactly 4MN bytes, the bf16 storage form two tiled copies of 2 bytes per entry of
    X zero-padded to multiples of 32 rows and columns, and the large workload's footprint
    is dominated by X and the packed C."""
    _lib_or_skip()
    M, N, K = 5000, 1_000_000, 50
    o = did.did_default_opts()
    o.borrow_x = 1
    borrowed = did.did_mem_estimate(M, N, K, o, x_on_device=True)
    copied = did.did_mem_estimate(M, N, K, o, x_on_device=False)
    assert copied - borrowed == 4 * M * N
    ob = did.did_default_opts()
    ob.x_dtype = did.DID_BF16
    Mp, Np = (M + 31) // 32 * 32, (N + 31) // 32 * 32
    assert did.did_mem_estimate(M, N, K, ob) - borrowed == 2 * 2 * Mp * Np
    # packed C: per 32-column tile (64/16*3 + 64/32*6) units of 64 x 16 bytes
    cq = (N + 31) // 32 * (12 + 12) * 64 * 16
    assert borrowed > cq + 4 * K * N and borrowed < 3e9


def test_batch_and_server_null_arguments():
    L = _lib_or_skip()
    assert L.did_batch_add(None, None) == did.DID_EINVAL
    assert L.did_batch_iterate(None, 1) == did.DID_EINVAL
    assert L.did_batch_free(None) == did.DID_OK
    assert L.did_server_step(None, None, None, None) == did.DID_EINVAL
    assert L.did_server_free(None) == did.DID_OK
    so = did.did_server_default_opts()
    so.max_active = 0
    h = ctypes.c_void_p()
    assert L.did_server_create(ctypes.byref(so), ctypes.byref(h)) == did.DID_EINVAL
    assert "server options" in did.did_last_error()
    so = did.did_server_default_opts()
    so.arena_reserve_gib = -1
    assert L.did_server_create(ctypes.byref(so), ctypes.byref(h)) == did.DID_EINVAL
    assert L.did_server_arena_stats(None, None, None, None, None) == did.DID_EINVAL


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; --gpus N with N > 1 exits with a message (checked
    before anything touches a device)."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_column_major_x_lane_offset_bound():
    """Column-major float32 X is addressed with 32-bit lane offsets of up to 32 M elements:
    a taller X is refused (before any allocation) unless it is kept in tile order."""
    _lib_or_skip()
    M, N, K = 140_000_000, 32, 8  # 32 M >= 2^32
    o = did.did_default_opts()
    o.borrow_x = 1
    with pytest.raises(did.DidError) as ei:
        did.did_mem_estimate(M, N, K, o)
    assert ei.value.code == did.DID_EINVAL and "32-bit lane offsets" in str(ei.value)
    o.x_tiled = 1
    assert did.did_mem_estimate(M, N, K, o) > 8 * M * N
    o.x_tiled = 0
    assert did.did_mem_estimate(134_217_727, N, K, o) > 0  # 32 M = 2^32 - 32: accepted
    L = did.lib()
    h = ctypes.c_void_p(7)
    dummy = (ctypes.c_float * 4)()
    assert L.did_init_ex(ctypes.cast(dummy, ctypes.c_void_p), M, N, K, 1, ctypes.byref(o), ctypes.byref(h)) == did.DID_EINVAL
    assert h.value is None


def test_fault_injection_needs_a_handle():
    L = _lib_or_skip()
    assert L.did_debug_inject_fault(None) == did.DID_EINVAL


def test_carried_residual_options_without_device():
    """refresh_every > 1 keeps the residual resident (4 M N more bytes plus the packed
    changes of B and C); it needs the MFMA path and 32 M < 2^32; 0 is refused."""
    _lib_or_skip()
    o = did.did_default_opts()
    o.borrow_x = 1
    base = did.did_mem_estimate(1000, 5000, 20, o)
    o.refresh_every = 10
    carried = did.did_mem_estimate(1000, 5000, 20, o)
    assert carried >= base + 4 * 1000 * 5000
    for M, N, K, r in ((5, 1000, 3, 2), (1000, 5000, 20, 0), (140_000_000, 32, 8, 2)):
        o.refresh_every = r
        o.x_tiled = 1 if M > 1000 else 0
        with pytest.raises(did.DidError) as ei:
            did.did_mem_estimate(M, N, K, o)
        assert ei.value.code == did.DID_EINVAL


def test_column_tile_option_without_device():
    """col_waves picks 4 or 8 waves per column-pass block; the per-block objective
    partials shrink with 8, and the carried form refuses 8."""
    _lib_or_skip()
    M, N, K = 1000, 1_000_000, 20
    o = did.did_default_opts()
    o.borrow_x = 1
    base = did.did_mem_estimate(M, N, K, o)
    o.col_waves = 4
    assert did.did_mem_estimate(M, N, K, o) == base
    o.col_waves = 8
    # one f64 partial per block: N/128 blocks with 4 waves, N/256 with 8
    assert base - did.did_mem_estimate(M, N, K, o) == 8 * (N // 128 - N // 256)
    for cw, r in ((6, 1), (-1, 1), (8, 10)):
        o.col_waves, o.refresh_every = cw, r
        with pytest.raises(did.DidError) as ei:
            did.did_mem_estimate(M, N, K, o)
        assert ei.value.code == did.DID_EINVAL
    o.col_waves, o.refresh_every = 4, 10
    assert did.did_mem_estimate(M, N, K, o) > base


def test_autotune_argument_checks_without_device():
    """The autotuner validates its arguments before it allocates the tuning input."""
    L = _lib_or_skip()
    rb, cw = ctypes.c_int32(7), ctypes.c_int32(7)
    bad = [(0, 10, 1, did.DID_F32, 0), (100, 100, 65, did.DID_F32, 0), (5, 1000, 3, did.DID_F32, 0),
           (100, 100, 10, 7, 0), (100, 100, 10, did.DID_F32, 2), (1 << 41, 10, 3, did.DID_F32, 1)]
    for M, N, K, xd, xt in bad:
        assert L.did_autotune(M, N, K, xd, xt, ctypes.byref(rb), ctypes.byref(cw), None) == did.DID_EINVAL, (M, N, K)
        assert (rb.value, cw.value) in ((0, 0), (7, 7))
    assert L.did_autotune(100, 100, 10, did.DID_F32, 0, ctypes.byref(rb), None, None) == did.DID_EINVAL


@pytest.mark.parametrize("M,N,K", [(5000, 1_000_000, 50), (2000, 200_000, 20), (784, 70_000, 16),
                                   (500, 150_000, 10), (1000, 20_000, 30), (3000, 3_000_000, 40)])
def test_default_row_target_follows_n(M, N, K):
    """With no tuned entry, the row pass's default target is N / 256 blocks clamped to
    [512, 4096]: the footprint (which counts the W partials of the column ranges) equals
    that of the explicit target."""
    _lib_or_skip()
    did.did_autotune_clear()
    o = did.did_default_opts()
    o.borrow_x = 1
    e = did.did_default_opts()
    e.borrow_x = 1
    e.row_blocks = min(4096, max(512, N // 256))
    assert did.did_mem_estimate(M, N, K, o) == did.did_mem_estimate(M, N, K, e)
