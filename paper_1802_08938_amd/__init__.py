"""Python binding of libdid, the MI355X DID engine (ctypes over the C ABI in include/did.h).

The functions carry the C names and only marshal arguments: every step of an iteration
runs in the HIP kernels of ``libdid.so``.  There is no fallback: if the library is not
built, every call raises ``DidLibraryMissing``.

Array arguments may be raw integer addresses, torch tensors (their ``data_ptr()``; device
or host) or NumPy arrays (host).  Matrices are column-major: pass X of shape (M, N) with
strides (1, M) -- e.g. ``torch.empty((N, M)).T`` or ``np.asfortranarray(X)``.
"""

from __future__ import annotations

import ctypes
import os

__all__ = [
    "DID_OK", "DID_EINVAL", "DID_ENOMEM", "DID_EDEVICE", "DID_ESTATE", "DID_F32", "DID_BF16", "DID_MAX_K",
    "DID_ALG_DID", "DID_ALG_DBCD",
    "DidError", "DidLibraryMissing", "did_opts", "lib", "library_path",
    "did_default_opts", "did_init", "did_init_ex", "did_init_from_factors", "did_iterate", "did_objective",
    "did_factors", "did_history", "did_iterations", "did_sync", "did_free", "did_last_error",
    "did_profile", "did_profile_read", "did_stage_name", "EXPORTED_SYMBOLS",
    "did_mem_bytes", "did_mem_estimate", "did_autotune", "did_autotune_clear",
    "did_batch_create", "did_batch_add", "did_batch_remove", "did_batch_size", "did_batch_iterate",
    "did_batch_objectives", "did_batch_sync", "did_batch_free",
    "did_server_opts", "did_server_default_opts", "did_server_create", "did_server_submit", "did_server_step",
    "did_server_poll", "did_server_result", "did_server_release", "did_server_memory", "did_server_arena_stats",
    "did_server_free",
    "DID_JOB_QUEUED", "DID_JOB_RUNNING", "DID_JOB_DONE", "DID_JOB_FAILED", "did_debug_inject_fault",
    "did_debug_check_guards", "did_iterate_static", "DID_STATIC_SCRATCH_BYTES", "DID_GUARD_ZONE_BYTES",
]

DID_OK, DID_EINVAL, DID_ENOMEM, DID_EDEVICE, DID_ESTATE = 0, -1, -2, -3, -4
DID_F32, DID_BF16 = 0, 1
DID_ALG_DID, DID_ALG_DBCD = 0, 1
DID_MAX_K = 64
DID_STATIC_SCRATCH_BYTES = 128 << 20
DID_GUARD_ZONE_BYTES = 4096
DID_JOB_QUEUED, DID_JOB_RUNNING, DID_JOB_DONE, DID_JOB_FAILED = 0, 1, 2, 3

EXPORTED_SYMBOLS = (
    "did_default_opts", "did_init", "did_init_ex", "did_init_from_factors", "did_iterate", "did_objective",
    "did_factors", "did_history", "did_iterations", "did_sync", "did_free", "did_last_error",
    "did_profile", "did_profile_read", "did_stage_name",
    "did_mem_bytes", "did_mem_estimate", "did_autotune", "did_autotune_clear",
    "did_batch_create", "did_batch_add", "did_batch_remove", "did_batch_size", "did_batch_iterate",
    "did_batch_objectives", "did_batch_sync", "did_batch_free",
    "did_server_default_opts", "did_server_create", "did_server_submit", "did_server_step", "did_server_poll",
    "did_server_result", "did_server_release", "did_server_memory", "did_server_arena_stats", "did_server_free",
    "did_debug_inject_fault", "did_debug_check_guards", "did_iterate_static",
)

_HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.environ.get("DID_LIBRARY", os.path.join(_HERE, "libdid.so"))


class DidLibraryMissing(RuntimeError):
    pass


class DidError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"DID error {code}: {msg}")
        self.code = code


class did_opts(ctypes.Structure):
    _fields_ = [
        ("n_blocks", ctypes.c_int32),
        ("x_dtype", ctypes.c_int32),
        ("refresh_every", ctypes.c_int32),
        ("init_scale", ctypes.c_int32),
        ("borrow_x", ctypes.c_int32),
        ("algorithm", ctypes.c_int32),
        ("row_blocks", ctypes.c_int32),
        ("x_tiled", ctypes.c_int32),
        ("col_waves", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
    ]


class did_server_opts(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_int64),
        ("max_active", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("rel_tol", ctypes.c_double),
        ("x_tiled", ctypes.c_int32),
        ("arena_reserve_gib", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """Load libdid.so once (raises DidLibraryMissing if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise DidLibraryMissing(f"{path} not found: build it with `python -m paper_1802_08938_amd.build`")
    L = ctypes.CDLL(path)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    sig = {
        "did_default_opts": [ctypes.POINTER(did_opts)],
        "did_init": [vp, i64, i64, i32, u64, ctypes.POINTER(vp)],
        "did_init_ex": [vp, i64, i64, i32, u64, ctypes.POINTER(did_opts), ctypes.POINTER(vp)],
        "did_init_from_factors": [vp, i64, i64, i32, vp, vp, ctypes.POINTER(did_opts), ctypes.POINTER(vp)],
        "did_iterate": [vp, i32],
        "did_objective": [vp, ctypes.POINTER(ctypes.c_double)],
        "did_factors": [vp, vp, vp],
        "did_history": [vp, ctypes.POINTER(ctypes.c_double), i64, ctypes.POINTER(i64)],
        "did_iterations": [vp, ctypes.POINTER(i64)],
        "did_sync": [vp],
        "did_free": [vp],
        "did_profile": [vp, i32],
        "did_profile_read": [vp, ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i32), ctypes.POINTER(i64)],
        "did_mem_bytes": [vp, ctypes.POINTER(i64)],
        "did_mem_estimate": [i64, i64, i32, ctypes.POINTER(did_opts), i32, ctypes.POINTER(i64)],
        "did_autotune": [i64, i64, i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                         ctypes.POINTER(ctypes.c_double)],
        "did_autotune_clear": [],
        "did_batch_create": [vp, ctypes.POINTER(vp)],
        "did_batch_add": [vp, vp],
        "did_batch_remove": [vp, vp],
        "did_batch_size": [vp, ctypes.POINTER(i32)],
        "did_batch_iterate": [vp, i32],
        "did_batch_objectives": [vp, ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i32)],
        "did_batch_sync": [vp],
        "did_batch_free": [vp],
        "did_server_default_opts": [ctypes.POINTER(did_server_opts)],
        "did_server_create": [ctypes.POINTER(did_server_opts), ctypes.POINTER(vp)],
        "did_server_submit": [vp, vp, i64, i64, i32, u64, i32, ctypes.POINTER(i64)],
        "did_server_step": [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "did_server_poll": [vp, i64, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
        "did_server_result": [vp, i64, vp, vp],
        "did_server_release": [vp, i64],
        "did_server_memory": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "did_server_arena_stats": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                   ctypes.POINTER(i64)],
        "did_server_free": [vp],
        "did_debug_inject_fault": [vp],
        "did_debug_check_guards": [vp, ctypes.POINTER(i64), ctypes.POINTER(i32)],
        "did_iterate_static": [vp, i64, i64, i32, vp, vp, i32, ctypes.POINTER(did_opts), vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.did_last_error.argtypes = []
    L.did_last_error.restype = ctypes.c_char_p
    L.did_stage_name.argtypes = [i32]
    L.did_stage_name.restype = ctypes.c_char_p
    _lib = L
    return L


def did_last_error() -> str:
    return lib().did_last_error().decode()


def _check(rc):
    if rc != DID_OK:
        raise DidError(rc, did_last_error())
    return rc


def _ptr(a):
    """Address of an array-like (int, torch tensor, NumPy array) or None."""
    if a is None:
        return None
    if isinstance(a, int):
        return a
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    if hasattr(a, "ctypes"):
        return a.ctypes.data
    raise TypeError(f"cannot take the address of {type(a).__name__}")


def did_default_opts() -> did_opts:
    o = did_opts()
    _check(lib().did_default_opts(ctypes.byref(o)))
    return o


def did_init(X, M, N, K, seed):
    h = ctypes.c_void_p()
    _check(lib().did_init(_ptr(X), M, N, K, seed, ctypes.byref(h)))
    return h


def did_init_ex(X, M, N, K, seed, opts=None):
    h = ctypes.c_void_p()
    op = ctypes.byref(opts) if opts is not None else None
    _check(lib().did_init_ex(_ptr(X), M, N, K, seed, op, ctypes.byref(h)))
    return h


def did_init_from_factors(X, M, N, K, B, C, opts=None):
    h = ctypes.c_void_p()
    op = ctypes.byref(opts) if opts is not None else None
    _check(lib().did_init_from_factors(_ptr(X), M, N, K, _ptr(B), _ptr(C), op, ctypes.byref(h)))
    return h


def did_iterate(h, n):
    _check(lib().did_iterate(h, n))


def did_objective(h) -> float:
    f = ctypes.c_double()
    _check(lib().did_objective(h, ctypes.byref(f)))
    return f.value


def did_factors(h, B=None, C=None):
    """Copy B (M x K) and C (K x N), column-major float32, into caller buffers."""
    _check(lib().did_factors(h, _ptr(B), _ptr(C)))


def did_history(h):
    """Objective history f[0..t-1] as a list of floats."""
    cnt = ctypes.c_int64()
    _check(lib().did_history(h, None, 0, ctypes.byref(cnt)))
    n = cnt.value
    buf = (ctypes.c_double * max(n, 1))()
    _check(lib().did_history(h, buf, n, ctypes.byref(cnt)))
    return list(buf[:n])


def did_iterations(h) -> int:
    t = ctypes.c_int64()
    _check(lib().did_iterations(h, ctypes.byref(t)))
    return t.value


def did_sync(h):
    _check(lib().did_sync(h))


def did_free(h):
    _check(lib().did_free(h))


def did_profile(h, enable=True):
    _check(lib().did_profile(h, 1 if enable else 0))


def did_profile_read(h):
    """Summed milliseconds per kernel stage since the last read: (dict name->ms, n_iters)."""
    buf = (ctypes.c_double * 32)()
    ns = ctypes.c_int32()
    ni = ctypes.c_int64()
    _check(lib().did_profile_read(h, buf, 32, ctypes.byref(ns), ctypes.byref(ni)))
    return {did_stage_name(i): buf[i] for i in range(ns.value)}, ni.value


def did_stage_name(i) -> str:
    return lib().did_stage_name(i).decode()


def did_mem_bytes(h) -> int:
    b = ctypes.c_int64()
    _check(lib().did_mem_bytes(h, ctypes.byref(b)))
    return b.value


def did_mem_estimate(M, N, K, opts=None, x_on_device=True) -> int:
    b = ctypes.c_int64()
    op = ctypes.byref(opts) if opts is not None else None
    _check(lib().did_mem_estimate(M, N, K, op, 1 if x_on_device else 0, ctypes.byref(b)))
    return b.value


def did_autotune(M, N, K, x_dtype=DID_F32, x_tiled=0):
    """Tune the pass tiles for the shape class of (M, N, K) and X storage; returns
    (row_blocks, col_waves, ms per iteration)."""
    rb = ctypes.c_int32()
    cw = ctypes.c_int32()
    ms = ctypes.c_double()
    _check(lib().did_autotune(M, N, K, x_dtype, x_tiled, ctypes.byref(rb), ctypes.byref(cw), ctypes.byref(ms)))
    return rb.value, cw.value, ms.value


def did_autotune_clear():
    _check(lib().did_autotune_clear())


def did_batch_create(stream=None):
    b = ctypes.c_void_p()
    _check(lib().did_batch_create(stream, ctypes.byref(b)))
    return b


def did_batch_add(b, h):
    _check(lib().did_batch_add(b, h))


def did_batch_remove(b, h):
    _check(lib().did_batch_remove(b, h))


def did_batch_size(b) -> int:
    n = ctypes.c_int32()
    _check(lib().did_batch_size(b, ctypes.byref(n)))
    return n.value


def did_batch_iterate(b, n):
    _check(lib().did_batch_iterate(b, n))


def did_batch_objectives(b):
    """Latest objective of every member, in admission order."""
    cap = 256
    buf = (ctypes.c_double * cap)()
    n = ctypes.c_int32()
    _check(lib().did_batch_objectives(b, buf, cap, ctypes.byref(n)))
    return list(buf[:n.value])


def did_batch_sync(b):
    _check(lib().did_batch_sync(b))


def did_batch_free(b):
    _check(lib().did_batch_free(b))


def did_server_default_opts() -> did_server_opts:
    o = did_server_opts()
    _check(lib().did_server_default_opts(ctypes.byref(o)))
    return o


def did_server_create(opts=None):
    s = ctypes.c_void_p()
    op = ctypes.byref(opts) if opts is not None else None
    _check(lib().did_server_create(op, ctypes.byref(s)))
    return s


def did_server_submit(s, X, M, N, K, seed, x_dtype=DID_F32) -> int:
    j = ctypes.c_int64()
    _check(lib().did_server_submit(s, _ptr(X), M, N, K, seed, x_dtype, ctypes.byref(j)))
    return j.value


def did_server_step(s):
    """One scheduling step; returns (running, queued, finished this step)."""
    r, q, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().did_server_step(s, ctypes.byref(r), ctypes.byref(q), ctypes.byref(f)))
    return r.value, q.value, f.value


def did_server_poll(s, job):
    """(state, iterations, latest objective, latency s, queueing s) of a job."""
    st, it = ctypes.c_int32(), ctypes.c_int32()
    f, lat, qs = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().did_server_poll(s, job, ctypes.byref(st), ctypes.byref(it), ctypes.byref(f), ctypes.byref(lat),
                                 ctypes.byref(qs)))
    return st.value, it.value, f.value, lat.value, qs.value


def did_server_result(s, job, B=None, C=None):
    _check(lib().did_server_result(s, job, _ptr(B), _ptr(C)))


def did_server_release(s, job):
    _check(lib().did_server_release(s, job))


def did_server_memory(s):
    u, p = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().did_server_memory(s, ctypes.byref(u), ctypes.byref(p)))
    return u.value, p.value


def did_server_arena_stats(s):
    """(arenas allocated, arenas reused from the pool, pooled arenas freed, bytes pooled)."""
    v = [ctypes.c_int64() for _ in range(4)]
    _check(lib().did_server_arena_stats(s, *(ctypes.byref(x) for x in v)))
    return tuple(x.value for x in v)


def did_server_free(s):
    _check(lib().did_server_free(s))


def did_iterate_static(X, M, N, K, B, C, n, opts=None, f=None):
    """n iterations from the caller's device factors B, C (overwritten), with every
    intermediate buffer in the library's static workspace (no device allocation).
    f: None or a device buffer of n float64 objectives."""
    op = ctypes.byref(opts) if opts is not None else None
    _check(lib().did_iterate_static(_ptr(X), M, N, K, _ptr(B), _ptr(C), n, op, _ptr(f)))


def did_debug_inject_fault(h):
    """Make the next checked call on h fail as a device error would (sticky DID_EDEVICE)."""
    _check(lib().did_debug_inject_fault(h))


def did_debug_check_guards(h):
    """(changed guard bytes past the ends of h's buffers, guard zones checked): handles made
    with the environment variable DID_DEBUG_GUARD_ZONES=1 have a zone after each buffer."""
    bad = ctypes.c_int64(0)
    zones = ctypes.c_int32(0)
    _check(lib().did_debug_check_guards(h, ctypes.byref(bad), ctypes.byref(zones)))
    return bad.value, zones.value
