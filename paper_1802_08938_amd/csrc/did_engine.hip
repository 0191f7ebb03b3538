// Host engine of libdid: the C ABI declared in include/did.h.
//
// The engine owns the device buffers of one NMF instance, validates arguments, draws the
// initial factors, and sequences the kernels of one DID iteration (Alg. 3) on a single
// HIP stream with no host round trips.  Every HIP status is checked; a runtime failure
// marks the handle sticky-failed (DID_EDEVICE).
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <iterator>
#include <string>
#include <vector>

#include "../../include/did.h"
#include "did_engine.h"
#include "did_kernels.h"

using didk::Shape;

namespace didengine {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

DeviceGuard::DeviceGuard(int dev) {
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  if (prev != dev) (void)hipSetDevice(dev);
}
DeviceGuard::~DeviceGuard() {
  int cur = -1;
  if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
}

int dev_fail(did_ctx* h, hipError_t e, const char* what) {
  if (h) h->sticky = 1;
  return fail(DID_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int dalloc_bytes(did_ctx* h, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 1;
  if (h->arena) {  // carve from the arena, 256-byte aligned, while it has room
    const size_t off = (h->arena_off + 255) & ~size_t(255);
    const size_t span = bytes + (h->guards ? (size_t)DID_GUARD_ZONE_BYTES : 0);
    if (off <= h->arena_cap && span <= h->arena_cap - off) {
      h->arena_off = off + span;
      h->dev_bytes += (int64_t)bytes;
      *p = h->arena + off;
      if (h->guards) {
        unsigned char* z = h->arena + off + bytes;
        if (hipMemsetAsync(z, DID_GUARD_BYTE, DID_GUARD_ZONE_BYTES, h->st) != hipSuccess) {
          (void)hipGetLastError();
          return fail(DID_EDEVICE, "guard zone fill failed");
        }
        h->guard_zones.emplace_back(z, (int)h->guard_zones.size());
      }
      return DID_OK;
    }
  }
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(DID_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed: " +
                                hipGetErrorString(e));
  }
  h->allocs.push_back(q);
  h->dev_bytes += (int64_t)bytes;
  *p = q;
  return DID_OK;
}

int check_handle(did_ctx* h) {
  if (!h) return fail(DID_EINVAL, "NULL handle");
  if (h->sticky) return fail(DID_EDEVICE, "handle is in a failed state after an earlier device error");
  if (h->inject_fault) {  // did_debug_inject_fault: fail as a device error would
    h->inject_fault = 0;
    return dev_fail(h, hipErrorLaunchFailure, "injected device fault (did_debug_inject_fault)");
  }
  return DID_OK;
}

int check_free_handle(did_ctx* h) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (h->batch) return fail(DID_ESTATE, "handle is a member of a batch; remove it first");
  return DID_OK;
}

}  // namespace didengine

using namespace didengine;

namespace didengine {

// Kernel stages of one iteration, in launch order.
constexpr int kStages = 8;
const char* const kStageNames[kStages] = {"column_pass", "reduce_f", "sweep_v",  "reduce_v",
                                          "row_pass",    "reduce_w", "b_update", "reduce_g"};

template <class T>
int dalloc(did_ctx* h, T** p, int64_t count) {
  void* q = nullptr;
  const int rc = dalloc_bytes(h, &q, (size_t)(count > 0 ? count : 1) * sizeof(T));
  *p = static_cast<T*>(q);
  return rc;
}

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

void release(did_ctx* h) {
  if (!h) return;
  DeviceGuard g(h->dev);
  if (h->st) (void)hipStreamSynchronize(h->st);
  if (h->st2) (void)hipStreamSynchronize(h->st2);
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  for (hipEvent_t ev : h->prof_events) (void)hipEventDestroy(ev);
  if (h->ev_c) (void)hipEventDestroy(h->ev_c);
  if (h->ev_v) (void)hipEventDestroy(h->ev_v);
  if (h->st2) (void)hipStreamDestroy(h->st2);
  h->prof_events.clear();
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
  if (h->pool && h->arena && h->arena_in_slab) {  // back to the slab, merged with free neighbours
    auto& fr = h->pool->slab_free;
    size_t off = (size_t)(h->arena - h->pool->slab), len = h->arena_cap;
    auto nx = fr.lower_bound(off);
    if (nx != fr.end() && nx->first == off + len) {
      len += nx->second;
      nx = fr.erase(nx);
    }
    if (nx != fr.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        off = pv->first;
        len += pv->second;
        fr.erase(pv);
      }
    }
    fr.emplace(off, len);
  } else if (h->pool && h->arena) {  // back to the serving loop's pool; trim its largest beyond the limit
    ArenaPool& P = *h->pool;
    P.free.emplace_back(h->arena, h->arena_cap);
    P.bytes += h->arena_cap;
    while (P.bytes > P.limit && !P.free.empty()) {
      size_t bi = 0;
      for (size_t i = 1; i < P.free.size(); ++i)
        if (P.free[i].second > P.free[bi].second) bi = i;
      (void)hipFree(P.free[bi].first);
      ++P.frees;
      P.bytes -= P.free[bi].second;
      P.free.erase(P.free.begin() + (ptrdiff_t)bi);
    }
  }
  if (h->own_stream && h->st) (void)hipStreamDestroy(h->st);
  (void)hipGetLastError();
  delete h;
}

// Parameters of the row pass's column ranges (didk::range_bounds): T tiles, P blocks (the
// paper's shards), at most S sub-ranges per block; W partials are summed in ascending
// range order.
void range_params(int64_t N, int64_t nchunks, int n_blocks, int row_blocks, int64_t* T, int64_t* P, int64_t* S) {
  *T = (N + 31) / 32;
  const int64_t slab_groups = (nchunks + 3) / 4;
  // about row_blocks blocks of (range, slab group).  The default, N / 256 within
  // [512, 4096], follows measurements across shapes: wide X wants several rounds of
  // resident blocks (5000 x 10^6: 9.77 ms per iteration at 4096 against 10.98 at 512),
  // narrower X fewer, longer ranges, whose W partials cost less to write and sum
  // (500 x 150000: 0.258 ms at 512 against 0.303 at 4096).
  const int64_t target = row_blocks > 0 ? row_blocks : std::min<int64_t>(4096, std::max<int64_t>(512, N / 256));
  int64_t want = (target + slab_groups - 1) / slab_groups;
  // at least 16 tiles (512 columns) per range: the W partials (R x KP x M floats) then
  // stay below a sixteenth of X for K <= 64
  want = std::max<int64_t>(1, std::min<int64_t>(want, std::max<int64_t>(1, *T / 16)));
  *P = n_blocks > 0 ? std::min<int64_t>(n_blocks, *T) : 1;
  *S = std::max<int64_t>(1, (want + *P - 1) / *P);
}

// The R + 1 tile bounds of the column ranges.
std::vector<int64_t> make_ranges(int64_t N, int64_t nchunks, int n_blocks, int row_blocks) {
  int64_t T, P, S;
  range_params(N, nchunks, n_blocks, row_blocks, &T, &P, &S);
  std::vector<int64_t> b((size_t)didk::range_bounds(T, P, S, nullptr) + 1);
  didk::range_bounds(T, P, S, b.data());
  return b;
}

int check_shape(int64_t M, int64_t N, int32_t K) {
  if (M < 1 || N < 1 || K < 1) return fail(DID_EINVAL, "M, N and K must be >= 1");
  if (K > DID_MAX_K) return fail(DID_EINVAL, "K > 64 is not supported");
  if ((int64_t)K > std::min(M, N)) return fail(DID_EINVAL, "K must not exceed min(M, N)");
  if (M > (int64_t(1) << 40) || N > (int64_t(1) << 40) || (double)M * (double)N >= 4.6e18)
    return fail(DID_EINVAL, "M * N is too large");
  return DID_OK;
}

// Option checks and the derived shape, shared by setup and did_mem_estimate.
int make_shape(Shape& s, int64_t M, int64_t N, int32_t K, const did_opts& o) {
  if (o.x_dtype != DID_F32 && o.x_dtype != DID_BF16) return fail(DID_EINVAL, "x_dtype must be DID_F32 or DID_BF16");
  if (o.refresh_every < 1) return fail(DID_EINVAL, "refresh_every must be >= 1");
  if (o.n_blocks < 0) return fail(DID_EINVAL, "n_blocks must be >= 0");
  if (o.row_blocks < 0) return fail(DID_EINVAL, "row_blocks must be >= 0");
  if (o.x_tiled != 0 && o.x_tiled != 1) return fail(DID_EINVAL, "x_tiled must be 0 or 1");
  s.M = M;
  s.N = N;
  s.K = K;
  s.KP = K <= 32 ? 32 : 64;
  s.nchunks = (M + 31) / 32;
  s.Mpad = s.nchunks * 32;
  s.xbf16 = o.x_dtype == DID_BF16;
  s.xtiled = s.xbf16 || o.x_tiled;
  s.thin = (M <= 16 && K <= 8 && (M <= 8 || K <= 4)) ? 1 : 0;
  if (o.algorithm != DID_ALG_DID && o.algorithm != DID_ALG_DBCD) return fail(DID_EINVAL, "unknown algorithm");
  if (o.algorithm == DID_ALG_DBCD && !s.thin)
    return fail(DID_EINVAL, "DID_ALG_DBCD runs on the thin-matrix path only (M <= 16, K <= 8, M <= 8 or K <= 4)");
  if (s.thin && s.xbf16) return fail(DID_EINVAL, "the thin-matrix path stores X as float32 only");
  if (s.thin && o.x_tiled) return fail(DID_EINVAL, "the thin-matrix path reads X as given (x_tiled must be 0)");
  // The passes address column-major X (and the carried residual) from a wave-uniform base
  // plus a 32-bit per-lane offset of up to 32 M elements: taller X must use a tiled storage.
  if (!s.thin && !s.xtiled && 32 * M > (int64_t)0xFFFFFFFF)
    return fail(DID_EINVAL, "column-major X needs 32 * M < 2^32 (32-bit lane offsets); use x_tiled = 1");
  if (o.refresh_every > 1 && s.thin)
    return fail(DID_EINVAL, "refresh_every > 1 (carried residual) runs the MFMA passes only, not the thin-matrix path");
  if (o.refresh_every > 1 && 32 * M > (int64_t)0xFFFFFFFF)
    return fail(DID_EINVAL, "the carried residual is column-major: refresh_every > 1 needs 32 * M < 2^32");
  if (o.col_waves != 0 && o.col_waves != 4 && o.col_waves != 8) return fail(DID_EINVAL, "col_waves must be 0, 4 or 8");
  if (o.col_waves == 8 && o.refresh_every > 1)
    return fail(DID_EINVAL, "the carried residual form runs the column pass with 4 waves per block");
  if (s.thin || o.refresh_every > 1)
    s.cwpb = 4;
  else
    s.cwpb = o.col_waves ? o.col_waves : tuned_col_waves(M, N, s.KP, didk::x_kind(s));
  if (s.thin && (s.thin_grid = didk::thin_grid_for(s)) < 1)
    return fail(DID_EDEVICE, "thin path: occupancy query failed");
  return DID_OK;
}

// Row-pass target of an instance: the option, else the tuned value for its shape class,
// else the default.
int row_target(const Shape& s, const did_opts& o) {
  if (o.row_blocks > 0) return o.row_blocks;
  return didengine::tuned_row_blocks(s.M, s.N, s.KP, didk::x_kind(s));
}

// Device bytes the engine allocates for an instance (the plan setup follows).
int64_t engine_bytes(const Shape& s, int R, bool x_copied, int refresh) {
  const int64_t M = s.M, N = s.N, K = s.K, KP = s.KP, NP = didk::n_pairs(s.KP);
  auto b = [](int64_t n) { return n > 0 ? n : 1; };
  int64_t t = b(4);  // flag
  if (s.xtiled)
    t += b(2 * didk::tiled_x_elems(s) * (s.xbf16 ? 2 : 4));
  else if (x_copied)
    t += b(M * N * 4);
  t += b(M * K * 4) + b(K * N * 4) + b(didk::packed_b_elems(s) * 2) + b(didk::bsc_floats(s.KP) * 4) + b(KP * KP * 8) +
       b((int64_t)didk::bupdate_blocks(s) * NP * 8) + b(KP * KP * 8) + b(KP * s.Mpad * 8);
  if (s.thin) {
    t += b(didk::thin_blocks(s) * didk::thin_slots_for(s) * 8);
  } else {
    t += b(didk::vgram_blocks(s) * NP * 8) + b(KP * N * 4) + b(didk::cq_bytes(s)) + b(didk::bsc_floats(s.KP) * 4) + b((int64_t)R * KP * s.Mpad * 4) +
         b((int64_t)(R + 1) * 8) + b(didk::colpass_blocks(s) * 8);
  }
  t += b(kHistCap * 8) + b(8) + b(8);  // fhist, fobj, tdev
  if (refresh > 1) t += b(M * N * 4) + b(didk::packed_b_elems(s) * 2) + b(didk::cqd_bytes(s));  // R, BqD, CqD
  return t;
}

// Allocate, copy/adopt X and validate it.  Leaves h ready for factor setup.
int setup(did_ctx* h, const void* Xv, int64_t M, int64_t N, int32_t K, const did_opts& o) {
  int rc;
  Shape& s = h->s;
  if ((rc = make_shape(s, M, N, K, o))) return rc;
  h->algorithm = o.algorithm;
  if (hipGetDevice(&h->dev) != hipSuccess) return fail(DID_EDEVICE, "no HIP device");
  {  // the arena: the engine's bytes for this instance plus alignment slack per buffer
    const char* gz = getenv("DID_DEBUG_GUARD_ZONES");
    h->guards = gz && atoi(gz) != 0;
    const bool xdev0 = is_device_ptr(Xv);
    const bool x_copied = !s.xtiled && !(xdev0 && o.borrow_x);
    const int R0 = s.thin ? 1 : (int)make_ranges(N, s.nchunks, o.n_blocks, row_target(s, o)).size() - 1;
    const size_t cap = (size_t)engine_bytes(s, R0, x_copied, o.refresh_every) +
                       64 * (256 + (h->guards ? (size_t)DID_GUARD_ZONE_BYTES : 0));
    void* q = nullptr;
    size_t qcap = cap;
    bool pooled = false;
    if (h->pool && h->pool->slab) {  // first fit in the slab
      auto& fr = h->pool->slab_free;
      const size_t need = (cap + 255) & ~size_t(255);
      for (auto it = fr.begin(); it != fr.end(); ++it) {
        if (it->second < need) continue;
        const size_t off = it->first, len = it->second;
        fr.erase(it);
        if (len > need) fr.emplace(off + need, len - need);
        q = h->pool->slab + off;
        qcap = need;
        h->arena_in_slab = true;
        pooled = true;
        ++h->pool->reuses;
        break;
      }
    }
    if (h->pool && !q) {  // the smallest pooled arena that fits without wasting more than half of it
      size_t bi = h->pool->free.size();
      for (size_t i = 0; i < h->pool->free.size(); ++i) {
        const size_t c = h->pool->free[i].second;
        if (c >= cap && c <= cap + cap / 2 && (bi == h->pool->free.size() || c < h->pool->free[bi].second)) bi = i;
      }
      if (bi < h->pool->free.size()) {
        q = h->pool->free[bi].first;
        qcap = h->pool->free[bi].second;
        h->pool->bytes -= qcap;
        h->pool->free.erase(h->pool->free.begin() + (ptrdiff_t)bi);
        ++h->pool->reuses;
        pooled = true;
      }
    }
    if (!q && hipMalloc(&q, cap) != hipSuccess) {
      (void)hipGetLastError();
      q = nullptr;
      // pooled arenas are idle (their handles' streams were drained at release) and are not
      // charged to the serving budget: give them back to the device and try once more, so
      // that the pool never makes an admission fail that would succeed without it
      if (h->pool && !h->pool->free.empty()) {
        pool_free_all(h->pool);
        if (hipMalloc(&q, cap) != hipSuccess) {
          (void)hipGetLastError();
          q = nullptr;
        }
      }
      if (!q) return fail(DID_ENOMEM, "device allocation of " + std::to_string(cap) + " bytes failed");
    }
    if (!h->pool) h->allocs.push_back(q);  // a pooled arena goes back to the pool at release
    else if (!pooled) ++h->pool->allocs;
    h->arena = static_cast<unsigned char*>(q);
    h->arena_cap = qcap;
    h->arena_off = 0;
  }
  if (o.stream) {
    h->st = static_cast<hipStream_t>(o.stream);
  } else {
    hipError_t e = hipStreamCreateWithFlags(&h->st, hipStreamNonBlocking);
    if (e != hipSuccess) return dev_fail(nullptr, e, "hipStreamCreate");
    h->own_stream = true;
  }

  // float32 view of X on the device: the caller's device buffer (borrowed, or read once for
  // the bf16 form) or an upload
  if ((rc = dalloc(h, &h->flag, 1))) return rc;
  hipError_t e;
  const bool xdev = is_device_ptr(Xv);
  const float* xin = nullptr;
  float* xtmp = nullptr;  // temporary upload for the tiled forms, freed below
  if (xdev && (o.borrow_x || s.xtiled)) {
    xin = static_cast<const float*>(Xv);
    h->own_x = !s.xtiled ? false : true;
  } else if (!s.xtiled) {
    float* xc = nullptr;
    if ((rc = dalloc(h, &xc, M * N))) return rc;
    if ((e = hipMemcpyAsync(xc, Xv, (size_t)(M * N) * sizeof(float), hipMemcpyDefault, h->st)) != hipSuccess)
      return dev_fail(h, e, "copy of X");
    xin = xc;
  } else {
    if ((e = hipMalloc(&xtmp, (size_t)(M * N) * sizeof(float))) != hipSuccess) {
      (void)hipGetLastError();
      return fail(DID_ENOMEM, "device allocation for the upload of X failed");
    }
    if ((e = hipMemcpyAsync(xtmp, Xv, (size_t)(M * N) * sizeof(float), hipMemcpyDefault, h->st)) != hipSuccess) {
      (void)hipFree(xtmp);
      return dev_fail(h, e, "copy of X");
    }
    xin = xtmp;
  }
  if (h->defer_checks && !xtmp) {  // X must be finite and nonnegative: checked later
    const int v4 = (M % 4 == 0) && ((reinterpret_cast<uintptr_t>(xin) & 15) == 0);
    if ((e = hipMemsetAsync(h->flag, 0, sizeof(int), h->st)) != hipSuccess ||
        (e = didk::validate(xin, M * N, v4, h->flag, h->st)) != hipSuccess)
      return dev_fail(h, e, "validate X");
    h->x_check_pending = true;
  } else {  // X must be finite and nonnegative
    const int v4 = (M % 4 == 0) && ((reinterpret_cast<uintptr_t>(xin) & 15) == 0);
    int flag = 0;
    if ((e = hipMemsetAsync(h->flag, 0, sizeof(int), h->st)) != hipSuccess ||
        (e = didk::validate(xin, M * N, v4, h->flag, h->st)) != hipSuccess ||
        (e = hipMemcpyAsync(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->st)) != hipSuccess ||
        (e = hipStreamSynchronize(h->st)) != hipSuccess) {
      if (xtmp) (void)hipFree(xtmp);
      return dev_fail(h, e, "validate X");
    }
    if (flag) {
      if (xtmp) (void)hipFree(xtmp);
      return fail(DID_EINVAL, "X must be finite and nonnegative");
    }
  }
  if (s.xtiled) {  // the two tiled copies (one per pass) in one allocation
    unsigned char* xb = nullptr;
    const int64_t te = didk::tiled_x_elems(s), esz = s.xbf16 ? 2 : 4;
    if ((rc = dalloc(h, &xb, 2 * te * esz))) {
      if (xtmp) (void)hipFree(xtmp);
      return rc;
    }
    e = didk::tile_x(s, xin, xb, xb + te * esz, h->st);
    if (e == hipSuccess && (xtmp || !h->defer_checks)) e = hipStreamSynchronize(h->st);
    if (xtmp) (void)hipFree(xtmp);
    if (e != hipSuccess) return dev_fail(h, e, "tiled storage of X");
    h->X = xb;
    h->XR = xb + te * esz;
    s.vec4 = 0;  // the tiled copies are read with their own full-width loads
  } else {
    h->X = const_cast<float*>(xin);
    h->XR = h->X;
    s.vec4 = (M % 4 == 0) && ((reinterpret_cast<uintptr_t>(xin) & 15) == 0);
  }

  const int NP = didk::n_pairs(s.KP);
  const std::vector<int64_t> rb = make_ranges(N, s.nchunks, o.n_blocks, row_target(s, o));
  h->R = (int)rb.size() - 1;
  if ((rc = dalloc(h, &h->B, M * K))) return rc;
  if ((rc = dalloc(h, &h->C, (int64_t)K * N))) return rc;
  if ((rc = dalloc(h, &h->Bq, didk::packed_b_elems(s)))) return rc;
  if ((rc = dalloc(h, &h->Bsc, didk::bsc_floats(s.KP)))) return rc;
  if ((rc = dalloc(h, &h->G, (int64_t)s.KP * s.KP))) return rc;
  if ((rc = dalloc(h, &h->Gpart, (int64_t)didk::bupdate_blocks(s) * NP))) return rc;
  if ((rc = dalloc(h, &h->V, (int64_t)s.KP * s.KP))) return rc;
  if ((rc = dalloc(h, &h->W, (int64_t)s.KP * s.Mpad))) return rc;
  if (s.thin) {
    if ((rc = dalloc(h, &h->tpart, didk::thin_blocks(s) * didk::thin_slots_for(s)))) return rc;
  } else {
    if ((rc = dalloc(h, &h->Vpart, didk::vgram_blocks(s) * NP))) return rc;
    if ((rc = dalloc(h, &h->H, (int64_t)s.KP * N))) return rc;
    unsigned char* cq = nullptr;
    if ((rc = dalloc(h, &cq, didk::cq_bytes(s)))) return rc;
    h->Cq = cq;
    if ((rc = dalloc(h, &h->Csc, didk::bsc_floats(s.KP)))) return rc;
    if ((rc = dalloc(h, &h->Wpart, (int64_t)h->R * s.KP * s.Mpad))) return rc;
    if ((rc = dalloc(h, &h->rbounds, (int64_t)rb.size()))) return rc;
    if ((rc = dalloc(h, &h->fpart, didk::colpass_blocks(s)))) return rc;
  }
  if ((rc = dalloc(h, &h->fhist, kHistCap))) return rc;
  if ((rc = dalloc(h, &h->fobj, 1))) return rc;
  if ((rc = dalloc(h, &h->tdev, 1))) return rc;
  h->refresh = o.refresh_every;
  if (h->refresh > 1) {
    if ((rc = dalloc(h, &h->Rres, M * N))) return rc;
    if ((rc = dalloc(h, &h->BqD, didk::packed_b_elems(s)))) return rc;
    unsigned char* cqd = nullptr;
    if ((rc = dalloc(h, &cqd, didk::cqd_bytes(s)))) return rc;
    h->CqD = cqd;
    if ((e = hipMemsetAsync(h->BqD, 0, (size_t)didk::packed_b_elems(s) * 2, h->st)) != hipSuccess ||
        (e = hipMemsetAsync(h->CqD, 0, (size_t)didk::cqd_bytes(s), h->st)) != hipSuccess)
      return dev_fail(h, e, "buffer setup");
  }

  if ((e = hipMemsetAsync(h->Bq, 0, (size_t)didk::packed_b_elems(s) * 2, h->st)) != hipSuccess ||
      (e = hipMemsetAsync(h->Bsc, 0, (size_t)didk::bsc_floats(s.KP) * 4, h->st)) != hipSuccess ||
      (e = hipMemsetAsync(h->V, 0, (size_t)s.KP * s.KP * 8, h->st)) != hipSuccess ||
      (e = hipMemsetAsync(h->W, 0, (size_t)s.KP * s.Mpad * 8, h->st)) != hipSuccess ||
      (!h->x_check_pending && (e = hipMemsetAsync(h->flag, 0, sizeof(int), h->st)) != hipSuccess) ||
      (e = hipMemsetAsync(h->tdev, 0, sizeof(int64_t), h->st)) != hipSuccess)
    return dev_fail(h, e, "buffer setup");
  if (!s.thin &&
      ((e = hipMemsetAsync(h->Cq, 0, (size_t)didk::cq_bytes(s), h->st)) != hipSuccess ||
       (e = hipMemsetAsync(h->Csc, 0, (size_t)didk::bsc_floats(s.KP) * 4, h->st)) != hipSuccess ||
       (e = hipMemcpyAsync(h->rbounds, rb.data(), rb.size() * sizeof(int64_t), hipMemcpyHostToDevice, h->st)) !=
           hipSuccess))
    return dev_fail(h, e, "buffer setup");
  return DID_OK;
}

// Pack B and form G = B^T B.
hipError_t refresh_b_derived(did_ctx* h) {
  hipError_t e = didk::bupdate(h->s, h->B, h->W, h->V, h->Bq, h->Bsc, h->Gpart, 0, h->st);
  if (e != hipSuccess) return e;
  return didk::reduce_sym(h->Gpart, didk::bupdate_blocks(h->s), h->s.KP, h->G, h->st);
}

int objective_pass(did_ctx* h) {
  hipError_t e;
  if (h->s.thin) {
    if ((e = didk::thin_pass(h->s, static_cast<const float*>(h->X), h->B, h->G, h->C, h->tpart, 1, h->st)) !=
            hipSuccess ||
        (e = didk::thin_reduce(h->s, h->tpart, h->W, h->V, h->fobj, 0.5, 0, h->st)) != hipSuccess)
      return dev_fail(h, e, "objective pass");
    return DID_OK;
  }
  if ((e = didk::colpass(h->s, h->X, h->Cq, h->Bq, h->Bsc, h->H, h->fpart, 0, h->st)) != hipSuccess)
    return dev_fail(h, e, "objective pass");
  if ((e = didk::reduce_f(h->fpart, didk::colpass_blocks(h->s), h->fobj, 0.5, h->st)) != hipSuccess)
    return dev_fail(h, e, "objective reduce");
  return DID_OK;
}

// Repack C after it was changed outside the sweep (the thin path keeps no packed copy).
hipError_t pack_c(did_ctx* h) {
  if (h->s.thin) return hipSuccess;
  return didk::packc(h->s, h->C, h->Cq, h->Csc, h->st);
}

int apply_init_scale(did_ctx* h) {
  // alpha minimising f over a common scale: f(a) = f0 - b a + c a^2 / 2 evaluated at
  // a = 1, 2, 4 by scaling C exactly by powers of two.
  double fv[3];
  const float mul[3] = {1.0f, 2.0f, 2.0f};
  const int64_t nC = (int64_t)h->s.K * h->s.N;
  hipError_t e;
  for (int q = 0; q < 3; ++q) {
    if (q && ((e = didk::scale(h->C, nC, mul[q], h->st)) != hipSuccess ||
              (e = pack_c(h)) != hipSuccess))
      return dev_fail(h, e, "init scale");
    int rc = objective_pass(h);
    if (rc) return rc;
    if ((e = hipMemcpyAsync(&fv[q], h->fobj, sizeof(double), hipMemcpyDeviceToHost, h->st)) != hipSuccess ||
        (e = hipStreamSynchronize(h->st)) != hipSuccess)
      return dev_fail(h, e, "init scale");
  }
  if ((e = didk::scale(h->C, nC, 0.25f, h->st)) != hipSuccess ||
      (e = pack_c(h)) != hipSuccess)
    return dev_fail(h, e, "init scale");
  const double c = (fv[2] - 3.0 * fv[1] + 2.0 * fv[0]) / 3.0;
  const double b = 1.5 * c - (fv[1] - fv[0]);
  if (c > 0.0 && b > 0.0 && std::isfinite(b / c)) {
    const float r = (float)std::sqrt(b / c);
    if ((e = didk::scale(h->C, nC, r, h->st)) != hipSuccess ||
        (e = didk::scale(h->B, h->s.M * h->s.K, r, h->st)) != hipSuccess ||
        (e = refresh_b_derived(h)) != hipSuccess || (e = pack_c(h)) != hipSuccess)
      return dev_fail(h, e, "init scale");
  }
  return DID_OK;
}

int init_common(const void* X, int64_t M, int64_t N, int32_t K, uint64_t seed, const float* B0, const float* C0,
                const did_opts* opts, did_handle* out, bool defer = false, ArenaPool* pool = nullptr) {
  if (!out) return fail(DID_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (!X) return fail(DID_EINVAL, "X must not be NULL");
  int rc = check_shape(M, N, K);
  if (rc) return rc;
  did_opts o;
  did_default_opts(&o);
  if (opts) o = *opts;
  did_ctx* h = new (std::nothrow) did_ctx();
  if (!h) return fail(DID_ENOMEM, "host allocation failed");
  h->defer_checks = defer && !B0;
  h->pool = pool;
  if ((rc = setup(h, X, M, N, K, o))) {
    release(h);
    return rc;
  }
  hipError_t e;
  if (B0) {
    if ((e = hipMemcpyAsync(h->B, B0, (size_t)(M * K) * 4, hipMemcpyDefault, h->st)) != hipSuccess ||
        (e = hipMemcpyAsync(h->C, C0, (size_t)((int64_t)K * N) * 4, hipMemcpyDefault, h->st)) != hipSuccess) {
      rc = dev_fail(h, e, "copy of B, C");
      release(h);
      return rc;
    }
    int flag = 0;
    if ((e = didk::validate(h->B, M * K, 0, h->flag, h->st)) != hipSuccess ||
        (e = didk::validate(h->C, (int64_t)K * N, 0, h->flag, h->st)) != hipSuccess ||
        (e = hipMemcpyAsync(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->st)) != hipSuccess ||
        (e = hipStreamSynchronize(h->st)) != hipSuccess) {
      rc = dev_fail(h, e, "validate B, C");
      release(h);
      return rc;
    }
    if (flag) {
      release(h);
      return fail(DID_EINVAL, "B and C must be finite and nonnegative");
    }
  } else {
    if ((e = didk::fill_uniform(h->B, M * K, didk::stream_key(seed, 1), h->st)) != hipSuccess ||
        (e = didk::fill_uniform(h->C, (int64_t)K * N, didk::stream_key(seed, 2), h->st)) != hipSuccess) {
      rc = dev_fail(h, e, "initial draw");
      release(h);
      return rc;
    }
  }
  if ((e = refresh_b_derived(h)) != hipSuccess || (e = pack_c(h)) != hipSuccess) {
    rc = dev_fail(h, e, "pack B, C");
    release(h);
    return rc;
  }
  if (!B0 && o.init_scale) {
    if ((rc = apply_init_scale(h))) {
      release(h);
      return rc;
    }
  }
  // deferred: the draw and packing stay queued ahead of everything the handle does next
  if ((e = h->defer_checks ? hipGetLastError() : hipStreamSynchronize(h->st)) != hipSuccess) {
    rc = dev_fail(h, e, "init");
    release(h);
    return rc;
  }
  *out = h;
  g_err.clear();
  return DID_OK;
}

int init_deferred(const void* X, int64_t M, int64_t N, int32_t K, uint64_t seed, const did_opts* opts,
                  did_handle* out, ArenaPool* pool) {
  return init_common(X, M, N, K, seed, nullptr, nullptr, opts, out, true, pool);
}

int pool_reserve_slab(ArenaPool* pool, size_t bytes) {
  bytes &= ~size_t(255);
  void* p = nullptr;
  if (bytes == 0) return DID_OK;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(DID_ENOMEM, "device allocation of the " + std::to_string(bytes) + "-byte arena reserve failed");
  }
  pool->slab = static_cast<unsigned char*>(p);
  pool->slab_cap = bytes;
  pool->slab_free.clear();
  pool->slab_free.emplace(0, bytes);
  return DID_OK;
}

void pool_free_slab(ArenaPool* pool) {
  if (!pool || !pool->slab) return;
  (void)hipFree(pool->slab);
  pool->slab = nullptr;
  pool->slab_cap = 0;
  pool->slab_free.clear();
}

void pool_free_all(ArenaPool* pool) {
  if (!pool) return;
  for (auto& a : pool->free) (void)hipFree(a.first);
  pool->frees += (int64_t)pool->free.size();
  pool->free.clear();
  pool->bytes = 0;
}

int check_deferred(did_ctx* h) {
  int rc = check_handle(h);
  if (rc) return rc;
  DeviceGuard g(h->dev);
  hipError_t e;
  if ((e = hipStreamSynchronize(h->st)) != hipSuccess) return dev_fail(h, e, "set-up");
  if (!h->x_check_pending) return DID_OK;
  int flag = 0;
  if ((e = hipMemcpy(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess)
    return dev_fail(h, e, "validate X");
  h->x_check_pending = false;
  if (flag) return fail(DID_EINVAL, "X must be finite and nonnegative");
  return DID_OK;
}

// One iteration of the MFMA path on the buffers of h, enqueued on h->st (and, unless
// one_stream, the V stages on h->st2), with a profiling event before the first and after
// every stage when ev is given.  The objective goes to fhist at the device iteration
// counter tdev, so the launches carry no host iteration index (the same launches can be
// captured once and replayed).
static int enqueue_iteration(did_ctx* h, hipEvent_t* ev, bool one_stream = false) {
  const Shape& s = h->s;
  hipError_t e;
#define DID_MARK(q) \
  if (ev && (e = hipEventRecord(ev[q], h->st)) != hipSuccess) return dev_fail(h, e, "profile record")
  // carried residual (refresh_every > 1): the column pass refreshes R from X every
  // refresh_every iterations and otherwise carries it (E = R - delta B C)
  const bool carry = h->refresh > 1;
  DID_MARK(0);
  if (carry)
    e = didk::colpass_carry(s, h->X, h->t % h->refresh == 0, h->Cq, h->Bq, h->BqD, h->Bsc, h->H, h->fpart, h->Rres,
                            h->st);
  else
    e = didk::colpass(s, h->X, h->Cq, h->Bq, h->Bsc, h->H, h->fpart, 1, h->st);
  if (e != hipSuccess) return dev_fail(h, e, "column pass");
  DID_MARK(1);
  if ((e = didk::reduce_f_hist(h->fpart, didk::colpass_blocks(s), h->fhist, h->hist_cap, h->tdev, 0.5, h->st)) !=
      hipSuccess)
    return dev_fail(h, e, "objective reduce");
  DID_MARK(2);
  if ((e = didk::sweep(s, h->H, h->C, h->Cq, h->Csc, h->G, h->st, carry ? h->CqD : nullptr)) != hipSuccess)
    return dev_fail(h, e, "sweep");
  // V = tril(C'C'^T), on the second stream when there is one (overlapped with the row pass
  // and the W reduction; the B update waits for it)
  hipStream_t st2 = one_stream ? nullptr : h->st2;
  hipStream_t sv = h->st;
  if (st2) {
    if ((e = hipEventRecord(h->ev_c, h->st)) != hipSuccess ||
        (e = hipStreamWaitEvent(st2, h->ev_c, 0)) != hipSuccess)
      return dev_fail(h, e, "stream order");
    sv = st2;
  }
  if ((e = didk::vgram(s, h->Cq, h->Csc, h->Vpart, sv)) != hipSuccess) return dev_fail(h, e, "V partials");
  if ((e = didk::reduce_sym(h->Vpart, didk::vgram_blocks(s), s.KP, h->V, sv)) != hipSuccess)
    return dev_fail(h, e, "V reduce");
  if (st2 && (e = hipEventRecord(h->ev_v, st2)) != hipSuccess) return dev_fail(h, e, "stream order");
  DID_MARK(3);
  DID_MARK(4);
  if (carry)
    e = didk::rowpass_carry(s, h->Rres, h->Cq, h->CqD, h->Csc, h->Bq, h->Wpart, h->rbounds, h->R, h->st);
  else
    e = didk::rowpass(s, h->XR, h->Cq, h->Csc, h->Bq, h->Wpart, h->rbounds, h->R, h->st);
  if (e != hipSuccess) return dev_fail(h, e, "row pass");
  DID_MARK(5);
  if ((e = didk::reduce_w(s, h->Wpart, h->R, h->W, h->st)) != hipSuccess) return dev_fail(h, e, "W reduce");
  DID_MARK(6);
  if (st2 && (e = hipStreamWaitEvent(h->st, h->ev_v, 0)) != hipSuccess) return dev_fail(h, e, "stream order");
  if ((e = didk::bupdate(s, h->B, h->W, h->V, h->Bq, h->Bsc, h->Gpart, 1, h->st, carry ? h->BqD : nullptr)) !=
      hipSuccess)
    return dev_fail(h, e, "B update");
  DID_MARK(7);
  if ((e = didk::reduce_sym(h->Gpart, didk::bupdate_blocks(s), s.KP, h->G, h->st)) != hipSuccess)
    return dev_fail(h, e, "G reduce");
  DID_MARK(8);
#undef DID_MARK
  return DID_OK;
}

// Iterations of the MFMA path on the buffers of h (shared by did_iterate and the
// allocation-free did_iterate_static).  With a second stream (h->st2) the V partials and
// their reduction overlap the row pass; without one they run in order on h->st.  Without
// profiling, two or more iterations of the refresh-every-iteration form replay one
// captured iteration (a hipGraph kept by the handle), which removes the host launch cost
// that bounds small shapes.  The captured iteration runs on h->st alone: a capture that
// forks onto a second stream and joins back left the device memory its kernels use
// allocated after hipGraphExecDestroy and hipFree (measured on ROCm 7.2), so the V stages
// give up their overlap with the row pass there.
int iterate_mfma(did_ctx* h, int32_t n) {
  hipError_t e;
  if (n <= 0) return DID_OK;
  if (h->use_graph && !h->profiling && h->refresh == 1 && n >= 2) {
    if (!h->gexec && !h->graph_failed) {
      hipGraph_t g = nullptr;
      if ((e = hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        (void)hipGetLastError();
        h->graph_failed = true;
      } else {
        const int rc = enqueue_iteration(h, nullptr, true);
        e = hipStreamEndCapture(h->st, &g);
        if (rc) {
          if (g) (void)hipGraphDestroy(g);
          return rc;
        }
        if (e != hipSuccess || !g || hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
          (void)hipGetLastError();
          h->gexec = nullptr;
          h->graph_failed = true;
        }
        if (g) (void)hipGraphDestroy(g);
      }
    }
    if (h->gexec) {
      for (int32_t it = 0; it < n; ++it)
        if ((e = hipGraphLaunch(h->gexec, h->st)) != hipSuccess) return dev_fail(h, e, "iteration graph launch");
      h->t += n;
      return DID_OK;
    }
  }
  // the second stream and its events, made on the first eager iteration (a handle that only
  // replays its graph or runs inside a batch never needs them)
  if (!h->st2 && h->may_create_st2) {
    if ((e = hipStreamCreateWithFlags(&h->st2, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&h->ev_c, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&h->ev_v, hipEventDisableTiming)) != hipSuccess)
      return dev_fail(h, e, "second stream");
  }
  for (int32_t it = 0; it < n; ++it) {
    hipEvent_t* ev = nullptr;
    if (h->profiling) {
      const size_t base = h->prof_events.size();
      h->prof_events.resize(base + kStages + 1, nullptr);
      for (int q = 0; q <= kStages; ++q)
        if ((e = hipEventCreate(&h->prof_events[base + q])) != hipSuccess) return dev_fail(h, e, "profile event");
      ev = h->prof_events.data() + base;
    }
    const int rc = enqueue_iteration(h, ev);
    if (rc) return rc;
    ++h->t;
  }
  return DID_OK;
}

}  // namespace didengine

extern "C" {

int did_default_opts(did_opts* o) {
  if (!o) return fail(DID_EINVAL, "opts must not be NULL");
  memset(o, 0, sizeof(*o));
  o->n_blocks = 0;
  o->x_dtype = DID_F32;
  o->refresh_every = 1;
  o->init_scale = 0;
  o->borrow_x = 0;
  o->algorithm = DID_ALG_DID;
  o->stream = nullptr;
  return DID_OK;
}

int did_init(const float* X, int64_t M, int64_t N, int32_t K, uint64_t seed, did_handle* out) {
  return init_common(X, M, N, K, seed, nullptr, nullptr, nullptr, out);
}

int did_init_ex(const void* X, int64_t M, int64_t N, int32_t K, uint64_t seed, const did_opts* opts,
                did_handle* out) {
  return init_common(X, M, N, K, seed, nullptr, nullptr, opts, out);
}

int did_init_from_factors(const void* X, int64_t M, int64_t N, int32_t K, const float* B, const float* C,
                          const did_opts* opts, did_handle* out) {
  if (!B || !C) {
    if (out) *out = nullptr;
    return fail(DID_EINVAL, "B and C must not be NULL");
  }
  return init_common(X, M, N, K, 0, B, C, opts, out);
}

// Thin-matrix iterations.  DID: one fused column pass (sweep, W/V/f partials), their
// fixed-order reduction, the B update and G.  DBCD: the C half, then per column of B one
// pass over X and one reduction, then G.  Stages are recorded at the same positions as the
// main path's (column_pass, reduce_f/_v/_w, b_update, reduce_g); unused ones are empty.
static int iterate_thin(did_ctx* h, int32_t n) {
  const Shape& s = h->s;
  hipError_t e;
  const float* X = static_cast<const float*>(h->X);
  for (int32_t it = 0; it < n; ++it) {
    hipEvent_t* ev = nullptr;
    if (h->profiling) {
      const size_t base = h->prof_events.size();
      h->prof_events.resize(base + kStages + 1, nullptr);
      for (int q = 0; q <= kStages; ++q)
        if ((e = hipEventCreate(&h->prof_events[base + q])) != hipSuccess) return dev_fail(h, e, "profile event");
      ev = h->prof_events.data() + base;
    }
    auto mark = [&](int q) { return ev ? hipEventRecord(ev[q], h->st) : hipSuccess; };
    if ((e = mark(0)) != hipSuccess) return dev_fail(h, e, "profile record");
    const int mode = h->algorithm == DID_ALG_DBCD ? 2 : 0;
    if ((e = didk::thin_pass(s, X, h->B, h->G, h->C, h->tpart, mode, h->st)) != hipSuccess)
      return dev_fail(h, e, "thin column pass");
    if ((e = mark(1)) != hipSuccess) return dev_fail(h, e, "profile record");
    if ((e = didk::thin_reduce(s, h->tpart, h->W, h->V, h->fhist + (h->t % h->hist_cap), 0.5, mode == 0, h->st)) !=
        hipSuccess)
      return dev_fail(h, e, "thin reduce");
    // the thin path has no separate sweep, V or row pass: their stages are empty
    for (int q = 2; q <= 6; ++q)
      if ((e = mark(q)) != hipSuccess) return dev_fail(h, e, "profile record");
    if (mode == 0) {
      if ((e = didk::bupdate(s, h->B, h->W, h->V, h->Bq, h->Bsc, h->Gpart, 1, h->st)) != hipSuccess)
        return dev_fail(h, e, "B update");
    } else {
      for (int i = 0; i < s.K; ++i)
        if ((e = didk::dbcd_b_step(s, X, h->B, h->C, h->tpart, h->W, i, h->st)) != hipSuccess)
          return dev_fail(h, e, "DBCD B step");
      if ((e = didk::bupdate(s, h->B, h->W, h->V, h->Bq, h->Bsc, h->Gpart, 0, h->st)) != hipSuccess)
        return dev_fail(h, e, "pack B");
    }
    if ((e = mark(7)) != hipSuccess) return dev_fail(h, e, "profile record");
    if ((e = didk::reduce_sym(h->Gpart, didk::bupdate_blocks(s), s.KP, h->G, h->st)) != hipSuccess)
      return dev_fail(h, e, "G reduce");
    if ((e = mark(8)) != hipSuccess) return dev_fail(h, e, "profile record");
    ++h->t;
  }
  return DID_OK;
}

int did_iterate(did_handle h, int32_t n) {
  int rc = check_free_handle(h);
  if (rc) return rc;
  if (n < 0) return fail(DID_EINVAL, "n must be >= 0");
  DeviceGuard g(h->dev);
  if (h->s.thin) return iterate_thin(h, n);
  return iterate_mfma(h, n);
}

int did_objective(did_handle h, double* f) {
  int rc = check_free_handle(h);
  if (rc) return rc;
  if (!f) return fail(DID_EINVAL, "f must not be NULL");
  DeviceGuard g(h->dev);
  if ((rc = objective_pass(h))) return rc;
  hipError_t e;
  if ((e = hipMemcpyAsync(f, h->fobj, sizeof(double), hipMemcpyDeviceToHost, h->st)) != hipSuccess ||
      (e = hipStreamSynchronize(h->st)) != hipSuccess)
    return dev_fail(h, e, "objective");
  return DID_OK;
}

int did_factors(did_handle h, float* B, float* C) {
  int rc = check_free_handle(h);
  if (rc) return rc;
  DeviceGuard g(h->dev);
  hipError_t e;
  if (B && (e = hipMemcpyAsync(B, h->B, (size_t)(h->s.M * h->s.K) * 4, hipMemcpyDefault, h->st)) != hipSuccess)
    return dev_fail(h, e, "copy of B");
  if (C && (e = hipMemcpyAsync(C, h->C, (size_t)((int64_t)h->s.K * h->s.N) * 4, hipMemcpyDefault, h->st)) !=
               hipSuccess)
    return dev_fail(h, e, "copy of C");
  if ((e = hipStreamSynchronize(h->st)) != hipSuccess) return dev_fail(h, e, "factors");
  return DID_OK;
}

int did_history(did_handle h, double* f, int64_t cap, int64_t* count) {
  int rc = check_free_handle(h);
  if (rc) return rc;
  if (!count) return fail(DID_EINVAL, "count must not be NULL");
  if (cap < 0 || (cap > 0 && !f)) return fail(DID_EINVAL, "bad output buffer");
  DeviceGuard g(h->dev);
  const int64_t avail = std::min<int64_t>(h->t, kHistCap);
  *count = h->t;
  const int64_t ncopy = std::min<int64_t>(cap, avail);
  hipError_t e;
  if (ncopy > 0) {
    if (h->t > kHistCap) return fail(DID_ESTATE, "objective history wrapped (more than 65536 iterations)");
    if ((e = hipMemcpyAsync(f, h->fhist, (size_t)ncopy * sizeof(double), hipMemcpyDeviceToHost, h->st)) !=
        hipSuccess)
      return dev_fail(h, e, "history");
  }
  if ((e = hipStreamSynchronize(h->st)) != hipSuccess) return dev_fail(h, e, "history");
  return DID_OK;
}

int did_iterations(did_handle h, int64_t* t) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!t) return fail(DID_EINVAL, "t must not be NULL");
  *t = h->t;
  return DID_OK;
}

int did_sync(did_handle h) {
  int rc = check_free_handle(h);
  if (rc) return rc;
  DeviceGuard g(h->dev);
  hipError_t e = hipStreamSynchronize(h->st);
  if (e != hipSuccess) return dev_fail(h, e, "sync");
  return DID_OK;
}

int did_profile(did_handle h, int32_t enable) {
  int rc = check_free_handle(h);
  if (rc) return rc;
  h->profiling = enable != 0;
  return DID_OK;
}

int did_profile_read(did_handle h, double* ms, int32_t cap, int32_t* n_stages, int64_t* n_iters) {
  int rc = check_free_handle(h);
  if (rc) return rc;
  if (!n_stages || !n_iters || cap < 0 || (cap > 0 && !ms)) return fail(DID_EINVAL, "bad output arguments");
  DeviceGuard g(h->dev);
  hipError_t e = hipStreamSynchronize(h->st);
  if (e != hipSuccess) return dev_fail(h, e, "profile sync");
  const size_t per = kStages + 1;
  const int64_t iters = (int64_t)(h->prof_events.size() / per);
  double acc[kStages] = {0};
  for (int64_t it = 0; it < iters; ++it)
    for (int q = 0; q < kStages; ++q) {
      float t = 0.0f;
      if ((e = hipEventElapsedTime(&t, h->prof_events[it * per + q], h->prof_events[it * per + q + 1])) !=
          hipSuccess)
        return dev_fail(h, e, "profile read");
      acc[q] += t;
    }
  for (hipEvent_t ev : h->prof_events) (void)hipEventDestroy(ev);
  h->prof_events.clear();
  for (int q = 0; q < kStages && q < cap; ++q) ms[q] = acc[q];
  *n_stages = kStages;
  *n_iters = iters;
  return DID_OK;
}

const char* did_stage_name(int32_t stage) {
  return (stage >= 0 && stage < kStages) ? kStageNames[stage] : "";
}

int did_free(did_handle h) {
  if (!h) return DID_OK;
  if (h->batch) return fail(DID_ESTATE, "handle is a member of a batch; remove it first");
  release(h);
  return DID_OK;
}

int did_mem_estimate(int64_t M, int64_t N, int32_t K, const did_opts* opts, int32_t x_on_device, int64_t* bytes) {
  if (!bytes) return fail(DID_EINVAL, "bytes must not be NULL");
  *bytes = 0;
  int rc = check_shape(M, N, K);
  if (rc) return rc;
  did_opts o;
  did_default_opts(&o);
  if (opts) o = *opts;
  Shape s{};
  if ((rc = make_shape(s, M, N, K, o))) return rc;
  const int R = s.thin ? 1 : (int)make_ranges(N, s.nchunks, o.n_blocks, row_target(s, o)).size() - 1;
  *bytes = engine_bytes(s, R, !(x_on_device && o.borrow_x), o.refresh_every);
  return DID_OK;
}

int did_mem_bytes(did_handle h, int64_t* bytes) {
  if (!h || !bytes) return fail(DID_EINVAL, "NULL argument");
  *bytes = h->dev_bytes;
  return DID_OK;
}

int did_debug_check_guards(did_handle h, int64_t* bad, int32_t* zones) {
  if (!h || !bad) return fail(DID_EINVAL, "NULL argument");
  *bad = 0;
  if (zones) *zones = (int32_t)h->guard_zones.size();
  if (h->guard_zones.empty()) return DID_OK;
  DeviceGuard g(h->dev);
  std::vector<unsigned char> z(DID_GUARD_ZONE_BYTES);
  std::string first;
  for (const auto& gzone : h->guard_zones) {
    hipError_t e;
    if ((e = hipMemcpyAsync(z.data(), gzone.first, z.size(), hipMemcpyDeviceToHost, h->st)) != hipSuccess ||
        (e = hipStreamSynchronize(h->st)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(DID_EDEVICE, std::string("guard zone read failed: ") + hipGetErrorString(e));
    }
    int64_t n = 0;
    for (unsigned char c : z) n += c != (unsigned char)DID_GUARD_BYTE;
    if (n && first.empty())
      first = "buffer " + std::to_string(gzone.second) + " (in allocation order) was written past its end (" +
              std::to_string(n) + " guard bytes changed)";
    *bad += n;
  }
  if (!first.empty()) g_err = first;
  return DID_OK;
}

int did_debug_inject_fault(did_handle h) {
  if (!h) return fail(DID_EINVAL, "NULL handle");
  h->inject_fault = 1;
  return DID_OK;
}

const char* did_last_error(void) { return g_err.c_str(); }

}  // extern "C"
