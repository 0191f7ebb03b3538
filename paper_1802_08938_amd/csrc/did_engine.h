// Internal declarations shared by the single-instance engine (did_engine.hip) and the
// batched/serving layer (did_batch.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/did.h"
#include "did_kernels.h"

struct did_batch_ctx;

// One NMF instance: its device buffers and stream.
// Device arenas kept for reuse by the handles of one serving loop: a handle made with a
// pool carves its buffers from the smallest pooled arena that fits (wasting at most half of
// it) and gives its arena back at release; the pool frees its largest arenas beyond limit.
//
// A serving loop may also reserve one slab of device memory when it is created; arenas are
// then carved from the slab first (first fit, adjacent free ranges merged at release), so
// that admissions call no hipMalloc while the slab has room.
struct ArenaPool {
  std::vector<std::pair<void*, size_t>> free;  // (pointer, capacity)
  size_t bytes = 0;
  size_t limit = size_t(48) << 30;
  // arenas allocated for admissions, taken from the pool or the slab, and freed
  int64_t allocs = 0, reuses = 0, frees = 0;
  unsigned char* slab = nullptr;
  size_t slab_cap = 0;
  std::map<size_t, size_t> slab_free;  // offset -> length of each free range of the slab
};

struct did_ctx {
  int dev = 0;
  hipStream_t st = nullptr;
  bool own_stream = false;
  // MFMA path: a second stream on which the V partials and their reduction run while the
  // row pass runs on st (both only read the packed C); ev_c: C packed, ev_v: V reduced
  hipStream_t st2 = nullptr;
  hipEvent_t ev_c = nullptr, ev_v = nullptr;
  didk::Shape s{};
  bool own_x = true;
  void* X = nullptr;   // float32 (column-major), or the column-pass tiled bf16 copy (s.xbf16)
  void* XR = nullptr;  // X as the row pass reads it: X itself, or the row-pass tiled bf16 copy
  float* B = nullptr;
  float* C = nullptr;
  _Float16* Bq = nullptr;  // B packed as MFMA operands (layout in did_kernels.h)
  float* Bsc = nullptr;     // column scales of the packed B
  float* Csc = nullptr;     // row scales of the packed C
  double* G = nullptr;
  double* Gpart = nullptr;
  double* V = nullptr;
  double* Vpart = nullptr;
  float* H = nullptr;
  void* Cq = nullptr;
  double* W = nullptr;
  float* Wpart = nullptr;
  double* tpart = nullptr;  // thin path: block partials
  // carried-residual form (refresh_every > 1): the residual R (column-major float32,
  // M x N), the E-order operands of delta B (layout of Bq) and of delta C (E part of Cq)
  int refresh = 1;
  float* Rres = nullptr;
  _Float16* BqD = nullptr;
  void* CqD = nullptr;
  int algorithm = DID_ALG_DID;
  int R = 1;
  int64_t* rbounds = nullptr;
  double* fpart = nullptr;
  double* fhist = nullptr;
  int64_t hist_cap = int64_t(1) << 16;  // entries of fhist (a ring indexed by t)
  double* fobj = nullptr;
  int64_t* tdev = nullptr;  // device copy of t (used by the batched form)
  int* flag = nullptr;
  int64_t t = 0;
  int sticky = 0;
  int inject_fault = 0;   // did_debug_inject_fault: the next checked call fails as a device error would
  int64_t dev_bytes = 0;  // device memory held by the engine for this instance
  did_batch_ctx* batch = nullptr;
  std::vector<void*> allocs;
  // one device allocation sized at setup from which the instance's buffers are carved (a
  // release is then one hipFree, which waits for the device, instead of one per buffer)
  unsigned char* arena = nullptr;
  size_t arena_cap = 0, arena_off = 0;
  ArenaPool* pool = nullptr;  // the serving loop's pool the arena comes from and returns to
  bool arena_in_slab = false;  // carved from the pool's slab (returned to the slab at release)
  // made by a serving loop: X's validation result and the set-up work stay queued on the
  // stream (no host wait); check_deferred reads the result once the stream has drained
  bool defer_checks = false;
  bool x_check_pending = false;
  // DID_DEBUG_GUARD_ZONES: a patterned zone after each buffer carved from the arena
  bool guards = false;
  std::vector<std::pair<unsigned char*, int>> guard_zones;  // zone start, buffer index
  // one captured iteration of the MFMA path, replayed by did_iterate (not in the carried
  // form, not while profiling; never by did_iterate_static, which must not allocate)
  bool use_graph = true;
  // whether eager iterations may create the second stream (not in did_iterate_static,
  // whose context lives on the caller's stack and must not create resources)
  bool may_create_st2 = true;
  bool graph_failed = false;
  hipGraphExec_t gexec = nullptr;
  // per-stage timing: kStages+1 events per profiled iteration
  bool profiling = false;
  std::vector<hipEvent_t> prof_events;
};

namespace didengine {

constexpr int64_t kHistCap = 1 << 16;

extern thread_local std::string g_err;
int fail(int code, const std::string& msg);
int dev_fail(did_ctx* h, hipError_t e, const char* what);
int dalloc_bytes(did_ctx* h, void** p, size_t bytes);
int check_handle(did_ctx* h);       // non-NULL and not sticky-failed
int check_free_handle(did_ctx* h);  // check_handle and not a batch member

// Row-pass target recorded by did_autotune for the shape class of (M, N, KP, X storage),
// else 0 (range_params's default).
int tuned_row_blocks(int64_t M, int64_t N, int KP, int xkind);
// Column-pass waves per block recorded by did_autotune for the shape class, else 4.
int tuned_col_waves(int64_t M, int64_t N, int KP, int xkind);

// Shared by the single-instance engine and the allocation-free entry point (did_engine.hip).
int check_shape(int64_t M, int64_t N, int32_t K);
int make_shape(didk::Shape& s, int64_t M, int64_t N, int32_t K, const did_opts& o);
int row_target(const didk::Shape& s, const did_opts& o);
void range_params(int64_t N, int64_t nchunks, int n_blocks, int row_blocks, int64_t* T, int64_t* P, int64_t* S);
hipError_t refresh_b_derived(did_ctx* h);  // pack B and form G = B^T B
hipError_t pack_c(did_ctx* h);             // pack C after it was set from outside the sweep
int iterate_mfma(did_ctx* h, int32_t n);   // n iterations of the MFMA path on h's buffers
// did_init_ex for a serving loop: X is validated on the device without a host wait (a
// device X only) and the set-up stays queued on the handle's stream; check_deferred waits
// for that stream and returns DID_EINVAL (with the message) if X was not finite and
// nonnegative, DID_OK otherwise (also for handles made without deferral).
int init_deferred(const void* X, int64_t M, int64_t N, int32_t K, uint64_t seed, const did_opts* opts,
                  did_handle* out, ArenaPool* pool = nullptr);
void pool_free_all(ArenaPool* pool);  // free every pooled arena (not the slab)
int pool_reserve_slab(ArenaPool* pool, size_t bytes);  // allocate the slab (DID_ENOMEM if it fails)
void pool_free_slab(ArenaPool* pool);                  // once no arena of the slab is in use
int check_deferred(did_ctx* h);

// Make a device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
};

}  // namespace didengine
