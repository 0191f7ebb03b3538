// Batched and serving forms of the DID engine, and the tile autotuner.
//
// Batch: many instances of uneven (M, N, K) advance together.  Members are grouped by
// (KP, X storage, column-pass block waves); each group has a device-resident table of instance descriptors and
// work-item prefixes, and one iteration of every member is one launch per stage and group
// of a grouped persistent kernel (did_kernels.hip).  The launch sequence is captured once
// into a hipGraph and replayed per iteration; admitting or removing members only rewrites
// the tables (the graph is captured again only when a group appears or empties).  Each
// member runs exactly the blocks of its single-instance launch, so its iterates do not
// depend on what else is in the batch.
//
// Server: a request loop over a batch.  Jobs wait in a FIFO queue and are admitted while
// a batch slot is free and the device-memory budget holds their resident footprint; every
// step runs one iteration of all admitted jobs, reads their objectives back, and retires
// the jobs that met their stopping rule, which frees their slots for the queue.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "did_engine.h"
#include "did_kernels.h"

using namespace didengine;
using didk::GInst;
using didk::GS_N;
using didk::GTable;
using didk::kMaxBatch;
constexpr int kGroups = 2 * didk::XK_N * 2;  // (K class, X storage kind, column-pass block waves)

// ------------------------------------------------------------------ autotuned tiles
namespace {

std::mutex g_tune_mu;
struct Tuned {
  int row_blocks;
  int col_waves;
};
std::map<uint64_t, Tuned> g_tuned;  // shape class -> tile choice

int log2_class(int64_t v) {
  int c = 0;
  while (v > 1) {
    v = (v + 1) >> 1;
    ++c;
  }
  return c;
}

// Shape class: KP, X storage kind, ceil(log2 M), ceil(log2 N).
uint64_t shape_class(int64_t M, int64_t N, int KP, int xkind) {
  return ((uint64_t)(KP == 64) << 40) | ((uint64_t)xkind << 32) | ((uint64_t)log2_class(M) << 16) |
         (uint64_t)log2_class(N);
}

constexpr int kRowCandidates[] = {512, 1024, 2048, 4096, 8192};
constexpr int kColCandidates[] = {4, 8};

}  // namespace

namespace didengine {

int tuned_row_blocks(int64_t M, int64_t N, int KP, int xkind) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(shape_class(M, N, KP, xkind));
  return it == g_tuned.end() ? 0 : it->second.row_blocks;  // 0: the default target
}

int tuned_col_waves(int64_t M, int64_t N, int KP, int xkind) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(shape_class(M, N, KP, xkind));
  return it == g_tuned.end() ? 4 : it->second.col_waves;
}

}  // namespace didengine

// ------------------------------------------------------------------ batch
struct did_batch_ctx {
  int dev = 0;
  hipStream_t st = nullptr;
  bool own_stream = false;
  std::vector<did_ctx*> members;  // admission order
  struct Group {
    std::vector<did_ctx*> m;
    GTable* dtab = nullptr;  // device copy
    GTable* htab = nullptr;  // host image, in pinned memory (a direct copy to the device)
    int64_t grids[GS_N] = {0};
    bool have_grids = false;
  } groups[kGroups];
  double* dfcur = nullptr;  // device: latest objective per slot
  std::vector<int> slot_of;  // parallel to members
  double* hf = nullptr;  // pinned: the objectives read back each step
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  unsigned captured_mask = 0;  // groups present when the graph was captured
  bool dirty = true;
  int sticky = 0;
};

namespace {

int group_of(const did_ctx* h) {
  return 2 * ((h->s.KP == 64 ? didk::XK_N : 0) + didk::x_kind(h->s)) + (h->s.cwpb == 8 ? 1 : 0);
}
int group_kp(int g) { return g / 2 >= didk::XK_N ? 64 : 32; }
int group_xkind(int g) { return (g / 2) % didk::XK_N; }
int group_cwpb(int g) { return g % 2 ? 8 : 4; }

int bdev_fail(did_batch_ctx* b, hipError_t e, const char* what) {
  if (b) b->sticky = 1;
  return fail(DID_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int check_batch(did_batch_ctx* b) {
  if (!b) return fail(DID_EINVAL, "NULL batch");
  if (b->sticky) return fail(DID_EDEVICE, "batch is in a failed state after an earlier device error");
  return DID_OK;
}

void fill_inst(GInst& d, did_ctx* h, double* fcur) {
  const didk::Shape& s = h->s;
  d.X = h->X;
  d.XR = h->XR;
  d.B = h->B;
  d.C = h->C;
  d.Cq = h->Cq;
  d.Csc = h->Csc;
  d.Bq = h->Bq;
  d.Bsc = h->Bsc;
  d.H = h->H;
  d.fpart = h->fpart;
  d.G = h->G;
  d.Gpart = h->Gpart;
  d.V = h->V;
  d.Vpart = h->Vpart;
  d.Wpart = h->Wpart;
  d.W = h->W;
  d.tb = h->rbounds;
  d.fhist = h->fhist;
  d.tdev = h->tdev;
  d.fcur = fcur;
  d.M = s.M;
  d.N = s.N;
  d.nchunks = s.nchunks;
  d.Mpad = s.Mpad;
  d.hist_cap = kHistCap;
  d.vblocks = didk::vgram_blocks(s);
  d.colblocks = didk::colpass_blocks(s);
  d.bupblocks = didk::bupdate_blocks(s);
  d.K = s.K;
  d.vec4 = s.vec4;
  d.R = h->R;
  d.nsg = (int)((s.nchunks + 3) / 4);
}

// Rewrite the group tables for the current members and, if the set of non-empty groups
// changed, capture the iteration graph again.
int rebuild(did_batch_ctx* b) {
  hipError_t e;
  unsigned mask = 0;
  // earlier table uploads and replays have finished before the host images change
  if ((e = hipStreamSynchronize(b->st)) != hipSuccess) return bdev_fail(b, e, "batch rebuild");
  for (int g = 0; g < kGroups; ++g) {
    auto& G = b->groups[g];
    G.m.clear();
  }
  for (size_t i = 0; i < b->members.size(); ++i) {
    did_ctx* h = b->members[i];
    b->groups[group_of(h)].m.push_back(h);
  }
  for (int g = 0; g < kGroups; ++g) {
    auto& G = b->groups[g];
    if (G.m.empty()) continue;
    mask |= 1u << g;
    if (!G.dtab) {
      void* p = nullptr;
      if ((e = hipMalloc(&p, sizeof(GTable))) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DID_ENOMEM, "device allocation of a batch table failed");
      }
      G.dtab = static_cast<GTable*>(p);
    }
    if (!G.htab) {
      void* p = nullptr;
      if ((e = hipHostMalloc(&p, sizeof(GTable), hipHostMallocDefault)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DID_ENOMEM, "pinned host allocation of a batch table failed");
      }
      G.htab = static_cast<GTable*>(p);
    }
    if (!G.have_grids) {
      if ((e = didk::group_grids(group_kp(g), group_xkind(g), group_cwpb(g), G.grids)) != hipSuccess)
        return bdev_fail(b, e, "occupancy of the grouped kernels");
      G.have_grids = true;
    }
    GTable& t = *G.htab;
    memset(&t, 0, sizeof(t));
    t.n = (int)G.m.size();
    for (int st = 0; st < GS_N; ++st) t.begin[st][0] = 0;
    for (int i = 0; i < t.n; ++i) {
      did_ctx* h = G.m[i];
      const size_t mi = std::find(b->members.begin(), b->members.end(), h) - b->members.begin();
      fill_inst(t.inst[i], h, b->dfcur + b->slot_of[mi]);
      int64_t items[GS_N];
      didk::ginst_items(h->s, h->R, items);
      for (int st = 0; st < GS_N; ++st) t.begin[st][i + 1] = t.begin[st][i] + items[st];
    }
    for (int st = 0; st < GS_N; ++st) t.total[st] = t.begin[st][t.n];
    if ((e = hipMemcpyAsync(G.dtab, &t, sizeof(GTable), hipMemcpyHostToDevice, b->st)) != hipSuccess)
      return bdev_fail(b, e, "batch table upload");
  }
  if (mask != b->captured_mask || !b->exec) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    if (mask) {
      if ((e = hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return bdev_fail(b, e, "graph capture");
      hipError_t le = hipSuccess;
      for (int g = 0; g < kGroups; ++g) {
        auto& G = b->groups[g];
        if (!(mask & (1u << g))) continue;
        hipError_t r = didk::group_iteration(group_kp(g), group_xkind(g), group_cwpb(g), G.dtab, G.grids, b->st);
        if (r != hipSuccess && le == hipSuccess) le = r;
      }
      if ((e = hipStreamEndCapture(b->st, &b->graph)) != hipSuccess) return bdev_fail(b, e, "graph capture");
      if (le != hipSuccess) return bdev_fail(b, le, "grouped launch during capture");
      if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess)
        return bdev_fail(b, e, "graph instantiate");
    }
    b->captured_mask = mask;
  }
  b->dirty = false;
  return DID_OK;
}

int free_slot(const did_batch_ctx* b) {
  for (int s = 0; s < kGroups * kMaxBatch; ++s)
    if (std::find(b->slot_of.begin(), b->slot_of.end(), s) == b->slot_of.end()) return s;
  return -1;
}

}  // namespace

extern "C" {

int did_batch_create(void* stream, did_batch* out) {
  if (!out) return fail(DID_EINVAL, "out must not be NULL");
  *out = nullptr;
  did_batch_ctx* b = new (std::nothrow) did_batch_ctx();
  if (!b) return fail(DID_ENOMEM, "host allocation failed");
  hipError_t e;
  if ((e = hipGetDevice(&b->dev)) != hipSuccess) {
    delete b;
    return fail(DID_EDEVICE, "no HIP device");
  }
  if (stream) {
    b->st = static_cast<hipStream_t>(stream);
  } else {
    if ((e = hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking)) != hipSuccess) {
      delete b;
      return fail(DID_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    }
    b->own_stream = true;
  }
  void* p = nullptr;
  if ((e = hipMalloc(&p, sizeof(double) * kGroups * kMaxBatch)) != hipSuccess) {
    (void)hipGetLastError();
    if (b->own_stream) (void)hipStreamDestroy(b->st);
    delete b;
    return fail(DID_ENOMEM, "device allocation failed");
  }
  b->dfcur = static_cast<double*>(p);
  if ((e = hipHostMalloc(&p, sizeof(double) * kGroups * kMaxBatch, hipHostMallocDefault)) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(b->dfcur);
    if (b->own_stream) (void)hipStreamDestroy(b->st);
    delete b;
    return fail(DID_ENOMEM, "pinned host allocation failed");
  }
  b->hf = static_cast<double*>(p);
  *out = b;
  return DID_OK;
}

int did_batch_add(did_batch b, did_handle h) {
  int rc = check_batch(b);
  if (rc) return rc;
  if ((rc = check_free_handle(h))) return rc;
  if (h->dev != b->dev) return fail(DID_EINVAL, "handle and batch are on different devices");
  if (h->s.thin) return fail(DID_EINVAL, "the batched form runs the MFMA passes; thin-matrix shapes are not accepted");
  if (h->algorithm != DID_ALG_DID) return fail(DID_EINVAL, "the batched form runs DID only");
  if (h->refresh != 1)
    return fail(DID_EINVAL, "the batched form refreshes the residual every iteration (refresh_every must be 1)");
  if (h->profiling) return fail(DID_ESTATE, "disable profiling before adding a handle to a batch");
  int n_in_group = 0;
  for (did_ctx* m : b->members) n_in_group += group_of(m) == group_of(h);
  if (n_in_group >= kMaxBatch) return fail(DID_ESTATE, "batch group is full (64 instances per (K class, X storage, column-pass block waves))");
  const int slot = free_slot(b);
  if (slot < 0) return fail(DID_ESTATE, "batch is full");
  DeviceGuard g(b->dev);
  hipError_t e;
  // the member's earlier work must be finished; its device iteration counter follows t
  if ((e = hipStreamSynchronize(h->st)) != hipSuccess) return dev_fail(h, e, "batch add");
  if ((e = hipMemcpy(h->tdev, &h->t, sizeof(int64_t), hipMemcpyHostToDevice)) != hipSuccess)
    return dev_fail(h, e, "batch add");
  b->members.push_back(h);
  b->slot_of.push_back(slot);
  h->batch = b;
  b->dirty = true;
  return DID_OK;
}

int did_batch_remove(did_batch b, did_handle h) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (!h || h->batch != b) return fail(DID_EINVAL, "handle is not a member of this batch");
  DeviceGuard g(b->dev);
  hipError_t e;
  if ((e = hipStreamSynchronize(b->st)) != hipSuccess) return bdev_fail(b, e, "batch remove");
  const size_t i = std::find(b->members.begin(), b->members.end(), h) - b->members.begin();
  b->members.erase(b->members.begin() + i);
  b->slot_of.erase(b->slot_of.begin() + i);
  h->batch = nullptr;
  b->dirty = true;
  return DID_OK;
}

int did_batch_size(did_batch b, int32_t* n) {
  if (!b || !n) return fail(DID_EINVAL, "NULL argument");
  *n = (int32_t)b->members.size();
  return DID_OK;
}

int did_batch_iterate(did_batch b, int32_t n) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (n < 0) return fail(DID_EINVAL, "n must be >= 0");
  if (b->members.empty() || n == 0) return DID_OK;
  DeviceGuard g(b->dev);
  if (b->dirty && (rc = rebuild(b))) return rc;
  hipError_t e;
  for (int32_t it = 0; it < n; ++it)
    if ((e = hipGraphLaunch(b->exec, b->st)) != hipSuccess) return bdev_fail(b, e, "graph launch");
  for (did_ctx* h : b->members) h->t += n;
  return DID_OK;
}

int did_batch_objectives(did_batch b, double* f, int32_t cap, int32_t* n) {
  int rc = check_batch(b);
  if (rc) return rc;
  if (!n || (cap > 0 && !f) || cap < 0) return fail(DID_EINVAL, "bad output arguments");
  DeviceGuard g(b->dev);
  hipError_t e;
  if ((e = hipMemcpyAsync(b->hf, b->dfcur, sizeof(double) * kGroups * kMaxBatch, hipMemcpyDeviceToHost, b->st)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(b->st)) != hipSuccess)
    return bdev_fail(b, e, "objective readback");
  *n = (int32_t)b->members.size();
  for (int32_t i = 0; i < *n && i < cap; ++i) f[i] = b->hf[b->slot_of[i]];
  return DID_OK;
}

int did_batch_sync(did_batch b) {
  int rc = check_batch(b);
  if (rc) return rc;
  DeviceGuard g(b->dev);
  hipError_t e = hipStreamSynchronize(b->st);
  return e == hipSuccess ? DID_OK : bdev_fail(b, e, "batch sync");
}

int did_batch_free(did_batch b) {
  if (!b) return DID_OK;
  DeviceGuard g(b->dev);
  (void)hipStreamSynchronize(b->st);
  for (did_ctx* h : b->members) h->batch = nullptr;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto& G : b->groups) {
    if (G.dtab) (void)hipFree(G.dtab);
    if (G.htab) (void)hipHostFree(G.htab);
  }
  if (b->dfcur) (void)hipFree(b->dfcur);
  if (b->hf) (void)hipHostFree(b->hf);
  if (b->own_stream) (void)hipStreamDestroy(b->st);
  (void)hipGetLastError();
  delete b;
  return DID_OK;
}

// ------------------------------------------------------------------ autotuner
int did_autotune(int64_t M, int64_t N, int32_t K, int32_t x_dtype, int32_t x_tiled, int32_t* row_blocks,
                 int32_t* col_waves, double* ms_per_iter) {
  if (!row_blocks || !col_waves) return fail(DID_EINVAL, "row_blocks and col_waves must not be NULL");
  *row_blocks = 0;
  *col_waves = 0;
  if (x_dtype != DID_F32 && x_dtype != DID_BF16) return fail(DID_EINVAL, "x_dtype must be DID_F32 or DID_BF16");
  if (x_tiled != 0 && x_tiled != 1) return fail(DID_EINVAL, "x_tiled must be 0 or 1");
  int rc0 = check_shape(M, N, K);  // before the tuning input is sized from M N
  if (rc0) return rc0;
  if (M <= 16 && K <= 8 && (M <= 8 || K <= 4))
    return fail(DID_EINVAL, "thin-matrix shapes have no row pass to tune");
  // a synthetic X of the shape: U[0,1) entries from the engine's own generator
  float* X = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&X, (size_t)(M * N) * sizeof(float))) != hipSuccess) {
    (void)hipGetLastError();
    return fail(DID_ENOMEM, "device allocation for the tuning input failed");
  }
  hipStream_t st = nullptr;
  if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess ||
      (e = didk::fill_uniform(X, M * N, didk::stream_key(0x7475, 9), st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    (void)hipFree(X);
    if (st) (void)hipStreamDestroy(st);
    return fail(DID_EDEVICE, std::string("tuning input: ") + hipGetErrorString(e));
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  Tuned best{0, 0};
  double best_ms = 0.0;
  int rc = DID_OK;
  for (int cw : kColCandidates) {
    for (int cand : kRowCandidates) {
      did_opts o;
      did_default_opts(&o);
      o.x_dtype = x_dtype;
      o.x_tiled = x_dtype == DID_F32 ? x_tiled : 0;
      o.borrow_x = 1;
      o.row_blocks = cand;
      o.col_waves = cw;
      o.stream = st;
      did_handle h = nullptr;
      if ((rc = did_init_ex(X, M, N, K, 1, &o, &h))) break;
      // one warm-up iteration, then the best of two runs of enough iterations to fill about
      // 10 ms (at least 3), so that short iterations are not timed one launch at a time
      double per = 0.0;
      int reps = 3;
      bool ok = (rc = did_iterate(h, 1)) == DID_OK;
      for (int run = 0; ok && run < 3; ++run) {
        float ms = 0.0f;
        const int n = run == 0 ? 1 : reps;
        ok = hipEventRecord(e0, st) == hipSuccess && (rc = did_iterate(h, n)) == DID_OK &&
             hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (!ok) break;
        if (run == 0)
          reps = std::max(3, std::min(200, (int)std::ceil(10.0 / std::max(ms, 1e-3f))));
        else if (run == 1 || ms / reps < per)
          per = ms / reps;
      }
      if (ok && (!best.row_blocks || per < best_ms)) {
        best = Tuned{cand, cw};
        best_ms = per;
      }
      did_free(h);
      if (rc) break;
    }
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(st);
  (void)hipFree(X);
  if (rc) return rc;
  if (!best.row_blocks) return fail(DID_EDEVICE, "tuning runs failed");
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const int xkind = x_dtype == DID_BF16 ? didk::XK_BF16 : x_tiled ? didk::XK_F32_TILED : didk::XK_F32;
    g_tuned[shape_class(M, N, K <= 32 ? 32 : 64, xkind)] = best;
  }
  *row_blocks = best.row_blocks;
  *col_waves = best.col_waves;
  if (ms_per_iter) *ms_per_iter = best_ms;
  return DID_OK;
}

int did_autotune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.clear();
  return DID_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ server
namespace {

struct Job {
  int64_t id = 0;
  const void* X = nullptr;
  int64_t M = 0, N = 0;
  int32_t K = 0;
  uint64_t seed = 0;
  int32_t x_dtype = DID_F32;
  int32_t state = DID_JOB_QUEUED;
  did_handle h = nullptr;
  int64_t bytes = 0;  // resident footprint charged to the budget
  double f_prev = -1.0, f_last = -1.0;
  int32_t iters = 0;
  std::chrono::steady_clock::time_point t_submit, t_start, t_done;
  std::string error;
};

}  // namespace

struct did_server_ctx {
  did_server_opts o{};
  hipStream_t st = nullptr;      // batch iterations
  hipStream_t adm_st = nullptr;  // initialisation of admitted jobs, beside the iterations
  bool own_stream = false;
  did_batch b = nullptr;
  int64_t next_id = 1;
  std::deque<int64_t> queue;
  std::map<int64_t, Job> jobs;
  std::vector<int64_t> running;   // batch member order
  std::vector<int64_t> admitted;  // initialised, joining the batch at the next step
  bool inflight = false;          // an iteration of the running jobs has been launched
  int64_t used = 0;               // bytes charged by admitted, unreleased jobs
  int64_t peak_used = 0;
  // handles of released jobs, freed at the next step once the batch stream has drained (a
  // device free waits for the device: called between steps it would hold the host until
  // the iteration in flight ends and leave the device idle afterwards)
  std::vector<did_handle> retired;
  ArenaPool pool;  // arenas of released jobs, reused by later admissions
};

namespace {

int check_server(did_server_ctx* s) {
  if (!s) return fail(DID_EINVAL, "NULL server");
  return DID_OK;
}

double secs(std::chrono::steady_clock::duration d) { return std::chrono::duration<double>(d).count(); }

}  // namespace

extern "C" {

int did_server_default_opts(did_server_opts* o) {
  if (!o) return fail(DID_EINVAL, "opts must not be NULL");
  memset(o, 0, sizeof(*o));
  o->hbm_budget = (int64_t)200 << 30;
  o->max_active = 64;
  o->max_iter = 50;
  o->rel_tol = 1e-4;
  o->stream = nullptr;
  return DID_OK;
}

int did_server_create(const did_server_opts* opts, did_server* out) {
  if (!out) return fail(DID_EINVAL, "out must not be NULL");
  *out = nullptr;
  did_server_opts o;
  did_server_default_opts(&o);
  if (opts) o = *opts;
  if (o.hbm_budget <= 0 || o.max_active < 1 || o.max_active > 4 * kMaxBatch || o.max_iter < 1 ||
      !(o.rel_tol >= 0.0) || (o.x_tiled != 0 && o.x_tiled != 1) || o.arena_reserve_gib < 0)
    return fail(DID_EINVAL, "bad server options");
  did_server_ctx* s = new (std::nothrow) did_server_ctx();
  if (!s) return fail(DID_ENOMEM, "host allocation failed");
  s->o = o;
  hipError_t e;
  if (o.stream) {
    s->st = static_cast<hipStream_t>(o.stream);
  } else {
    if ((e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking)) != hipSuccess) {
      delete s;
      return fail(DID_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    }
    s->own_stream = true;
  }
  if ((e = hipStreamCreateWithFlags(&s->adm_st, hipStreamNonBlocking)) != hipSuccess) {
    if (s->own_stream) (void)hipStreamDestroy(s->st);
    delete s;
    return fail(DID_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
  }
  int rc = did_batch_create(s->st, &s->b);
  if (!rc && o.arena_reserve_gib > 0) {
    if ((rc = didengine::pool_reserve_slab(&s->pool, (size_t)o.arena_reserve_gib << 30))) did_batch_free(s->b);
  }
  if (rc) {
    (void)hipStreamDestroy(s->adm_st);
    if (s->own_stream) (void)hipStreamDestroy(s->st);
    delete s;
    return rc;
  }
  *out = s;
  return DID_OK;
}

int did_server_submit(did_server s, const void* X, int64_t M, int64_t N, int32_t K, uint64_t seed, int32_t x_dtype,
                      int64_t* job) {
  int rc = check_server(s);
  if (rc) return rc;
  if (!X || !job) return fail(DID_EINVAL, "NULL argument");
  *job = 0;
  did_opts o;
  did_default_opts(&o);
  o.x_dtype = x_dtype;
  o.borrow_x = 1;
  o.x_tiled = s->o.x_tiled;
  int64_t bytes = 0;
  if ((rc = did_mem_estimate(M, N, K, &o, 1, &bytes))) return rc;
  if (M <= 16 && K <= 8 && (M <= 8 || K <= 4)) return fail(DID_EINVAL, "the server runs the MFMA passes; thin shapes are not served");
  if (x_dtype == DID_F32) bytes += M * N * 4;  // the borrowed X stays resident
  if (bytes > s->o.hbm_budget) return fail(DID_ENOMEM, "job footprint exceeds the server's memory budget");
  Job j;
  j.id = s->next_id++;
  j.X = X;
  j.M = M;
  j.N = N;
  j.K = K;
  j.seed = seed;
  j.x_dtype = x_dtype;
  j.bytes = bytes;
  j.t_submit = std::chrono::steady_clock::now();
  s->jobs[j.id] = j;
  s->queue.push_back(j.id);
  *job = j.id;
  return DID_OK;
}

// One scheduling step, pipelined so that host work overlaps an iteration on the device:
//   1. collect the iteration launched by the previous step (objectives of every running
//      job), retire the jobs that met their stopping rule;
//   2. the jobs initialised by the previous step join the batch;
//   3. launch the next iteration of all running jobs (asynchronous);
//   4. admit queued jobs first-in first-out while a slot is free, their batch group has
//      room and the budget holds them, and initialise them on the admission stream while
//      the iteration runs; they join at the next step.
int did_server_step(did_server s, int32_t* n_running, int32_t* n_queued, int32_t* n_finished) {
  int rc = check_server(s);
  if (rc) return rc;
  // admissions allocate, and take pooled arenas, on the server's device whatever device
  // the calling thread has made current since did_server_create
  DeviceGuard g(s->b->dev);
  int32_t finished = 0;
  if (s->inflight) {
    s->inflight = false;
    std::vector<double> f(s->running.size());
    int32_t n = 0;
    if ((rc = did_batch_objectives(s->b, f.data(), (int32_t)f.size(), &n))) return rc;
    const auto now = std::chrono::steady_clock::now();
    std::vector<int64_t> keep;
    for (size_t i = 0; i < s->running.size(); ++i) {
      Job& j = s->jobs[s->running[i]];
      j.iters += 1;
      j.f_prev = j.f_last;
      j.f_last = f[i];  // f(B^{t-1}, C^{t-1}), formed by this iteration's column pass
      const bool conv = j.f_prev >= 0.0 && std::fabs(j.f_prev - j.f_last) <= s->o.rel_tol * j.f_last;
      if (j.iters >= s->o.max_iter || conv) {
        if ((rc = did_batch_remove(s->b, j.h))) return rc;
        j.state = DID_JOB_DONE;
        j.t_done = now;
        ++finished;
      } else {
        keep.push_back(j.id);
      }
    }
    s->running.swap(keep);
  }
  // the iteration in flight has ended (its objectives were read back): free the handles
  // released since, before any admission counts on their memory
  for (did_handle h : s->retired) did_free(h);
  s->retired.clear();
  for (int64_t id : s->admitted) {
    Job& j = s->jobs[id];
    // the job's set-up ran on the admission stream beside the last iteration; X's check
    // is read here (an X that is not finite and nonnegative fails the job)
    if ((rc = didengine::check_deferred(j.h)) || (rc = did_batch_add(s->b, j.h))) {
      j.state = DID_JOB_FAILED;
      j.error = g_err;
      did_free(j.h);
      j.h = nullptr;
      s->used -= j.bytes;
      j.t_done = std::chrono::steady_clock::now();
      ++finished;
      if (rc == DID_EDEVICE) return rc;
      continue;
    }
    s->running.push_back(id);
  }
  s->admitted.clear();
  if (!s->running.empty()) {
    if ((rc = did_batch_iterate(s->b, 1))) return rc;
    s->inflight = true;
  }
  while (!s->queue.empty() && (int)(s->running.size() + s->admitted.size()) < s->o.max_active) {
    Job& j = s->jobs[s->queue.front()];
    if (s->used + j.bytes > s->o.hbm_budget) break;
    int same_group = 0;
    for (const auto* list : {&s->running, &s->admitted})
      for (int64_t id : *list) {
        const Job& r = s->jobs[id];
        same_group += ((r.K > 32) == (j.K > 32)) && (r.x_dtype == j.x_dtype);
      }
    if (same_group >= kMaxBatch) break;
    did_opts o;
    did_default_opts(&o);
    o.x_dtype = j.x_dtype;
    o.borrow_x = 1;
    o.x_tiled = s->o.x_tiled;
    o.stream = s->adm_st;
    s->queue.pop_front();
    j.t_start = std::chrono::steady_clock::now();
    if ((rc = didengine::init_deferred(j.X, j.M, j.N, j.K, j.seed, &o, &j.h, &s->pool))) {
      j.state = DID_JOB_FAILED;
      j.error = g_err;
      j.h = nullptr;
      j.t_done = std::chrono::steady_clock::now();
      ++finished;
      if (rc == DID_EDEVICE) return rc;
      continue;
    }
    j.state = DID_JOB_RUNNING;
    s->used += j.bytes;
    s->peak_used = std::max(s->peak_used, s->used);
    s->admitted.push_back(j.id);
  }
  if (n_running) *n_running = (int32_t)(s->running.size() + s->admitted.size());
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  if (n_finished) *n_finished = finished;
  return DID_OK;
}

int did_server_poll(did_server s, int64_t job, int32_t* state, int32_t* iters, double* f, double* latency_s,
                    double* queue_s) {
  int rc = check_server(s);
  if (rc) return rc;
  auto it = s->jobs.find(job);
  if (it == s->jobs.end()) return fail(DID_EINVAL, "unknown job");
  const Job& j = it->second;
  if (state) *state = j.state;
  if (iters) *iters = j.iters;
  if (f) *f = j.f_last;
  const bool ended = j.state == DID_JOB_DONE || j.state == DID_JOB_FAILED;
  if (latency_s) *latency_s = ended ? secs(j.t_done - j.t_submit) : -1.0;
  if (queue_s) *queue_s = j.state == DID_JOB_QUEUED ? -1.0 : secs(j.t_start - j.t_submit);
  return DID_OK;
}

int did_server_result(did_server s, int64_t job, float* B, float* C) {
  int rc = check_server(s);
  if (rc) return rc;
  auto it = s->jobs.find(job);
  if (it == s->jobs.end()) return fail(DID_EINVAL, "unknown job");
  Job& j = it->second;
  if (j.state == DID_JOB_FAILED) return fail(DID_ESTATE, "job failed: " + j.error);
  if (j.state != DID_JOB_DONE || !j.h) return fail(DID_ESTATE, "job has no result (not done or released)");
  return did_factors(j.h, B, C);
}

int did_server_release(did_server s, int64_t job) {
  int rc = check_server(s);
  if (rc) return rc;
  auto it = s->jobs.find(job);
  if (it == s->jobs.end()) return fail(DID_EINVAL, "unknown job");
  Job& j = it->second;
  if (j.state == DID_JOB_QUEUED || j.state == DID_JOB_RUNNING) return fail(DID_ESTATE, "job is still in progress");
  if (j.h) {
    s->retired.push_back(j.h);
    j.h = nullptr;
    s->used -= j.bytes;
  }
  s->jobs.erase(it);
  return DID_OK;
}

int did_server_memory(did_server s, int64_t* used, int64_t* peak) {
  int rc = check_server(s);
  if (rc) return rc;
  if (used) *used = s->used;
  if (peak) *peak = s->peak_used;
  return DID_OK;
}

int did_server_arena_stats(did_server s, int64_t* allocs, int64_t* reuses, int64_t* frees, int64_t* pooled_bytes) {
  int rc = check_server(s);
  if (rc) return rc;
  if (allocs) *allocs = s->pool.allocs;
  if (reuses) *reuses = s->pool.reuses;
  if (frees) *frees = s->pool.frees;
  if (pooled_bytes) *pooled_bytes = (int64_t)s->pool.bytes;
  return DID_OK;
}

int did_server_free(did_server s) {
  if (!s) return DID_OK;
  DeviceGuard g(s->b->dev);  // a server always has its batch (did_server_create)
  if (s->b) {
    (void)did_batch_sync(s->b);
    for (int64_t id : s->running) (void)did_batch_remove(s->b, s->jobs[id].h);
  }
  for (auto& kv : s->jobs)
    if (kv.second.h) did_free(kv.second.h);
  for (did_handle h : s->retired) did_free(h);
  didengine::pool_free_all(&s->pool);
  didengine::pool_free_slab(&s->pool);  // every handle, and so every arena carved from it, is gone
  did_batch_free(s->b);
  if (s->adm_st) (void)hipStreamDestroy(s->adm_st);
  if (s->own_stream) (void)hipStreamDestroy(s->st);
  delete s;
  return DID_OK;
}

}  // extern "C"
