/*
 * did.h -- C ABI of libdid, an MI355X (gfx950) engine for DID: distributed incremental
 * block coordinate descent for nonnegative matrix factorisation (Gao & Chu, AAAI-18,
 * arXiv 1802.08938).
 *
 * Problem (Introduction, eq. opt:nmf): given X in R_+^{M x N} whose columns are samples,
 * find B in R_+^{M x K} and C in R_+^{K x N} minimising f(B, C) = 1/2 ||X - BC||_F^2.
 *
 * One iteration (Section 4, Alg. 3) updates every row of C by the closed-form coordinate
 * rule (eq. sol:c_ij, applied against the running residual as in eq. up:c), forms the
 * messages W = E C^T and V = tril(C C^T) (eqs. W_j, V_j) per column block and sums them
 * once (the paper's single Allreduce, here an in-device fixed-order block reduction), and
 * then updates the columns of B incrementally (the delta-b rule of Section 4,
 * "Incremental Update for b_i").
 *
 * Conventions shared by every call
 * --------------------------------
 * - All matrices are column-major: X and the residual have leading dimension M (a sample
 *   x_j is contiguous), B has leading dimension M (a basis column b_k is contiguous), C
 *   has leading dimension K (a coordinate vector c_j is contiguous).
 * - Every call returns an int: DID_OK (0) on success, a negative DID_E* code otherwise.
 *   Nothing aborts or throws across the ABI.  After a failure, did_last_error() returns
 *   a message for the calling thread.
 * - A device fault during any call makes the handle sticky-failed: every later call on
 *   it returns DID_EDEVICE (did_free still releases it).
 * - A handle is not thread-safe.  Distinct handles on distinct streams are independent.
 *   All work of a handle is ordered on its stream; calls that return host data
 *   (did_objective, did_factors, did_history) synchronise that stream.
 * - The library owns every buffer it allocates and never frees caller memory.
 * - Sizes: 1 <= K <= min(M, N) and K <= 64 (the register-resident sweep supports up to
 *   64 coordinates); M, N >= 1; M * N < 2^62.  Violations return DID_EINVAL.
 */
#ifndef DID_H
#define DID_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct did_ctx* did_handle; /* opaque; one handle = one NMF instance */

enum {
  DID_OK = 0,
  DID_EINVAL = -1,  /* bad argument, bad shape, or X not finite / not nonnegative */
  DID_ENOMEM = -2,  /* device allocation failed */
  DID_EDEVICE = -3, /* HIP runtime or kernel failure (sticky) */
  DID_ESTATE = -4   /* call not valid in the handle's current state */
};

enum { DID_F32 = 0, DID_BF16 = 1 }; /* storage type of X inside the engine */

/* Update order of one iteration (did_opts.algorithm). */
enum {
  DID_ALG_DID = 0, /* Alg. 3: C sweep, one reduction of (W, V), incremental B update */
  DID_ALG_DBCD = 1 /* Alg. 2 (DBCD), an ablation: one reduction per column of B; same iterates */
};

#define DID_MAX_K 64

/*
 * Options for did_init_ex.  Fill with did_default_opts() and override fields.
 *   n_blocks       number P of contiguous column blocks (the paper's per-node shards,
 *                  Section 3 "Distributed ADMM" / Section 4): the messages W_p, V_p are
 *                  formed per block and added in ascending block order.  0 lets the
 *                  engine choose; results depend on P only through summation order.
 *   x_dtype        DID_F32: X is used as given.  DID_BF16: X (still passed as float32)
 *                  is rounded to bf16 (round to nearest even) on the device and stored in
 *                  that form, as two copies in 32 x 32 tile order (one per pass over X,
 *                  each zero-padded to multiples of 32 rows and columns: together about
 *                  the size of the float32 X), halving the bytes each pass streams and
 *                  letting both passes load whole tiles with full-width loads; B, C, the residual
 *                  and every product stay float32-accurate and the objective is reduced in
 *                  float64, so the engine solves the problem for the rounded data exactly
 *                  as DID_F32 would.  borrow_x does not apply to DID_BF16.
 *   refresh_every  1 (default): the residual is formed afresh from X at the start of
 *                  every iteration, as Alg. 3 does.  r > 1: the engine keeps the residual
 *                  R = X - BC resident (column-major float32, 4 M N more bytes) and
 *                  carries it incrementally (Section 4, "Incremental Update for b_i": the
 *                  C sweep's r_j -= b_i delta c_ij and E := E - delta b_i c_i^r), and
 *                  forms it afresh from X every r-th iteration (t = 0, r, 2r, ...) to win
 *                  back the drift of the carried float32 residual.  Each pass then reads
 *                  and writes R (16 bytes per entry per iteration against 2 or 4 bytes of
 *                  X read twice), so the default is the faster form; the carried form is
 *                  the paper's own bookkeeping.  Needs the MFMA path (not the thin-matrix
 *                  shapes), 32 M < 2^32, and is not accepted by the batched form.
 *   init_scale     0: initial B, C are U[0,1) draws as they are.  1: both are then scaled
 *                  by sqrt(alpha), alpha = <X, BC> / ||BC||_F^2, which minimises f over a
 *                  common scale (the experiments' "well scaled initial points").
 *   borrow_x       0: X is copied into engine-owned memory.  1: a device X is adopted
 *                  without a copy; the caller keeps it alive and unmodified until
 *                  did_free.  Ignored (copy) for host pointers.
 *   algorithm      DID_ALG_DID (default) or DID_ALG_DBCD.  DBCD is available on the
 *                  thin-matrix path only (DID_EINVAL otherwise).
 *   row_blocks     tile shape of the row pass along N: about this many (column range,
 *                  32-row slab group) blocks per launch, which sets the number of column
 *                  ranges whose W partials are summed (in ascending order).  0 takes the
 *                  value did_autotune recorded for the instance's shape class, else
 *                  N / 256 clamped to [512, 4096].
 *                  Results depend on it only through summation order.
 *   x_tiled        float32 form only.  0: the passes read X as given (column-major).
 *                  1: the engine keeps X as two float32 copies in 32 x 32 tile order, one
 *                  per pass over X (the layout DID_BF16 uses), zero-padded to multiples of
 *                  32 rows and columns, so that both passes load whole tiles with
 *                  full-width loads.  Costs 8 * Mpad * Npad bytes of device memory and one
 *                  conversion pass at init; borrow_x does not apply.  Results are the same
 *                  bit for bit.  Not accepted on the thin-matrix path.
 *   col_waves      tile shape of the column pass: 4 or 8 waves per block, each wave one
 *                  32-column tile, the block's columns sharing one staged copy of B.
 *                  0 takes the value did_autotune recorded for the instance's shape class,
 *                  else 4.  The carried form (refresh_every > 1) runs 4 (8 is DID_EINVAL);
 *                  ignored on the thin-matrix path.  Any other value is DID_EINVAL.  B, C
 *                  and H do not depend on it; the objective does through summation order.
 *   stream         hipStream_t to order all work on; NULL = a stream owned by the handle.
 *
 * Shapes with M <= 16, K <= 8 and M <= 8 or K <= 4 (such as the experiments' synthetic
 * sets, M = 5, K = 3) run on a thin-matrix path that keeps each column in registers and
 * makes one fused pass over X per iteration; other shapes run the MFMA column/row passes.
 */
typedef struct did_opts {
  int32_t n_blocks;
  int32_t x_dtype;
  int32_t refresh_every;
  int32_t init_scale;
  int32_t borrow_x;
  int32_t algorithm;
  int32_t row_blocks;
  int32_t x_tiled;
  int32_t col_waves;
  void* stream;
} did_opts;

/* Fill *opts with the defaults: n_blocks 0, DID_F32, refresh_every 1, init_scale 0,
 * borrow_x 0, DID_ALG_DID, row_blocks 0, x_tiled 0, col_waves 0, stream NULL.  Returns DID_EINVAL for a NULL
 * pointer. */
int did_default_opts(did_opts* opts);

/*
 * Create an instance for X (M x N, column-major float32, host or device pointer; a host
 * pointer is uploaded) with K coordinates, and draw the initial factors.
 *   X must be finite and >= 0 (eq. opt:nmf takes X in R_+^{M x N}); a negative, NaN or
 *   infinite entry returns DID_EINVAL.
 *   A device X must be complete when the call is made: the engine reads it on its own
 *   stream (opts.stream, or a stream it creates), which is not ordered after other streams,
 *   so the caller synchronises the stream that wrote X first.  A borrowed X (borrow_x = 1)
 *   must not be written while the handle lives.
 *   Column-major float32 X (DID_F32 with x_tiled = 0, outside the thin-matrix path) needs
 *   32 M < 2^32; taller X returns DID_EINVAL and is accepted with x_tiled = 1.
 *   seed selects B^0 and C^0: entry i (column-major index) of B is U[0,1) from
 *   splitmix64 (Steele, Lea & Flood, OOPSLA 2014) keyed by (seed, 1, i), of C keyed by
 *   (seed, 2, i); the draw does not depend on the launch configuration.
 *   On success *out receives the handle.  On failure *out is set to NULL.
 */
int did_init(const float* X, int64_t M, int64_t N, int32_t K, uint64_t seed, did_handle* out);

/* did_init with options (opts may be NULL for the defaults); X is a float32 pointer. */
int did_init_ex(const void* X, int64_t M, int64_t N, int32_t K, uint64_t seed,
                const did_opts* opts, did_handle* out);

/*
 * Create an instance that resumes from given factors (checkpoint/restart): B (M x K,
 * column-major) and C (K x N, column-major), host or device float32 pointers, copied in.
 * B and C must be finite and >= 0.  The DID state is exactly (X, B, C): a resumed run
 * follows the same iterates as an uninterrupted one.
 */
int did_init_from_factors(const void* X, int64_t M, int64_t N, int32_t K, const float* B,
                          const float* C, const did_opts* opts, did_handle* out);

/*
 * Run n >= 0 full DID iterations (Alg. 3), stream-ordered, without host round trips.
 * Each iteration also records f(B^t, C^t) of the iterate it starts from (a by-product of
 * forming the residual) in the objective history.  Returns without synchronising.
 */
int did_iterate(did_handle h, int32_t n);

/* *f = f(B, C) = 1/2 ||X - BC||_F^2 at the current factors (eq. opt:nmf), accumulated in
 * float64 over the float32 residual.  Synchronises the handle's stream. */
int did_objective(did_handle h, double* f);

/*
 * Copy the current factors out: the problem's outputs B >= 0 (M x K, ld M) and C >= 0
 * (K x N, ld K) of eq. opt:nmf, float32, at the current iterate.  Either pointer may be
 * NULL to skip it; each may be host or device memory the caller owns (the library writes
 * M K and K N floats and never keeps the pointers).  Synchronises the handle's stream.
 * Returns DID_EDEVICE if the copy fails (the handle then becomes sticky-failed).
 */
int did_factors(did_handle h, float* B, float* C);

/*
 * Objective history: f[t] = f(B^t, C^t) for t = 0 .. count-1, where t counts iterations
 * since init and f[t] was recorded at the start of iteration t+1.  Copies
 * min(count, cap) leading values (f may be NULL with cap 0 to query) to host memory and
 * stores the number available in *count.  Synchronises the handle's stream.
 */
int did_history(did_handle h, double* f, int64_t cap, int64_t* count);

/* Number of iterations run since init. */
int did_iterations(did_handle h, int64_t* t);

/* Block until all queued work of the handle has finished. */
int did_sync(did_handle h);

/*
 * Per-stage timing, a profiling aid.  While enabled, did_iterate records a HIP event on
 * the handle's stream before the first and after every kernel stage of each iteration.
 * did_profile_read synchronises, stores the milliseconds summed per stage over the
 * iterations recorded since the last read into ms[0 .. min(cap, *n_stages)-1], the stage
 * count into *n_stages and the iteration count into *n_iters, and clears the record.
 * did_stage_name(i) names stage i ("column_pass", "row_pass", ...; "" if out of range).
 * On the MFMA path the V partials and their reduction run on a second stream, overlapped
 * with the row pass, so "sweep_v" times the sweep and the packing of the swept C for the
 * row pass, and "reduce_v" is empty.
 */
int did_profile(did_handle h, int32_t enable);
int did_profile_read(did_handle h, double* ms, int32_t cap, int32_t* n_stages, int64_t* n_iters);
const char* did_stage_name(int32_t stage);

/* Release every engine-owned resource of h (the state of one problem of eq. opt:nmf: its
 * copy of X, the factors and the derived buffers), after the queued work has finished.
 * NULL is a no-op (returns DID_OK).  Also accepted for a sticky-failed handle.  A batch
 * member must be removed from its batch first (DID_ESTATE); caller memory (a borrowed X,
 * the stream passed in opts) is never released. */
int did_free(did_handle h);

/* Device bytes the engine holds for h (X included when the engine owns a copy). */
int did_mem_bytes(did_handle h, int64_t* bytes);

/* Device bytes did_init_ex would allocate for an (M, N, K) instance with these options
 * (opts may be NULL); x_on_device = 1 when X will be passed as a device pointer (then
 * borrow_x = 1 allocates no copy of it; the tiled storages, DID_BF16 or x_tiled = 1,
 * always allocate their two copies).  Sizes are validated as did_init_ex does. */
int did_mem_estimate(int64_t M, int64_t N, int32_t K, const did_opts* opts, int32_t x_on_device,
                     int64_t* bytes);

/*
 * Tile autotuner.  Times DID iterations (after one warm-up, the better of two runs of
 * enough iterations to fill about 10 ms, at least three) of a synthetic
 * U[0,1) instance of shape (M, N, K) and X storage (x_dtype, and x_tiled for DID_F32;
 * ignored for DID_BF16) for each pair of column-pass block waves (4, 8) and row_blocks
 * value (512, 1024, 2048, 4096, 8192), records the fastest pair for the shape class
 * (K <= 32 or not, X storage: float32 as given, float32 tiled or bf16, ceil(log2 M),
 * ceil(log2 N)) in a process-wide table used by every later instance of the class
 * created with row_blocks = 0 or col_waves = 0, and returns it in *row_blocks and
 * *col_waves (and its time in *ms_per_iter if not NULL).  Allocates the tuning input
 * (4MN bytes) and the instance's own storage for the duration of the call.
 * Thin-matrix shapes, NULL row_blocks or col_waves and x_tiled outside {0, 1} return
 * DID_EINVAL.  did_autotune_clear() empties the table.
 */
int did_autotune(int64_t M, int64_t N, int32_t K, int32_t x_dtype, int32_t x_tiled,
                 int32_t* row_blocks, int32_t* col_waves, double* ms_per_iter);
int did_autotune_clear(void);

/*
 * Batched form: many instances of uneven (M, N, K) advanced together.
 * Members are grouped by (K <= 32 or not, X storage: float32 as given, float32 tiled or
 * bf16, column-pass block waves); each stage of an iteration is one
 * launch per group of a persistent kernel that walks the work items of all the group's
 * members from a device-resident table, and the launches of one iteration are captured
 * once in a hipGraph that each iteration replays.  A member runs exactly the work of its
 * own did_iterate, so its iterates equal those it would follow alone.
 *   did_batch_create  stream: hipStream_t for all batch work (NULL: one owned by the
 *                     batch).  *out receives the batch.
 *   did_batch_add     h joins the batch (same device; MFMA-path shapes only, algorithm
 *                     DID, profiling off; at most 64 members per group).  h's queued work
 *                     is waited for.  While a member, h accepts no did_iterate,
 *                     did_objective, did_factors, did_history, did_sync, did_profile* or
 *                     did_free (DID_ESTATE).
 *   did_batch_remove  h leaves the batch after the batch's queued work has finished; its
 *                     iteration count and objective history include the batched iterations.
 *   did_batch_iterate n iterations of every member (n graph replays), stream-ordered.
 *   did_batch_objectives  synchronises and stores, for member i in admission order, the
 *                     objective its latest iteration formed (f of the iterate that
 *                     iteration started from) into f[i], i < cap; *n = member count.
 *   did_batch_size, did_batch_sync, did_batch_free (members are detached, not freed).
 */
typedef struct did_batch_ctx* did_batch;
int did_batch_create(void* stream, did_batch* out);
int did_batch_add(did_batch b, did_handle h);
int did_batch_remove(did_batch b, did_handle h);
int did_batch_size(did_batch b, int32_t* n);
int did_batch_iterate(did_batch b, int32_t n);
int did_batch_objectives(did_batch b, double* f, int32_t cap, int32_t* n);
int did_batch_sync(did_batch b);
int did_batch_free(did_batch b);

/*
 * Serving form: a request loop over a batch (continuous batching).
 * Jobs are submitted with a device X (float32, column-major, borrowed until the job is
 * released), queue in FIFO order, and are admitted while a batch slot is free and the
 * memory budget holds the job's resident footprint (engine buffers, plus X for float32
 * storage).  Each did_server_step (1) collects the batched iteration the previous step
 * launched: it reads every running job's objective and retires a job once it has run
 * max_iter iterations or its objective changed by at most rel_tol relative between
 * consecutive iterations (the experiments' stopping criterion on the objective); (2) adds
 * the jobs admitted by the previous step to the batch; (3) launches the next iteration of
 * all running jobs and returns without waiting for it; (4) admits queued jobs and
 * initialises them on a second stream while that iteration runs.  Retired jobs keep their
 * factors until released.
 *   hbm_budget   bytes the admitted and unreleased jobs may hold (default 200 GiB)
 *   max_active   batch slots (1..256, default 64)
 *   max_iter     iteration cap per job (default 50)
 *   rel_tol      relative objective change that ends a job (default 1e-4)
 *   x_tiled      1: float32 jobs keep X in tile order (did_opts.x_tiled), which makes
 *                their iterations faster and adds 8 bytes per (padded) entry of X to
 *                their footprint; 0 (default): float32 jobs read the borrowed X as given
 *   arena_reserve_gib  GiB of device memory reserved when the server is created, from
 *                which admitted jobs' buffers are carved (first fit) before any other
 *                device allocation; default 0 (none).  Jobs then start without a
 *                hipMalloc, whose cost varies with the device's state.  The reserve is
 *                held until did_server_free, beside what the pool keeps.
 *   stream       hipStream_t for all server work (NULL: one owned by the server)
 * Job states: DID_JOB_QUEUED, DID_JOB_RUNNING, DID_JOB_DONE, DID_JOB_FAILED.
 *   did_server_submit  queue a job (x_dtype DID_F32 or DID_BF16; the init seed as in
 *                      did_init); *job receives its id.  A footprint above the whole
 *                      budget returns DID_ENOMEM; thin-matrix shapes return DID_EINVAL.
 *   did_server_step    *n_running (jobs running or admitted), *n_queued after the step,
 *                      *n_finished this step (any pointer may be NULL).
 *   did_server_poll    state, iterations, latest objective, seconds from submission to
 *                      retirement (-1 while not retired) and from submission to admission
 *                      (-1 while queued).
 *   did_server_result  copy a done job's B (M x K) and C (K x N) out, as did_factors.
 *                      For a failed job it returns DID_ESTATE, and did_last_error()
 *                      then gives the reason the job failed (an invalid X, a device
 *                      allocation that failed at admission, ...).
 *   did_server_release forget a retired job and return its memory to the budget; its
 *                      handle is released at the next did_server_step (once the iteration
 *                      in flight has ended) or by did_server_free.  X is not read after
 *                      the job retired, so the caller may free it.  Memory carved from the
 *                      reserve (arena_reserve_gib) goes back to it; the server keeps the
 *                      other device memory of released jobs (up to 48 GB) for later admissions,
 *                      which would otherwise allocate and free it job by job, and frees
 *                      it in did_server_free, or at once when an admission's device
 *                      allocation fails (the admission then tries once more).  The budget
 *                      is the server's share: device memory the caller holds (inputs not
 *                      yet submitted, other allocations) must fit beside it.
 *   did_server_memory  bytes charged to the budget now and at most so far.
 *   did_server_arena_stats  how admissions got their device memory so far: arenas
 *                      allocated (hipMalloc), arenas carved from the reserve or taken
 *                      from the pool of released jobs' memory, pooled arenas freed (beyond the pool's limit, or
 *                      to retry a failed allocation), and the bytes pooled now (any
 *                      pointer may be NULL).  Allocations and frees wait for the device
 *                      to drain, so many of them in a serving run cost throughput.
 * A server, like a handle, is driven from one thread.  Admission is strictly first-in
 * first-out: a head job that does not fit yet (budget, slots, or 64 running jobs of its
 * K class and X storage) holds back the jobs behind it.
 */
enum { DID_JOB_QUEUED = 0, DID_JOB_RUNNING = 1, DID_JOB_DONE = 2, DID_JOB_FAILED = 3 };
typedef struct did_server_opts {
  int64_t hbm_budget;
  int32_t max_active;
  int32_t max_iter;
  double rel_tol;
  int32_t x_tiled;
  int32_t arena_reserve_gib;
  void* stream;
} did_server_opts;
typedef struct did_server_ctx* did_server;
int did_server_default_opts(did_server_opts* opts);
int did_server_create(const did_server_opts* opts, did_server* out);
int did_server_submit(did_server s, const void* X, int64_t M, int64_t N, int32_t K, uint64_t seed,
                      int32_t x_dtype, int64_t* job);
int did_server_step(did_server s, int32_t* n_running, int32_t* n_queued, int32_t* n_finished);
int did_server_poll(did_server s, int64_t job, int32_t* state, int32_t* iters, double* f,
                    double* latency_s, double* queue_s);
int did_server_result(did_server s, int64_t job, float* B, float* C);
int did_server_release(did_server s, int64_t job);
int did_server_memory(did_server s, int64_t* used, int64_t* peak);
int did_server_arena_stats(did_server s, int64_t* allocs, int64_t* reuses, int64_t* frees, int64_t* pooled_bytes);
int did_server_free(did_server s);

/*
 * Allocation-free form of did_iterate, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  It runs
 * n >= 0 DID iterations (Alg. 3) from the caller's factors, with the same kernels and the
 * same iterates as did_init_from_factors(X, M, N, K, B, C, opts) followed by
 * did_iterate(n), and leaves B^n, C^n in place of B, C.
 *   X   device pointer, column-major float32 M x N (read as given; 32 M < 2^32), complete
 *       on opts->stream when the work starts and unchanged until it has finished.
 *   B   device pointer, M x K column-major float32, read and overwritten.
 *   C   device pointer, K x N column-major float32, read and overwritten.
 *   f   NULL, or a device pointer to n doubles: f[t] = f(B^t, C^t) (eq. opt:nmf), the
 *       objective of the iterate that iteration t+1 starts from.
 *   opts  NULL for the defaults; n_blocks and row_blocks are honoured; x_dtype must be
 *       DID_F32, x_tiled 0, refresh_every 1 and algorithm DID_ALG_DID; borrow_x and
 *       init_scale do not apply.  All work is queued on opts->stream (NULL: the null
 *       stream) and the call returns without synchronising.
 * Every intermediate buffer lives in one static device array of DID_STATIC_SCRATCH_BYTES
 * (128 MiB; each device the library runs on holds it until the process ends): the call
 * makes no device allocation, no memset and no host round trip.  At K > 32 an instance
 * needs about 772 bytes per column of X, 1028 bytes per row, and 256 bytes per row for
 * each of the row pass's column ranges (half of each at K <= 32); one that does not fit
 * returns DID_EINVAL with the size it needs (fewer ranges, a smaller row_blocks, shrink it).
 * Shapes of the thin-matrix path (M <= 16, K <= 8, M <= 8 or K <= 4) return DID_EINVAL.
 * X, B and C are not validated (that would need a host round trip): they must be finite
 * and nonnegative.  Calls that overlap on one device race on the shared array: the caller
 * serialises them (one stream, or events).
 */
#define DID_STATIC_SCRATCH_BYTES ((int64_t)128 << 20)
int did_iterate_static(const float* X, int64_t M, int64_t N, int32_t K, float* B, float* C, int32_t n,
                       const did_opts* opts, double* f);

/* Message for the calling thread's last failure ("" if none): the reason a call returned
 * a DID_E* code (a violated condition of eq. opt:nmf's input, a shape limit, or the HIP
 * error behind DID_EDEVICE).  The string is owned by the library and valid until the next
 * call on the same thread. */
const char* did_last_error(void);

/* Debugging aid for failure handling: the next call on h that checks the handle fails
 * with DID_EDEVICE as a device error would, and h becomes sticky-failed (every later call
 * returns DID_EDEVICE; did_free still releases it).  No device work is involved.  Returns
 * DID_EINVAL for NULL. */
int did_debug_inject_fault(did_handle h);

/* Debugging aid for out-of-bounds writes: with the environment variable
 * DID_DEBUG_GUARD_ZONES set to a nonzero integer when a handle is created, each of the
 * handle's device buffers is followed by a guard zone of DID_GUARD_ZONE_BYTES bytes
 * filled with the byte DID_GUARD_BYTE.  did_debug_check_guards synchronises the handle's
 * stream (a batch member's writes are on the batch's stream: call did_batch_sync first)
 * and stores in *bad the number of guard bytes that no longer hold the pattern
 * (0: no buffer was written past its end), and in *zones (if not NULL) the number of
 * zones checked (0 for a handle made without them); the message of the first damaged zone
 * names the buffer and is kept for did_last_error.  Returns DID_EINVAL for NULL h or bad,
 * DID_EDEVICE if the copies fail. */
#define DID_GUARD_ZONE_BYTES 4096
#define DID_GUARD_BYTE 0xA5
int did_debug_check_guards(did_handle h, int64_t* bad, int32_t* zones);

#ifdef __cplusplus
}
#endif

#endif /* DID_H */
