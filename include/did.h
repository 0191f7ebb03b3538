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
 *                  that form, halving the bytes streamed per iteration; B, C, the residual
 *                  and every product stay float32-accurate and the objective is reduced in
 *                  float64, so the engine solves the problem for the rounded data exactly
 *                  as DID_F32 would.  borrow_x does not apply to DID_BF16.
 *   refresh_every  1: the residual is formed afresh from X at the start of every
 *                  iteration, as Alg. 3 does.  Other values are reserved (DID_EINVAL):
 *                  carrying the residual between refreshes would stream and write 8 bytes
 *                  per entry per pass instead of re-reading 2 or 4 bytes of X.
 *   init_scale     0: initial B, C are U[0,1) draws as they are.  1: both are then scaled
 *                  by sqrt(alpha), alpha = <X, BC> / ||BC||_F^2, which minimises f over a
 *                  common scale (the experiments' "well scaled initial points").
 *   borrow_x       0: X is copied into engine-owned memory.  1: a device X is adopted
 *                  without a copy; the caller keeps it alive and unmodified until
 *                  did_free.  Ignored (copy) for host pointers.
 *   algorithm      DID_ALG_DID (default) or DID_ALG_DBCD.  DBCD is available on the
 *                  thin-matrix path only (DID_EINVAL otherwise).
 *   stream         hipStream_t to order all work on; NULL = a stream owned by the handle.
 *
 * Shapes with M <= 16, K <= 8 and M <= 8 or K <= 4 (such as the experiments' synthetic
 * sets, M = 5, K = 3) run on a thin-matrix path that keeps each column in registers and makes one fused pass
 * over X per iteration; other shapes run the MFMA column/row passes.
 */
typedef struct did_opts {
  int32_t n_blocks;
  int32_t x_dtype;
  int32_t refresh_every;
  int32_t init_scale;
  int32_t borrow_x;
  int32_t algorithm;
  void* stream;
} did_opts;

/* Fill *opts with the defaults: n_blocks 0, DID_F32, refresh_every 1, init_scale 0,
 * borrow_x 0, DID_ALG_DID, stream NULL.  Returns DID_EINVAL for a NULL pointer. */
int did_default_opts(did_opts* opts);

/*
 * Create an instance for X (M x N, column-major float32, host or device pointer; a host
 * pointer is uploaded) with K coordinates, and draw the initial factors.
 *   X must be finite and >= 0 (eq. opt:nmf takes X in R_+^{M x N}); a negative, NaN or
 *   infinite entry returns DID_EINVAL.
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
 * Copy the current factors out: B (M x K, ld M) and C (K x N, ld K), float32.  Either
 * pointer may be NULL to skip it; each may be host or device memory the caller owns.
 * Synchronises the handle's stream.
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
 */
int did_profile(did_handle h, int32_t enable);
int did_profile_read(did_handle h, double* ms, int32_t cap, int32_t* n_stages, int64_t* n_iters);
const char* did_stage_name(int32_t stage);

/* Release every engine-owned resource of h.  NULL is a no-op (returns DID_OK). */
int did_free(did_handle h);

/* Message for the calling thread's last failure ("" if none).  Valid until the next
 * call on the same thread. */
const char* did_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DID_H */
