// Internal interface between the DID engine (did_engine.hip) and its gfx950 kernels
// (did_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace didk {

// Shapes derived once per instance.
struct Shape {
  int64_t M, N;      // rows (features) and columns (samples) of X
  int K;             // coordinates
  int KP;            // K padded to the MFMA output tile (32 or 64)
  int64_t nchunks;   // ceil(M / 32): 32-row chunks of the basis
  int64_t Mpad;      // nchunks * 32
  int vec4;          // vector loads of X are aligned (M % 4 == 0 and X aligned)
  int xbf16;         // X is stored as bf16 (reduced-precision storage form), else float32
  int xtiled;        // X is stored in tile order (always for bf16; float32 on request)
  int thin;          // thin-matrix path (M <= 16, K <= 8, M <= 8 or K <= 4): one fused pass per iteration
  int cwpb;          // waves per column-pass block (4 or 8): the block's 32 cwpb columns share one staged B
  int64_t thin_grid; // thin path: blocks per launch (one wave of resident blocks)
};

// Packed B: per 32-row chunk, B in the two MFMA operand orders as 16-byte units of eight
// fp16 values, E order (KP/16 * 2 * 64 units: two pieces of -B scaled per row) then H order
// (KP/32 * 2 * 2 * 64 units, the same count: two pieces of B scaled per column), then 8
// units holding the chunk's 32 row scales as float32, so that one chunk's operands are
// one contiguous run of bq_units_chunk units.
constexpr inline int bq_units_e(int KP) { return (KP / 16) * 2 * 64; }
constexpr inline int bq_units_chunk(int KP) { return 2 * bq_units_e(KP) + 8; }
// fp16 entries of the packed B buffer
inline int64_t packed_b_elems(const Shape& s) { return s.nchunks * (int64_t)bq_units_chunk(s.KP) * 8; }
inline int n_pairs(int KP) { return KP * (KP + 1) / 2; }

// Packed C: per 32-column tile, C in the two MFMA operand orders, as 16-byte units of eight
// fp16 values: E order (KP/16 * 2 * 64 units: two pieces of C scaled per column, then 8
// units holding the tile's 32 inverse column scales as float32) and W order
// (KP/32 * 2 * 2 * 64 units: two pieces of C scaled per row).
constexpr inline int cq_units_e(int KP) { return (KP / 16) * 2 * 64 + 8; }
constexpr inline int cq_units_w(int KP) { return (KP / 32) * 2 * 2 * 64; }
constexpr inline int cq_units(int KP) { return cq_units_e(KP) + cq_units_w(KP); }
inline int64_t n_tiles32(const Shape& s) { return (s.N + 31) / 32; }
// bytes of the packed C buffer
inline int64_t cq_bytes(const Shape& s) { return n_tiles32(s) * cq_units(s.KP) * 16; }
// Column scales of B for the H-order operands (Bsc), and row scales of C for the W-order
// operands (Csc): floats [0, KP) hold the maxima (gathered by the kernel that changes the
// factor), [KP, 2 KP) the inverse scales.
inline int bsc_floats(int KP) { return 2 * KP; }

// splitmix64 finaliser (Steele, Lea & Flood, OOPSLA 2014).
__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(seed ^ (stream * 0xD1B54A32D192ED03ull));
}

// Column ranges of the row pass, in 32-column tiles: P contiguous blocks of the T tiles
// (the paper's shards; block p holds tiles [T p / P, T (p+1) / P)), each split into up to S
// sub-ranges.  Writes the R + 1 bounds into b (if not null) and returns R.  Shared by the
// host plan and the device kernel that the allocation-free entry point uses.
__host__ __device__ inline int64_t range_bounds(int64_t T, int64_t P, int64_t S, int64_t* b) {
  int64_t r = 0;
  if (b) b[0] = 0;
  for (int64_t p = 0; p < P; ++p) {
    const int64_t a0 = T * p / P, a1 = T * (p + 1) / P, n = a1 - a0;
    const int64_t Sp = S < n ? (S > 1 ? S : 1) : (n > 1 ? n : 1);
    for (int64_t q = 1; q <= Sp; ++q) {
      ++r;
      if (b) b[r] = a0 + (n * q) / Sp;
    }
  }
  return r;
}

// ---- launchers (all asynchronous on `st`; they return the launch status) ----
// zero `bytes` (a multiple of 16) bytes at the 16-byte aligned p with a fill kernel
hipError_t zero16(void* p, int64_t bytes, hipStream_t st);
// range_bounds on the device into tb (R + 1 entries)
hipError_t ranges_on_device(int64_t* tb, int64_t T, int64_t P, int64_t S, hipStream_t st);
hipError_t fill_uniform(float* out, int64_t n, uint64_t key, hipStream_t st);
hipError_t validate(const float* p, int64_t n, int vec4, int* flag, hipStream_t st);
// Tiled storage of X (the bf16 form, and the float32 form on request): two copies in
// 32 x 32 tile order, one per pass, zero-padded to
// Mpad x (32 * ntiles).  A tile holds 1024 values as 16-byte units, E = 8 (bf16) or 4
// (float32) values per unit, 16 / E units per lane: unit q*64 + l, element t is value
// i = E q + t of lane l's MFMA accumulator tile, for l = 32h + r:
//   column-pass copy XC, tile (T, c) at (T * nchunks + c) * 1024:
//       X[32c + 8(i/4) + 4h + i%4][32T + r]      (the accumulator layout of X)
//   row-pass copy XR, tile (c, T) at (c * ntiles + T) * 1024:
//       X[32c + r][32T + 8(i/4) + 4h + i%4]      (the accumulator layout of X^T)
// so that a pass loads a lane's 16 values with two 16-byte loads and a wave's tile in two
// fully used 1 kB runs.  bf16 values are rounded to nearest even.
inline int64_t n_tiles(const Shape& s) { return (s.N + 31) / 32; }
inline int64_t tiled_x_elems(const Shape& s) { return s.nchunks * n_tiles(s) * 1024; }
// xc and xr each hold tiled_x_elems(s) values of the storage type (s.xbf16)
hipError_t tile_x(const Shape& s, const float* src, void* xc, void* xr, hipStream_t st);
hipError_t scale(float* p, int64_t n, float a, hipStream_t st);

// Pack B into MFMA operand order (Bq, layout above; Bsc: its column scales), optionally
// applying the incremental B update from the reduced messages W (KP x Mpad, float64) and V
// (KP x KP, float64) first; writes per-block partials of B^T B into Gpart (n_pairs(KP)
// doubles per block).  The thin path packs nothing (Bq and Bsc may be null there).
// With BqD (carried-residual form) the change delta B of the update is also packed there
// (E-order units and row scales, the layout of Bq).
hipError_t bupdate(const Shape& s, float* B, const double* W, const double* V, _Float16* Bq, float* Bsc,
                   double* Gpart, int update, hipStream_t st, _Float16* BqD = nullptr);
int bupdate_blocks(const Shape& s);

// Column pass: E = X - BC per 32-column tile, one partial of sum E^2 per block, and
// (with_h = 1) H = B^T E written as KP x N floats, row kk contiguous (index kk * N + j).
// C enters through its packed pieces Cq.
hipError_t colpass(const Shape& s, const void* X, const void* Cq, const _Float16* Bq, const float* Bsc,
                   float* Hout, double* fpart, int with_h, hipStream_t st);
int64_t colpass_blocks(const Shape& s);  // blocks of 32 cwpb columns

// Carried-residual form (refresh_every > 1) of the two passes; R is the column-major
// float32 residual (M x N, ld M), carried across iterations.
//   colpass_carry: refresh = 1: E = X - B C from the stored X; refresh = 0: E = R - dB C
//     (dB = the last B update's change, packed in BqD by bupdate); H = B^T E, the f
//     partials, and E stored into R.
//   rowpass_carry: E' = R - B dC (dC = C' - C, packed in CqD by the sweep), the W
//     partials with C' from Cq, and E' stored into R.
hipError_t colpass_carry(const Shape& s, const void* X, int refresh, const void* Cq, const _Float16* Bq,
                         const _Float16* BqD, const float* Bsc, float* Hout, double* fpart, float* R,
                         hipStream_t st);
hipError_t rowpass_carry(const Shape& s, float* R, const void* Cq, const void* CqD, const float* Csc,
                         const _Float16* Bq, float* Wpart, const int64_t* tb, int Rn, hipStream_t st);

// Coordinate sweep over the rows of C from H and G = B^T B (float64), in place on C, and
// repacking of the updated columns into Cq (row scales in Csc).
// With CqD (carried-residual form) delta C = C' - C is also packed there (E-order units
// and inverse column scales, CqL<KP>::E units per tile: cqd_bytes).
hipError_t sweep(const Shape& s, const float* Hin, float* C, void* Cq, float* Csc, const double* G,
                 hipStream_t st, void* CqD = nullptr);
inline int64_t cqd_bytes(const Shape& s) { return n_tiles32(s) * cq_units_e(s.KP) * 16; }
// Pack C into Cq (after C was set from outside the sweep).
hipError_t packc(const Shape& s, const float* C, void* Cq, float* Csc, hipStream_t st);

// V partials: tril(C C^T) per block of tiles from the packed C (float64, n_pairs(KP) per
// block).
hipError_t vgram(const Shape& s, const void* Cq, const float* Csc, double* Vpart, hipStream_t st);
int64_t vgram_blocks(const Shape& s);

// Row pass: W partial per column range r: Wpart[r] = (X - BC)[:, range] C[:, range]^T.
// Range r covers 32-column tiles [tb[r], tb[r+1]); C enters through Cq.
hipError_t rowpass(const Shape& s, const void* X, const void* Cq, const float* Csc, const _Float16* Bq, float* Wpart,
                   const int64_t* tb, int R, hipStream_t st);

// Fixed-order reductions.
hipError_t reduce_w(const Shape& s, const float* Wpart, int R, double* W, hipStream_t st);
hipError_t reduce_sym(const double* part, int64_t P, int KP, double* full, hipStream_t st);
hipError_t reduce_full(const double* part, int64_t P, int KP, double* full, hipStream_t st);
hipError_t reduce_f(const double* part, int64_t P, double* out, double scale, hipStream_t st);
// scale * sum of the partials into fhist[*tdev % cap], then *tdev += 1 (replayable)
hipError_t reduce_f_hist(const double* part, int64_t P, double* fhist, int64_t cap, int64_t* tdev, double scale,
                         hipStream_t st);
// *p = v from a kernel (no memset node, no host memory)
hipError_t set_i64(int64_t* p, int64_t v, hipStream_t st);

// ---- batched form: grouped persistent kernels over a device-resident instance table ----
// One group holds instances of one (KP, X storage, column-pass block waves) triple.  Every stage of an iteration is a
// single persistent launch whose blocks walk the concatenated work items of all the
// group's instances; an instance's items are exactly the blocks of its single-instance
// launch, run by the same device code, so its results do not depend on the batch.
constexpr int kMaxBatch = 64;  // instances per group
enum GStage { GS_COL = 0, GS_REDF, GS_SWEEP, GS_PACKW, GS_VGRAM, GS_REDV, GS_ROW, GS_REDW, GS_BUP, GS_REDG, GS_ADV, GS_N };

struct GInst {
  const void* X;   // X as the column pass reads it
  const void* XR;  // X as the row pass reads it
  float* B;
  float* C;
  void* Cq;
  float* Csc;
  _Float16* Bq;
  float* Bsc;
  float* H;
  double* fpart;
  double* G;
  double* Gpart;
  double* V;
  double* Vpart;
  float* Wpart;
  double* W;
  const int64_t* tb;
  double* fhist;  // objective history (ring of hist_cap entries)
  int64_t* tdev;  // iteration counter (index into fhist)
  double* fcur;   // latest objective, for the host
  int64_t M, N, nchunks, Mpad, hist_cap, vblocks, colblocks, bupblocks;
  int K, vec4, R, nsg;
};

struct GTable {
  int n;
  int64_t total[GS_N];
  int64_t begin[GS_N][kMaxBatch + 1];  // first item of instance i in stage st; begin[st][n] = total
  GInst inst[kMaxBatch];
};

// work items of one instance in each stage (rows of the row pass are a multiple of 8)
void ginst_items(const Shape& s, int R, int64_t items[GS_N]);
// Storage kinds of X in the batched form: float32 column-major, bf16 tiled, float32 tiled.
enum { XK_F32 = 0, XK_BF16 = 1, XK_F32_TILED = 2, XK_N = 3 };
inline int x_kind(const Shape& s) { return s.xbf16 ? XK_BF16 : (s.xtiled ? XK_F32_TILED : XK_F32); }
// persistent grid of each grouped stage kernel on the current device (resident blocks)
hipError_t group_grids(int KP, int xkind, int cwpb, int64_t grids[GS_N]);
// one iteration of every instance in the group table dtab (device memory)
hipError_t group_iteration(int KP, int xkind, int cwpb, const GTable* dtab, const int64_t grids[GS_N],
                           hipStream_t st);

// ---- thin-matrix path (did_thin.hip) ----
// mode 0: DID column work (sweep, W/V/f block partials); 1: objective partials only;
// 2: DBCD C half (sweep, f partials).
hipError_t thin_pass(const Shape& s, const float* X, const float* B, const double* G, float* C, double* part,
                     int mode, hipStream_t st);
// W (KP x Mpad), V (KP x KP) and *fout = scale * f from the block partials (with_wv = 0: f only)
hipError_t thin_reduce(const Shape& s, const double* part, double* W, double* V, double* fout, double scale,
                       int with_wv, hipStream_t st);
// one DBCD column update b_i (a pass over X and a reduction); yz holds M + 1 doubles of
// scratch (at least 17)
hipError_t dbcd_b_step(const Shape& s, const float* X, float* B, const float* C, double* part, double* yz, int i,
                       hipStream_t st);
int64_t thin_blocks(const Shape& s);
// blocks for the thin kernels on the current device (< 0: the runtime query failed)
int64_t thin_grid_for(const Shape& s);
int thin_slots(int MM, int KK);
// slots per block of the instance that runs shape s (the block partials hold thin_blocks(s)
// times as many doubles)
int thin_slots_for(const Shape& s);

}  // namespace didk
