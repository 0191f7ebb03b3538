// gfx950 kernels of the DID engine.
//
// One DID iteration (Alg. 3 of Gao & Chu, AAAI-18) is carried out as
//   colpass column pass over X: E = X - B C (MFMA), f partial = sum E^2 (float64),
//           H = B^T E (MFMA),
//   sweep   the coordinate sweep over the rows of C (float64, one thread per column),
//   vgram   V = tril(C C^T) partials of the updated C (MFMA, float64 sums),
//   rowpass row pass over X: E' = X - B C' (MFMA) and W = E' C'^T per column range (MFMA),
//   reduce  fixed-order sums of the V, W and f partials (the paper's one Allreduce),
//   bupdate incremental update of the columns of B, one thread per row of B.
// Every MFMA product is float32-accurate: each float32 operand is split into two fp16
// pieces under a power-of-two scale and each product is formed from three fp16 MFMAs
// (split2 and mfma_x3 below).
//
// The coordinate sweep over c_j is written in inner-product form.  With the residual
// e_j of the column at the start of the sweep and h = B^T e_j, the running inner product
// b_i^T e_j after coordinates k < i moved by delta c_k is h_i - sum_{k<i} (b_i^T b_k)
// delta c_k, so eq. up:c becomes c_ij := [c_ij + (h_i - sum_{k<i} G_ik delta c_kj) / G_ii]_+
// with G = B^T B.  This is the same identity Section 4 uses for the columns of B (the
// v_ik delta b_k term); it turns the K dependent length-M reductions of the sweep into
// one MFMA contraction plus O(K^2) float64 work per column.
//
// MFMA lane layouts used (v_mfma_f32_32x32x16_f16): lane l supplies A[l%32][8(l/32) + t]
// and B[8(l/32) + t][l%32], t = 0..7; accumulator register i of lane l holds
// D[row32(i, l/32)][l%32] with row32(i, h) = 8*(i/4) + 4*h + i%4.  Because the
// accumulator's row index pairs with l/32, accumulator registers 8q..8q+7 can be fed back
// directly (after the split) as the B operand of a second MFMA that reduces over those
// sixteen rows; no lane shuffles are needed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "did_kernels.h"

namespace didk {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int row32(int i, int h) { return 8 * (i >> 2) + 4 * h + (i & 3); }

// 16-byte unit counts of the packed operand buffers (layouts at the packing code below),
// the single definition every kernel takes its offsets and strides from.
template <int KP>
struct CqL {  // one 32-column tile of packed C
  static constexpr int E0 = (KP / 16) * 2 * 64;  // E-order units
  static constexpr int E = E0 + 8;               // ... and the tile's 32 inverse column scales
  static constexpr int W = (KP / 32) * 2 * 2 * 64;  // W-order units
  static constexpr int T = E + W;
};
template <int KP>
struct BqL {  // one 32-row chunk of packed B
  static constexpr int E = (KP / 16) * 2 * 64;      // E-order units
  static constexpr int H = (KP / 32) * 2 * 2 * 64;  // H-order units
  static constexpr int S = E + H;                   // the chunk's 32 row scales start here
  static constexpr int C = S + 8;
};
static_assert(CqL<32>::T == cq_units(32) && CqL<64>::T == cq_units(64), "packed C layout");
static_assert(CqL<32>::E == cq_units_e(32) && CqL<64>::E == cq_units_e(64), "packed C layout");
static_assert(BqL<32>::C == bq_units_chunk(32) && BqL<64>::C == bq_units_chunk(64), "packed B layout");
static_assert(BqL<32>::E == bq_units_e(32) && BqL<64>::E == bq_units_e(64), "packed B layout");

// Scaled two-way fp16 split, used for the products whose operands carry a power-of-two
// scale per row, column or tile.  For a value y whose scale group has its largest magnitude
// in [2^14, 2^15), hi = fp16(y) and lo = fp16(y - hi) (both rounded to nearest even; y - hi
// is exact in float32).  For |y| >= 2^-3 both pieces are normal fp16 numbers and
// |y - hi - lo| <= 2^-22 |y|; smaller values keep an absolute error below 2^-25 (the fp16
// subnormal spacing), 2^-40 of the group's largest magnitude.  A float32 product a*b is
// then formed from the three piece products hi*hi, hi*lo, lo*hi (each exact in float32,
// accumulated in float32 by the MFMA); the dropped lo*lo is below 2^-22 |a b|.  (A
// three-way bf16 split by truncation reaches the same accuracy with six MFMAs per product:
// bf16 keeps the float32 exponent range, but its 8-bit significand needs a third piece.)
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
struct Split2 {
  f16x8 p[2];
};

typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// y - hi for the low (SEL = 0) or high (SEL = 1) fp16 half of hp, in one mixed-precision
// fma (v_fma_mix_f32 widens the fp16 operand inside the instruction).  Exact: y - hi is a
// float32 number, so this is the same value as y - (float)hi.
template <int SEL>
__device__ __forceinline__ float sub_f16(float y, f16x2 hp) {
  float r;
  const unsigned u = __builtin_bit_cast(unsigned, hp);
  if constexpr (SEL == 0)
    asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(u), "v"(y));
  else
    asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(u), "v"(y));
  return r;
}

// hi: two values per packed conversion; lo = fp16(y - hi) with y - hi formed from the
// packed hi directly, so a value costs two instructions (rather than a scalar conversion
// and its inverse, a subtraction and a share of two packings).
__device__ __forceinline__ Split2 split2(const float (&v)[8]) {
  Split2 r;
#pragma unroll
  for (int t = 0; t < 8; t += 2) {
    f16x2 hp;
    hp.x = (_Float16)v[t];
    hp.y = (_Float16)v[t + 1];
    const float l0 = sub_f16<0>(v[t], hp);
    const float l1 = sub_f16<1>(v[t + 1], hp);
    r.p[0][t] = hp.x;
    r.p[0][t + 1] = hp.y;
    r.p[1][t] = (_Float16)l0;
    r.p[1][t + 1] = (_Float16)l1;
  }
  return r;
}

// v_mfma_f32_32x32x16_f16: D(32x32, fp32) += A(32x16) B(16x32); lane l supplies
// A[l%32][8(l/32) + t] and B[8(l/32) + t][l%32] for t = 0..7 (the layout at the top).
__device__ __forceinline__ f32x16 mfma16h(f16x8 a, f16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// acc += a * b as three fp16 MFMAs, smallest terms first.
__device__ __forceinline__ f32x16 mfma_x3(const f16x8 (&a)[2], const f16x8 (&b)[2], f32x16 acc) {
  acc = mfma16h(a[1], b[0], acc);
  acc = mfma16h(a[0], b[1], acc);
  acc = mfma16h(a[0], b[0], acc);
  return acc;
}

__device__ __forceinline__ f16x8 as_f16x8(f32x4 v) { return __builtin_bit_cast(f16x8, v); }
__device__ __forceinline__ f32x4 f16_as_f32x4(f16x8 v) { return __builtin_bit_cast(f32x4, v); }

// Scale exponent of a group whose largest magnitude is x: the s with x 2^s in [2^14, 2^15)
// (x = m 2^e with m in [0.5, 1), so s = 15 - e), kept within [-113, 126] so that 2^s and
// 2^-s are normal float32 numbers; 0 for an all-zero group.
__device__ __forceinline__ int scale_exp(float x) {
  if (!(x > 0.0f)) return 0;
  int e;
  (void)frexpf(x, &e);
  const int s = 15 - e;
  return s < -113 ? -113 : (s > 126 ? 126 : s);
}
__device__ __forceinline__ float pow2f(int s) { return ldexpf(1.0f, s); }

// Largest spread of scale exponents at which a group of rows of B (a 32-row chunk) or of
// columns of C (a 32-column tile) shares one scale, that of its largest member.
constexpr int kUniformSpread = 2;

// Element types of X as the passes read it: float (column-major, as given), or one of the
// two tiled storages (layout in did_kernels.h), bf16 or float32 (xtf32, a distinct type so
// that the tiled loads are selected at compile time).
struct xtf32 {
  float v;
};
template <typename XT>
struct x_is_tiled {
  static constexpr bool value = std::is_same<XT, __bf16>::value || std::is_same<XT, xtf32>::value;
};

// Packed C (Cq), per 32-column tile T, in 16-byte units of eight fp16 values
// (UE = KP/16 * 2 * 64 + 8):
//   E order, unit (s*2 + p)*64 + l, element t: piece p of
//       C[16s + 8(l/32) + t][j] * 2^t_j,  j = 32T + l%32
//       (B operand of E = X - BC in the column pass; A operand of E'^T in the row pass),
//       with t_j = scale_exp(max_k C[k][j]) per column;
//   units KP/16 * 2 * 64 + u, u < 8: the inverse scales 2^-t_j of the tile's 32 columns
//       (float32, column 32T + 4u + e in element e);
//   W order, unit UE + ((b*2 + q)*2 + p)*64 + l, element t: piece p of
//       C[kk][32T + row32(8q + t, l/32)] * 2^w_kk,  kk = 32b + l%32,
//       with w_kk = scale_exp(max_j C[kk][j]) per row, over all N columns
//       (A operand of W^T in the row pass; both operands of C C^T).
// Entries with kk >= K or column >= N are zero.  The E order depends only on the column,
// so it is written by the kernel that changes C (the sweep, or k_packc); that kernel also
// gathers the row maxima into Csc[0, KP) with atomic maxima (exact, so the result does not
// depend on the order), and k_packw writes the W order afterwards, storing 2^-w_kk into
// Csc[KP + kk].
//
// dst[e] = src[e] for e = threadIdx.x, threadIdx.x + 256, ... < n (a block of 256 threads
// copying between global memory and LDS): each thread issues G loads before their stores,
// so that it waits for one memory round trip per G elements (a plain strided loop is
// compiled as load, wait, store).
template <int G = 16>
__device__ __forceinline__ void block_copy(float* dst, const float* src, int n) {
  int e = threadIdx.x;
  for (; e + (G - 1) * 256 < n; e += G * 256) {
    float v[G];
#pragma unroll
    for (int u = 0; u < G; ++u) v[u] = src[e + u * 256];
#pragma unroll
    for (int u = 0; u < G; ++u) dst[e + u * 256] = v[u];
  }
  for (; e < n; e += 256) dst[e] = src[e];
}

// pack_block takes the (up to) eight tiles of columns j0 .. j0 + nv - 1, whose values sit
// in LDS as Ct[j * K + kk] (j relative to j0); every thread builds whole 16-byte units, so
// the global stores are coalesced.  All threads of the block call it, after Ct is
// complete; it takes 256 ints of LDS scratch (cs) from the caller.
// DELTA: the values are a signed change of C (the carried-residual form packs delta C into
// its own buffer of E-order units only, tile stride CqL<KP>::E): the column scales come
// from the largest magnitude and no row maxima are gathered.
template <int KP, bool DELTA = false>
__device__ __forceinline__ void pack_block(f32x4* __restrict__ Cq, float* __restrict__ cmax, int64_t j0, int nv,
                                           const float* Ct, int K, int64_t ntiles, int* cs) {
  constexpr int KS = KP / 16;
  constexpr int UE0 = CqL<KP>::E0;
  constexpr int UT = DELTA ? CqL<KP>::E : CqL<KP>::T;  // units per tile of the target buffer
  constexpr int GE = 8 * KS * 64;  // E groups per block: (tile, s, half, jj)
  const int tid = threadIdx.x;     // cs[j]: scale exponent of column j0 + j
  const int64_t T0 = j0 >> 5;
  {
    float mx = 0.0f;
    if (tid < nv)
      for (int kk = 0; kk < K; ++kk) mx = fmaxf(mx, DELTA ? fabsf(Ct[tid * K + kk]) : Ct[tid * K + kk]);
    int sc = scale_exp(mx);
    if constexpr (!DELTA) {
      // a tile's 32 columns are 32 consecutive lanes: when the scales of its nonzero columns
      // lie within kUniformSpread of each other, every column takes the smallest, so that
      // the passes scale the tile's products with one multiplier (the tile is then flagged
      // by the sign of its first inverse scale, below)
      const bool has = tid < nv && mx > 0.0f;
      int smin = has ? sc : INT_MAX, smax = has ? sc : INT_MIN;
#pragma unroll
      for (int off = 1; off < 32; off <<= 1) {
        smin = min(smin, __shfl_xor(smin, off, 64));
        smax = max(smax, __shfl_xor(smax, off, 64));
      }
      if (smin <= smax && smax - smin <= kUniformSpread) sc = smin;
    }
    cs[tid] = sc;
  }
  if (!DELTA && tid < K) {  // row maxima over the block's columns (C >= 0: integer order = float order)
    float mx = 0.0f;
    for (int j = 0; j < nv; ++j) mx = fmaxf(mx, Ct[j * K + tid]);
    if (mx > 0.0f) atomicMax(reinterpret_cast<int*>(cmax) + tid, __float_as_int(mx));
  }
  __syncthreads();
  for (int g = tid; g < GE; g += 256) {
    const int tb = g / (KS * 64), rem = g % (KS * 64), sh = rem >> 5, jj = rem & 31;
    const int s = sh >> 1, h = sh & 1;
    if (T0 + tb >= ntiles) continue;
    const int j = 32 * tb + jj;
    const float sc = pow2f(cs[j]);
    float v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int kk = 16 * s + 8 * h + t;
      v[t] = (j < nv && kk < K) ? Ct[j * K + kk] * sc : 0.0f;
    }
    const Split2 sp = split2(v);
    f32x4* tile = Cq + (T0 + tb) * UT;
#pragma unroll
    for (int p = 0; p < 2; ++p) tile[(s * 2 + p) * 64 + jj + 32 * h] = f16_as_f32x4(sp.p[p]);
  }
  if (tid < 64) {  // inverse scales: tile tid / 8, unit tid % 8
    const int tb = tid >> 3, u = tid & 7;
    if (T0 + tb < ntiles) {
      f32x4 w;
#pragma unroll
      for (int e = 0; e < 4; ++e) w[e] = pow2f(-cs[32 * tb + 4 * u + e]);
      if (!DELTA && u == 0) {  // all 32 columns on one scale: the sign of the first flags it
        bool same = true;
        for (int j = 1; j < 32; ++j) same = same && cs[32 * tb + j] == cs[32 * tb];
        if (same) w[0] = -w[0];
      }
      Cq[(T0 + tb) * UT + UE0 + u] = w;
    }
  }
}

// W-order units of the eight tiles of columns 256 bid .. 256 bid + 255, read straight from
// C (each group's eight loads are coalesced across the lanes, which take consecutive
// coordinates), with the row scales from the maxima in Csc[0, KP); block 0 stores the
// inverse scales into Csc[KP, 2 KP).  No LDS staging, so that many blocks stay resident.
template <int KP>
__device__ __forceinline__ void packw_body(const float* __restrict__ C, f32x4* __restrict__ Cq,
                                           float* __restrict__ Csc, int64_t N, int K, int64_t bid) {
  constexpr int NB = KP / 32;
  constexpr int UE = CqL<KP>::E;
  constexpr int UT = CqL<KP>::T;
  constexpr int GW = 8 * NB * 128;  // W groups per block: (tile, b, q, lane)
  static_assert(GW % 512 == 0, "two groups per thread and step");
  __shared__ float ws[KP];
  const int tid = threadIdx.x;
  const int64_t j0 = bid * 256, T0 = bid * 8, ntiles = (N + 31) / 32;
  if (tid < KP) {
    const int w = tid < K ? scale_exp(Csc[tid]) : 0;
    ws[tid] = pow2f(w);
    if (bid == 0) Csc[KP + tid] = pow2f(-w);
  }
  __syncthreads();
  // two groups per step (g and g + 256; GW is a multiple of 512): their sixteen loads are
  // issued before either group is split and stored
  for (int g0 = tid; g0 < GW; g0 += 512) {
    float v[2][8];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int g = g0 + 256 * r;
      const int tb = g / (NB * 128), rem = g % (NB * 128), bq = rem >> 6, l = rem & 63;
      const int b = bq >> 1, q = bq & 1;
      const int kk = 32 * b + (l & 31), h = l >> 5;
      const bool ok = T0 + tb < ntiles && kk < K;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int64_t j = j0 + 32 * tb + row32(8 * q + t, h);
        v[r][t] = (ok && j < N) ? C[j * K + kk] : 0.0f;
      }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int g = g0 + 256 * r;
      const int tb = g / (NB * 128), rem = g % (NB * 128), bq = rem >> 6, l = rem & 63;
      const int b = bq >> 1, q = bq & 1;
      if (T0 + tb >= ntiles) continue;
      const int kk = 32 * b + (l & 31);
      const float sc = ws[kk];
#pragma unroll
      for (int t = 0; t < 8; ++t) v[r][t] *= sc;
      const Split2 sp = split2(v[r]);
      f32x4* tile = Cq + (T0 + tb) * UT;
#pragma unroll
      for (int p = 0; p < 2; ++p) tile[UE + ((b * 2 + q) * 2 + p) * 64 + l] = f16_as_f32x4(sp.p[p]);
    }
  }
}

// Pair index q -> (a, b) with a >= b, q = a(a+1)/2 + b.
__device__ __forceinline__ void pair_of(int q, int& a, int& b) {
  int r = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= q) ++r;
  while (r * (r + 1) / 2 > q) --r;
  a = r;
  b = q - r * (r + 1) / 2;
}

// ------------------------------------------------------------------ initial draws
__global__ void k_fill_uniform(float* out, int64_t n, uint64_t key) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t z = mix64(key + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull);
    out[i] = (float)(z >> 40) * 0x1.0p-24f;  // 24 random bits: exact in float32, [0, 1)
  }
}

hipError_t fill_uniform(float* out, int64_t n, uint64_t key, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_fill_uniform<<<(unsigned)blocks, 256, 0, st>>>(out, n, key);
  return hipGetLastError();
}

__global__ void k_scale(float* p, int64_t n, float a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] *= a;
}

hipError_t scale(float* p, int64_t n, float a, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_scale<<<(unsigned)blocks, 256, 0, st>>>(p, n, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ tiled storage of X
// Both tiled copies of X (layout in did_kernels.h), elements of type T (bf16 rounded to
// nearest even, or float32); one thread per 16-byte unit of each copy, zero outside M x N.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <typename ET>
__global__ void k_tile_x(const float* __restrict__ src, int64_t M, int64_t N, int64_t nchunks, int64_t ntiles,
                         ET* __restrict__ xc, ET* __restrict__ xr) {
  constexpr int E = 16 / (int)sizeof(ET);  // values per unit
  constexpr int Q = 16 / E;               // units per lane
  const int64_t units = nchunks * ntiles * 64 * Q;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < units; u += stride) {
    const int64_t tile = u / (64 * Q);  // the same index in both copies' own tile order
    const int q = (int)(u / 64 % Q), l = (int)u & 63, h = l >> 5, r = l & 31;
    const int64_t at = tile * 1024 + (int64_t)(q * 64 + l) * E;
    {  // column-pass copy: tile (T, c)
      const int64_t T = tile / nchunks, c = tile - T * nchunks;
      const int64_t j = T * 32 + r;
      ET v[E];
#pragma unroll
      for (int t = 0; t < E; ++t) {
        const int i = E * q + t;
        const int64_t m = c * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
        v[t] = (ET)((m < M && j < N) ? src[j * M + m] : 0.0f);
      }
      *reinterpret_cast<u32x4*>(xc + at) = __builtin_bit_cast(u32x4, v);
    }
    {  // row-pass copy: tile (c, T)
      const int64_t c = tile / ntiles, T = tile - c * ntiles;
      const int64_t m = c * 32 + r;
      ET v[E];
#pragma unroll
      for (int t = 0; t < E; ++t) {
        const int i = E * q + t;
        const int64_t j = T * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
        v[t] = (ET)((m < M && j < N) ? src[j * M + m] : 0.0f);
      }
      *reinterpret_cast<u32x4*>(xr + at) = __builtin_bit_cast(u32x4, v);
    }
  }
}

hipError_t tile_x(const Shape& s, const float* src, void* xc, void* xr, hipStream_t st) {
  const int64_t units = s.nchunks * n_tiles(s) * 64 * (s.xbf16 ? 2 : 4);
  int64_t blocks = (units + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (s.xbf16)
    k_tile_x<__bf16><<<(unsigned)blocks, 256, 0, st>>>(src, s.M, s.N, s.nchunks, n_tiles(s),
                                                        static_cast<__bf16*>(xc), static_cast<__bf16*>(xr));
  else
    k_tile_x<float><<<(unsigned)blocks, 256, 0, st>>>(src, s.M, s.N, s.nchunks, n_tiles(s), static_cast<float*>(xc),
                                                       static_cast<float*>(xr));
  return hipGetLastError();
}

// The 16 values of one lane's accumulator tile from a tiled copy of X.
__device__ __forceinline__ f32x16 ld_tile(const __bf16* tile, int l) {
  f32x16 v;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const u32x4 w = *reinterpret_cast<const u32x4*>(tile + (q * 64 + l) * 8);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[8 * q + 2 * k] = __builtin_bit_cast(float, w[k] << 16);
      v[8 * q + 2 * k + 1] = __builtin_bit_cast(float, w[k] & 0xffff0000u);
    }
  }
  return v;
}
__device__ __forceinline__ f32x16 ld_tile(const xtf32* tile, int l) {
  f32x16 v;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const f32x4 w = *reinterpret_cast<const f32x4*>(tile + (q * 64 + l) * 4);
#pragma unroll
    for (int k = 0; k < 4; ++k) v[4 * q + k] = w[k];
  }
  return v;
}

// ------------------------------------------------------------------ validation
// flag |= 1 if any entry is negative, NaN or infinite (X must lie in R_+^{M x N}).
__global__ void k_validate(const float* p, int64_t n, int vec4, int* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int bad = 0;
  if (vec4) {
    const int64_t n4 = n / 4;
    const f32x4* p4 = reinterpret_cast<const f32x4*>(p);
    for (int64_t i = t0; i < n4; i += stride) {
      const f32x4 v = p4[i];
      for (int u = 0; u < 4; ++u) bad |= !(v[u] >= 0.0f && v[u] <= 3.4028234663852886e38f);
    }
    for (int64_t i = 4 * n4 + t0; i < n; i += stride) bad |= !(p[i] >= 0.0f && p[i] <= 3.4028234663852886e38f);
  } else {
    for (int64_t i = t0; i < n; i += stride) bad |= !(p[i] >= 0.0f && p[i] <= 3.4028234663852886e38f);
  }
  if (bad) atomicOr(flag, 1);
}

hipError_t validate(const float* p, int64_t n, int vec4, int* flag, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n / (vec4 ? 4 : 1) + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 16384) blocks = 16384;
  k_validate<<<(unsigned)blocks, 256, 0, st>>>(p, n, vec4, flag);
  return hipGetLastError();
}

// ------------------------------------------------------------------ B update + packing
// Packed operand buffer of B (rows >= M and columns >= K stay zero from allocation).  A
// 16-byte unit holds the eight fp16 values lane l feeds to one MFMA; chunk c's units form
// one contiguous run of UC = 2 * UE + 8 units (UE = KP/16 * 2 * 64):
//   unit c*UC + (s*2 + p)*64 + l, element t: piece p of -B[m][16s + 8(l/32) + t] * 2^s_m,
//       m = 32c + l%32, with s_m = scale_exp(max_k B[m][k])  (A operand of E = X - B C in
//       the column pass; B operand of E'^T in the row pass);
//   unit c*UC + UE + ((b*2 + q)*2 + p)*64 + l, element t: piece p of
//       B[32c + row32(8q + t, l/32)][kk] * 2^u_kk, kk = 32b + l%32, with
//       u_kk = scale_exp(max_m B[m][kk])   (A operand of H = B^T E);
//   units c*UC + 2*UE + u, u < 8: 2^-s_m of rows m = 32c + 4u + e (float32, element e).
// The per-row part is written by the B update (one thread per row); the per-column part
// needs the column maxima over all rows, which the B update gathers into Bsc[0, KP) with
// atomic maxima (exact, so the result does not depend on the order), and is written by
// k_packh afterwards, which also stores 2^-u_kk into Bsc[KP + kk].
constexpr int kBupRows = 64;      // rows of B per block (one thread each for the update)
constexpr int kBupThreads = 256;  // threads per block (all of them form the G partial)

// RW (the carried-residual form): the change delta B = B^{t+1} - B^t of the stored float32
// values is also packed, as E-order units of -delta B scaled per row with the row's inverse
// scale, into BqD (the layout of Bq), for the next column pass's update of the residual.
// HOIST: the row's values of B are all loaded before the first coordinate moves (the
// single-instance kernel); the grouped kernel loads each as it goes, which keeps it at two
// waves per SIMD (with the hoisted loads it needs 256 VGPRs).
template <int KP, bool RW = false, bool HOIST = true>
__device__ __forceinline__ void bupdate_body(float* __restrict__ B, int64_t M, int K, const double* __restrict__ W,
                                             int64_t Mpad, const double* __restrict__ V, _Float16* __restrict__ Bq,
                                             float* __restrict__ bmax, double* __restrict__ Gpart, int update,
                                             int64_t bid, _Float16* __restrict__ BqD = nullptr) {
  constexpr int64_t UC = BqL<KP>::C;
  constexpr int US = BqL<KP>::S;
  __shared__ float dfl[RW ? KP * kBupRows : 1];  // delta B of the stored values, [i][row]
  // V is the same for every row.  The whole block stages it in LDS before the update (a
  // few memory round trips in all), since the update's dependent chain would otherwise wait
  // on a load of V at every coordinate: V was just written by another kernel, on whichever
  // XCD, and a scalar load of it misses this XCD's caches.
  __shared__ double Vs[KP * (KP + 1) / 2];  // lower triangle, row-major pairs
  __shared__ float Bt[kBupRows * (KP + 1)];
  const int tid = threadIdx.x;
  if (update)
    for (int q = tid; q < KP * (KP + 1) / 2; q += kBupThreads) {
      int a, b;
      pair_of(q, a, b);
      Vs[q] = V[a * KP + b];
    }
  auto vv = [&](int a, int b) -> double { return Vs[a * (a + 1) / 2 + b]; };  // V[a][b] for a >= b
  __syncthreads();
  const int64_t m = bid * kBupRows + tid;
  const bool ok = m < M;
  if (tid < kBupRows) {  // the row update, one thread per row of B
    float mx = 0.0f;
    // sq[q] = w_q - sum_{k < i} v_qk delta b_k for the coordinates q not yet updated: once
    // coordinate i has moved, every later sq[q] takes its term at once, so the terms still
    // arrive in ascending k (the order of the sum in the update rule) while the dependent
    // chain per coordinate is one division and one FMA.  A skipped coordinate (v_ii = 0: a
    // zero row of C, whose row of V is zero too) moves by delta b_i = +0.
    // The coordinates run to KQ, K rounded up to a multiple of 8 (a compile-time bound, so
    // that sq stays in registers and no FMA is spent on the padding up to KP).
    auto rows = [&](auto kq) {
      constexpr int KQ = decltype(kq)::value;
      double sq[KP];
      float bo[KP];  // the row's current values (HOIST)
      if constexpr (HOIST) {
#pragma unroll
        for (int q = 0; q < KQ; ++q) bo[q] = (q < K && ok) ? B[(int64_t)q * M + m] : 0.0f;
      }
      if (update) {
#pragma unroll
        for (int q = 0; q < KQ; ++q) sq[q] = (q < K && ok) ? W[(int64_t)q * Mpad + m] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < KP; ++i) {
        float bnew = 0.0f;
        if (i < KQ && i < K && ok) {
          double bold;
          if constexpr (HOIST)
            bold = (double)bo[i];
          else
            bold = (double)B[(int64_t)i * M + m];
          double bn = bold;
          if (update) {
            const double vii = vv(i, i);
            if (vii > 0.0) {
              bn = bold + sq[i] / vii;
              bn = bn > 0.0 ? bn : 0.0;
            }
            const double d = bn - bold;
#pragma unroll
            for (int q = i + 1; q < KQ; ++q) sq[q] -= vv(q, i) * d;
          }
          bnew = (float)bn;
          if (update) B[(int64_t)i * M + m] = bnew;
          if constexpr (RW) dfl[i * kBupRows + tid] = (float)((double)bnew - bold);
        } else if constexpr (RW) {
          dfl[i * kBupRows + tid] = 0.0f;
        }
        Bt[tid * (KP + 1) + i] = bnew;
        mx = fmaxf(mx, bnew);
      }
    };
    // K <= 32 runs with KP = 32 and 32 < K <= 64 with KP = 64
    switch ((K + 7) >> 3) {
      case 1: case 5: rows(std::integral_constant<int, KP == 32 ? 8 : 40>{}); break;
      case 2: case 6: rows(std::integral_constant<int, KP == 32 ? 16 : 48>{}); break;
      case 3: case 7: rows(std::integral_constant<int, KP == 32 ? 24 : 56>{}); break;
      default: rows(std::integral_constant<int, KP>{}); break;
    }
    // Scale of row m's E-order operand.  A chunk's 32 rows are 32 consecutive lanes of this
    // wave; when the scales of its nonzero rows lie within kUniformSpread of each other,
    // every row takes the smallest (the largest row's), so that the passes scale the
    // chunk's products with one multiplier: a row then sits at most 2^kUniformSpread below
    // the top of the fp16 range, and its values keep full accuracy down to
    // 2^-(17 - kUniformSpread) of its maximum.  Row 0's stored inverse scale then carries
    // the sign bit as the chunk's flag.
    int sm = scale_exp(mx);
    bool uniform = false;
    {
      const bool has = ok && mx > 0.0f;
      int smin = has ? sm : INT_MAX, smax = has ? sm : INT_MIN;
#pragma unroll
      for (int off = 1; off < 32; off <<= 1) {  // within the lane's half of the wave
        smin = min(smin, __shfl_xor(smin, off, 64));
        smax = max(smax, __shfl_xor(smax, off, 64));
      }
      uniform = smin <= smax && smax - smin <= kUniformSpread;
      if (uniform) sm = smin;
    }
    if constexpr (RW) {  // E-order units of -delta B for row m, scaled per row, and the inverse scale
      if (ok) {
        float dm = 0.0f;
#pragma unroll
        for (int i = 0; i < KP; ++i) dm = fmaxf(dm, fabsf(dfl[i * kBupRows + tid]));
        const int sd = scale_exp(dm);
        const float scd = pow2f(sd);
        const int64_t c = m >> 5;
        const int r = (int)(m & 31);
#pragma unroll
        for (int i = 0; i < KP; ++i) {
          if (i < K) {
            const float y = -dfl[i * kBupRows + tid] * scd;
            const _Float16 hi = (_Float16)y;
            const _Float16 lo = (_Float16)(y - (float)hi);
            const int sq = i >> 4, h = (i >> 3) & 1, t = i & 7, l = r + 32 * h;
            BqD[(c * UC + (sq * 2 + 0) * 64 + l) * 8 + t] = hi;
            BqD[(c * UC + (sq * 2 + 1) * 64 + l) * 8 + t] = lo;
          }
        }
        reinterpret_cast<float*>(BqD + (c * UC + US) * 8)[r] = pow2f(-sd);
      }
    }
    if (Bq && ok) {  // E-order units of row m and its inverse scale
      const float sc = pow2f(sm);
      const int64_t c = m >> 5;
      const int r = (int)(m & 31);
#pragma unroll
      for (int i = 0; i < KP; ++i) {
        if (i < K) {
          const float y = -Bt[tid * (KP + 1) + i] * sc;
          const _Float16 hi = (_Float16)y;
          const _Float16 lo = (_Float16)(y - (float)hi);
          const int sq = i >> 4, h = (i >> 3) & 1, t = i & 7, l = r + 32 * h;
          Bq[(c * UC + (sq * 2 + 0) * 64 + l) * 8 + t] = hi;
          Bq[(c * UC + (sq * 2 + 1) * 64 + l) * 8 + t] = lo;
        }
      }
      reinterpret_cast<float*>(Bq + (c * UC + US) * 8)[r] = (uniform && r == 0) ? -pow2f(-sm) : pow2f(-sm);
    }
  }
  __syncthreads();
  if (bmax && tid < K) {  // column maxima over this block's rows (B >= 0: integer order = float order)
    float mx = 0.0f;
    for (int r = 0; r < kBupRows; ++r) mx = fmaxf(mx, Bt[r * (KP + 1) + tid]);
    if (mx > 0.0f) atomicMax(reinterpret_cast<int*>(bmax) + tid, __float_as_int(mx));
  }
  // Partial of G = B^T B over this block's rows, float64, pairs (a >= b).
  constexpr int NP = KP * (KP + 1) / 2;
  for (int q = tid; q < NP; q += kBupThreads) {
    int a, b;
    pair_of(q, a, b);
    double s0 = 0.0, s1 = 0.0;
    for (int r = 0; r < kBupRows; r += 2) {
      s0 += (double)Bt[r * (KP + 1) + a] * (double)Bt[r * (KP + 1) + b];
      s1 += (double)Bt[(r + 1) * (KP + 1) + a] * (double)Bt[(r + 1) * (KP + 1) + b];
    }
    Gpart[bid * NP + q] = s0 + s1;
  }
}

template <int KP, bool RW>
__global__ __launch_bounds__(kBupThreads) void k_bupdate(float* __restrict__ B, int64_t M, int K,
                                                 const double* __restrict__ W, int64_t Mpad,
                                                 const double* __restrict__ V, _Float16* __restrict__ Bq,
                                                 float* __restrict__ bmax, double* __restrict__ Gpart,
                                                 int update, _Float16* __restrict__ BqD) {
  bupdate_body<KP, RW>(B, M, K, W, Mpad, V, Bq, bmax, Gpart, update, blockIdx.x, BqD);
}

// H-order units of the two chunks 2*bid, 2*bid + 1 from B and the column maxima in
// Bsc[0, KP); block 0 also stores 2^-u_kk into Bsc[KP + kk].  256 threads.
template <int KP>
__device__ __forceinline__ void packh_body(const float* __restrict__ B, int64_t M, int K, int64_t nchunks,
                                           _Float16* __restrict__ Bq, float* __restrict__ Bsc, int64_t bid) {
  constexpr int NB = KP / 32;
  constexpr int UE = BqL<KP>::E;
  constexpr int64_t UC = BqL<KP>::C;
  constexpr int GC = NB * 2 * 64;  // groups (b, q, lane) per chunk
  __shared__ float us[KP];
  const int tid = threadIdx.x;
  if (tid < KP) {
    const int u = tid < K ? scale_exp(Bsc[tid]) : 0;
    us[tid] = pow2f(u);
    if (bid == 0) Bsc[KP + tid] = pow2f(-u);
  }
  __syncthreads();
  for (int g = tid; g < 2 * GC; g += 256) {
    const int64_t c = 2 * bid + g / GC;
    if (c >= nchunks) continue;
    const int rem = g % GC, bq = rem >> 6, l = rem & 63;
    const int b = bq >> 1, q = bq & 1, h = l >> 5;
    const int kk = 32 * b + (l & 31);
    const float sc = us[kk];
    float v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t m = 32 * c + row32(8 * q + t, h);
      v[t] = (m < M && kk < K) ? B[(int64_t)kk * M + m] * sc : 0.0f;
    }
    const Split2 sp = split2(v);
    f32x4* u = reinterpret_cast<f32x4*>(Bq) + c * UC + UE + (int64_t)(bq * 2) * 64 + l;
    u[0] = f16_as_f32x4(sp.p[0]);
    u[64] = f16_as_f32x4(sp.p[1]);
  }
}

template <int KP>
__global__ __launch_bounds__(256) void k_packh(const float* __restrict__ B, int64_t M, int K, int64_t nchunks,
                                               _Float16* __restrict__ Bq, float* __restrict__ Bsc) {
  packh_body<KP>(B, M, K, nchunks, Bq, Bsc, blockIdx.x);
}

__global__ void k_zero16(f32x4* p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = f32x4{0, 0, 0, 0};
}

hipError_t zero16(void* p, int64_t bytes, hipStream_t st) {
  const int64_t n = bytes / 16;
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_zero16<<<(unsigned)blocks, 256, 0, st>>>(static_cast<f32x4*>(p), n);
  return hipGetLastError();
}

__global__ void k_ranges(int64_t* tb, int64_t T, int64_t P, int64_t S) {
  if (blockIdx.x == 0 && threadIdx.x == 0) (void)range_bounds(T, P, S, tb);
}

hipError_t ranges_on_device(int64_t* tb, int64_t T, int64_t P, int64_t S, hipStream_t st) {
  k_ranges<<<1, 64, 0, st>>>(tb, T, P, S);
  return hipGetLastError();
}

__global__ void k_zero_f32(float* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0.0f;
}

int bupdate_blocks(const Shape& s) { return (int)((s.M + kBupRows - 1) / kBupRows); }

hipError_t bupdate(const Shape& s, float* B, const double* W, const double* V, _Float16* Bq, float* Bsc,
                   double* Gpart, int update, hipStream_t st, _Float16* BqD) {
  const unsigned g = (unsigned)bupdate_blocks(s);
  if (s.thin) {
    Bq = nullptr;
    Bsc = nullptr;
    BqD = nullptr;
  } else {
    k_zero_f32<<<1, 64, 0, st>>>(Bsc, s.KP);
  }
  if (BqD) {
    if (s.KP == 32)
      k_bupdate<32, true><<<g, kBupThreads, 0, st>>>(B, s.M, s.K, W, s.Mpad, V, Bq, Bsc, Gpart, update, BqD);
    else
      k_bupdate<64, true><<<g, kBupThreads, 0, st>>>(B, s.M, s.K, W, s.Mpad, V, Bq, Bsc, Gpart, update, BqD);
  } else if (s.KP == 32) {
    k_bupdate<32, false><<<g, kBupThreads, 0, st>>>(B, s.M, s.K, W, s.Mpad, V, Bq, Bsc, Gpart, update, nullptr);
  } else {
    k_bupdate<64, false><<<g, kBupThreads, 0, st>>>(B, s.M, s.K, W, s.Mpad, V, Bq, Bsc, Gpart, update, nullptr);
  }
  if (!s.thin) {
    if (s.KP == 32)
      k_packh<32><<<g, 256, 0, st>>>(B, s.M, s.K, s.nchunks, Bq, Bsc);
    else
      k_packh<64><<<g, 256, 0, st>>>(B, s.M, s.K, s.nchunks, Bq, Bsc);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ column pass
// Block = 4 waves = 128 consecutive columns; wave w owns columns 128*blockIdx + 32w ..+31
// and walks all M rows in 32-row chunks:
//   P    = (-B[chunk, :] 2^s) (C[:, cols] 2^t)     (KP/16 scaled fp16 steps)
//   acc  = X[chunk, cols] + P 2^-(s_m + t_j)        (one fma per entry) -> E = X - B C
//   fsum += sum acc^2                               (float64)
//   H   += (B[chunk, :] 2^u)^T (acc 2^v)            (2 scaled fp16 steps per 32 rows of H)
// Every float32 product is formed by three fp16 MFMAs over scaled two-way splits (split2).
// The operands of P carry one power-of-two scale per row of B and per column of C, fixed
// when they are packed; those of H one per column of B (packed) and one per column of E,
// v_j, chosen per chunk from the chunk's largest |E| in the column and never raised: when
// it drops, the running H of the column is rescaled (exactly, by a power of two) before the
// chunk is added.  Powers of two commute with rounding, so the scales change no result
// beyond the splits themselves.  The packed B run of chunk c+1 is staged into LDS (double
// buffer shared by the four waves) and the X tile of chunk c+1 is loaded into registers
// while chunk c is computed.  H is written as KP x N with row kk contiguous over the
// columns.
//
// RW (the carried-residual form): the E-order operand and the row scales of each chunk
// come from BqE (delta B in a carried iteration, B in a refresh iteration) while the
// H-order operand comes from Bq, and E is stored to the column-major float32 residual
// Rout (rvec4: 16-byte stores are aligned), so that the row pass can carry it on.  The
// source X is then either the data (refresh) or Rout itself (carry: E = R - delta B C).
template <int KP, bool WITH_H, typename XT, bool RW = false, int WPB = 4>
__device__ __forceinline__ void colpass_body(const XT* __restrict__ X, int64_t M, int64_t N, int K,
                                             const f32x4* __restrict__ Cq, const _Float16* __restrict__ Bq,
                                             const float* __restrict__ Bsc, float* __restrict__ Hout,
                                             double* __restrict__ fpart, int64_t nchunks, int vec4, int64_t bid,
                                             const _Float16* __restrict__ BqE = nullptr, float* Rout = nullptr,
                                             int rvec4 = 0) {
  constexpr int NB = KP / 32;
  constexpr int KS = KP / 16;
  constexpr int UE = BqL<KP>::E;      // 16-byte units of the E operand per chunk
  constexpr int US = BqL<KP>::S;      // the chunk's 32 row scales
  constexpr int U = BqL<KP>::C;       // the chunk's whole run
  constexpr int NV = (U + 64 * WPB - 1) / (64 * WPB);  // units per thread per chunk
  constexpr int UCT = CqL<KP>::T;     // units per packed C tile
  constexpr int UCE0 = CqL<KP>::E0;   // the tile's inverse column scales
  __shared__ f32x4 sb[2][U];
  __shared__ double fw[WPB];
  // the wave index is uniform: from a scalar register, so that wave-based addresses stay scalar
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, half = l >> 5,
            lc = l & 31;
  const int64_t T = bid * WPB + wave;  // this wave's 32-column tile
  const int64_t j0 = T * 32;
  const int64_t col = j0 + lc;
  const bool colok = col < N;
  const bool tileok = j0 < N;
  // X of this tile from a wave-uniform base plus a 32-bit lane offset
  const XT* xtile = X + (tileok ? j0 : 0) * M;
  const uint32_t loff = (uint32_t)(lc * M + 4 * half);

  f16x8 cP[KS][2];  // pieces of C[16s + 8*half + t][col] 2^t_col, from the packed tile
  float ct = 1.0f;  // 2^-t_col
  if (tileok) {
    const f32x4* ctile = Cq + T * UCT;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int p = 0; p < 2; ++p) cP[s][p] = as_f16x8(ctile[(s * 2 + p) * 64 + l]);
    ct = fabsf(reinterpret_cast<const float*>(ctile + UCE0)[lc]);  // column 0's may carry the tile's flag
  } else {
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int p = 0; p < 2; ++p) cP[s][p] = as_f16x8(f32x4{0, 0, 0, 0});
  }
  f32x16 H[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int i = 0; i < 16; ++i) H[b][i] = 0.0f;
  int vcur = 126;  // current scale exponent of this column's E operand (never raised)
  double fs0 = 0.0, fs1 = 0.0;

  f32x4 stg[NV];
  auto gload = [&](int64_t c) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int u = tid + 64 * WPB * v;
      const int uu = u < U ? u : U - 1;  // threads past the end reload the last unit
      const _Float16* base = Bq;
      if constexpr (RW) base = (uu < UE || uu >= US) ? BqE : Bq;
      const f32x4* src = reinterpret_cast<const f32x4*>(base) + c * U + uu;
      stg[v] = *src;
    }
  };
  // the residual store of the carried form: the accumulator layout of E, column-major
  float* const rtile = RW ? Rout + (tileok ? j0 : 0) * M : nullptr;
  const uint32_t roff = (uint32_t)(lc * M + 4 * half);
  const bool rfull = RW && rvec4 && tileok && (j0 + 32 <= N);  // wave-uniform
  auto rstore = [&](int64_t c, const f32x16& e) {
    const int64_t m0 = c * 32;
    if (rfull && m0 + 32 <= M) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        *reinterpret_cast<f32x4*>(rtile + m0 + 8 * q + roff) = f32x4{e[4 * q], e[4 * q + 1], e[4 * q + 2], e[4 * q + 3]};
    } else if (tileok) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int64_t r = m0 + 8 * q + 4 * half + t;
          if (colok && r < M) rtile[(int64_t)lc * M + r] = e[4 * q + t];
        }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int u = tid + 64 * WPB * v;
      if (u < U) sb[buf][u] = stg[v];
    }
  };
  const bool tilefull = vec4 && (j0 + 32 <= N);  // wave-uniform
  auto xload = [&](int64_t c) {
    f32x16 v;
    if constexpr (x_is_tiled<XT>::value) {  // tiled copy XC
      // A wave past the last tile reads tile 0, in bounds (no branch in the chunk loop);
      // its f partial is dropped and its H stores are masked by col < N.
      return ld_tile(X + ((tileok ? T : 0) * nchunks + c) * 1024, l);
    } else {  // column-major float32 X
      const int64_t m0 = c * 32;
      if (tilefull && m0 + 32 <= M) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float* xb = xtile + m0 + 8 * q;  // wave-uniform base, 32-bit lane offset
          const f32x4 t = *reinterpret_cast<const f32x4*>(xb + loff);
          v[4 * q + 0] = t[0];
          v[4 * q + 1] = t[1];
          v[4 * q + 2] = t[2];
          v[4 * q + 3] = t[3];
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t r = m0 + 8 * q + 4 * half + e;
            v[4 * q + e] = (colok && r < M) ? xtile[(int64_t)lc * M + r] : 0.0f;
          }
      }
      return v;
    }
  };

  // One chunk: compute chunk c from the X tile in xc (loaded one chunk earlier) and the
  // staged B operands in LDS buffer c & 1; meanwhile stage chunk c+1's B operands and load
  // its X tile into xn (the two tiles alternate roles from one chunk to the next, so
  // nothing is copied).
  auto step = [&](int64_t c, const f32x16& xc, f32x16& xn) {
    const int buf = (int)(c & 1);
    const int64_t cn = c + 1 < nchunks ? c + 1 : c;
    gload(cn);
    xn = xload(cn);
    // E of the chunk, a value of its own (not written over the X tile, which would make the
    // two alternating tiles cost a copy per chunk)
    f32x16 acc;
    {  // E = X - B C: KS steps of three MFMAs, operands of step s+1 read from LDS during step s
      const f32x4* ue = &sb[buf][0] + l;
      f16x8 a[2], an[2];
      f32x16 P;
#pragma unroll
      for (int i = 0; i < 16; ++i) P[i] = 0.0f;
#pragma unroll
      for (int p = 0; p < 2; ++p) a[p] = as_f16x8(ue[p * 64]);
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        if (s + 1 < KS) {
#pragma unroll
          for (int p = 0; p < 2; ++p) an[p] = as_f16x8(ue[((s + 1) * 2 + p) * 64]);
        }
        P = mfma_x3(a, cP[s], P);
        if (s + 1 < KS) {
#pragma unroll
          for (int p = 0; p < 2; ++p) a[p] = an[p];
        }
      }
      // rows row32(4q + e, half) = 8q + 4 half + e: their inverse scales are unit 2q + half.
      // A negative first scale flags a chunk whose rows share one scale (the B update):
      // one multiplier for the whole tile.
      const f32x4* rs = &sb[buf][US];
      const float s0 =
          __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, rs[0][0])));
      if (s0 < 0.0f) {
        const float mu = -s0 * ct;
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = fmaf(P[i], mu, xc[i]);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const f32x4 r4 = rs[2 * q + half];
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[4 * q + e] = fmaf(P[4 * q + e], r4[e] * ct, xc[4 * q + e]);
        }
      }
    }
    if constexpr (RW) rstore(c, acc);
    {  // sum of squares of this 32x32 tile in float32, accumulated across tiles in float64
      float a0 = 0.0f, a1 = 0.0f;
#pragma unroll
      for (int i = 0; i < 16; i += 2) {
        a0 += acc[i] * acc[i];
        a1 += acc[i + 1] * acc[i + 1];
      }
      if (c & 1) fs1 += (double)(a0 + a1);
      else fs0 += (double)(a0 + a1);
    }
    if (WITH_H) {
      // scale of this chunk's E operand: the largest |E| of the column over the chunk (the
      // lane and its partner l ^ 32 hold the column's 32 rows)
      float em = 0.0f;
#pragma unroll
      for (int i = 0; i < 16; ++i) em = fmaxf(em, fabsf(acc[i]));
      em = fmaxf(em, __shfl_xor(em, 32, 64));
      int v = scale_exp(em);
      v = (em > 0.0f && v < vcur) ? v : vcur;
      if (__ballot(v != vcur)) {  // wave-uniform: rescale only when some column's scale drops
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int i = 0; i < 16; ++i) H[b][i] = ldexpf(H[b][i], v - vcur);
        vcur = v;
      }
      const f32x4* uh = &sb[buf][UE] + l;
      f16x8 h[2], hn[2];
      f16x8 eP[2][2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        float y[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) y[t] = ldexpf(acc[8 * q + t], v);
        const Split2 sp = split2(y);
#pragma unroll
        for (int p = 0; p < 2; ++p) eP[q][p] = sp.p[p];
      }
      // accumulators alternate: (b, q) = (0, 0), (1, 0), ..., (0, 1), (1, 1), ...; each H[b]
      // still takes q = 0 before q = 1
      auto hunit = [&](int gg) { return ((gg % NB) * 2 + gg / NB) * 2; };
#pragma unroll
      for (int p = 0; p < 2; ++p) h[p] = as_f16x8(uh[(hunit(0) + p) * 64]);
#pragma unroll
      for (int gg = 0; gg < NB * 2; ++gg) {
        if (gg + 1 < NB * 2) {
#pragma unroll
          for (int p = 0; p < 2; ++p) hn[p] = as_f16x8(uh[(hunit(gg + 1) + p) * 64]);
        }
        H[gg % NB] = mfma_x3(h, eP[gg / NB], H[gg % NB]);
        if (gg + 1 < NB * 2) {
#pragma unroll
          for (int p = 0; p < 2; ++p) h[p] = hn[p];
        }
      }
    }
    sstore(buf ^ 1);
    __syncthreads();
  };

  f32x16 x0 = xload(0);
  gload(0);
  sstore(0);
  __syncthreads();
  f32x16 x1;
  for (int64_t c = 0; c < nchunks; c += 2) {
    step(c, x0, x1);
    if (c + 1 < nchunks) step(c + 1, x1, x0);
  }

  if (WITH_H && colok) {  // row kk of H contiguous over columns: coalesced stores
    const float* ku = Bsc + KP;  // 2^-u_kk
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int kk = 32 * b + row32(i, half);
        Hout[(int64_t)kk * N + col] = ldexpf(H[b][i], -vcur) * ku[kk];
      }
  }

  double fsum = fs0 + fs1;
  if (!tileok) fsum = 0.0;  // a wave past the last tile
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) fsum += __shfl_xor(fsum, off, 64);
  if (l == 0) fw[wave] = fsum;
  __syncthreads();
  if (tid == 0) {  // the block's waves in a fixed pairwise order
    double w4[2];
#pragma unroll
    for (int h = 0; h < WPB / 4; ++h) w4[h] = (fw[4 * h] + fw[4 * h + 1]) + (fw[4 * h + 2] + fw[4 * h + 3]);
    fpart[bid] = WPB == 8 ? w4[0] + w4[1] : w4[0];
  }
}

template <int KP, bool WITH_H, typename XT, int WPB>
__global__ __launch_bounds__(64 * WPB, 8 / WPB) void k_colpass(const XT* __restrict__ X, int64_t M, int64_t N, int K,
                                                               const f32x4* __restrict__ Cq,
                                                               const _Float16* __restrict__ Bq,
                                                               const float* __restrict__ Bsc, float* __restrict__ Hout,
                                                               double* __restrict__ fpart, int64_t nchunks, int vec4) {
  colpass_body<KP, WITH_H, XT, false, WPB>(X, M, N, K, Cq, Bq, Bsc, Hout, fpart, nchunks, vec4, blockIdx.x);
}

// The carried-residual form of the column pass (always forms H).
template <int KP, typename XT>
__global__ __launch_bounds__(256, 2) void k_colpass_rw(const XT* X, int64_t M, int64_t N, int K,
                                                       const f32x4* __restrict__ Cq, const _Float16* __restrict__ Bq,
                                                       const _Float16* __restrict__ BqE,
                                                       const float* __restrict__ Bsc, float* __restrict__ Hout,
                                                       double* __restrict__ fpart, int64_t nchunks, int vec4,
                                                       float* R, int rvec4) {
  colpass_body<KP, true, XT, true>(X, M, N, K, Cq, Bq, Bsc, Hout, fpart, nchunks, vec4, blockIdx.x, BqE, R, rvec4);
}

int64_t colpass_blocks(const Shape& s) {
  const int64_t cols = 32 * (int64_t)(s.cwpb == 8 ? 8 : 4);
  return (s.N + cols - 1) / cols;
}

template <typename XT, int WPB>
static void colpass_launch_w(const Shape& s, const XT* X, const f32x4* C, const _Float16* Bq, const float* Bsc,
                             float* Hout, double* fpart, int with_h, hipStream_t st) {
  const unsigned g = (unsigned)colpass_blocks(s);
  if (s.KP == 32) {
    if (with_h)
      k_colpass<32, true, XT, WPB><<<g, 64 * WPB, 0, st>>>(X, s.M, s.N, s.K, C, Bq, Bsc, Hout, fpart, s.nchunks, s.vec4);
    else
      k_colpass<32, false, XT, WPB><<<g, 64 * WPB, 0, st>>>(X, s.M, s.N, s.K, C, Bq, Bsc, Hout, fpart, s.nchunks, s.vec4);
  } else {
    if (with_h)
      k_colpass<64, true, XT, WPB><<<g, 64 * WPB, 0, st>>>(X, s.M, s.N, s.K, C, Bq, Bsc, Hout, fpart, s.nchunks, s.vec4);
    else
      k_colpass<64, false, XT, WPB><<<g, 64 * WPB, 0, st>>>(X, s.M, s.N, s.K, C, Bq, Bsc, Hout, fpart, s.nchunks, s.vec4);
  }
}

template <typename XT>
static void colpass_launch(const Shape& s, const XT* X, const f32x4* C, const _Float16* Bq, const float* Bsc,
                           float* Hout, double* fpart, int with_h, hipStream_t st) {
  if (s.cwpb == 8)
    colpass_launch_w<XT, 8>(s, X, C, Bq, Bsc, Hout, fpart, with_h, st);
  else
    colpass_launch_w<XT, 4>(s, X, C, Bq, Bsc, Hout, fpart, with_h, st);
}

template <typename XT>
static void colpass_rw_launch(const Shape& s, const XT* X, int vec4, const f32x4* C, const _Float16* Bq,
                              const _Float16* BqE, const float* Bsc, float* Hout, double* fpart, float* R,
                              hipStream_t st) {
  const unsigned g = (unsigned)colpass_blocks(s);
  const int rvec4 = (s.M % 4 == 0) && ((reinterpret_cast<uintptr_t>(R) & 15) == 0);
  if (s.KP == 32)
    k_colpass_rw<32, XT><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, C, Bq, BqE, Bsc, Hout, fpart, s.nchunks, vec4, R, rvec4);
  else
    k_colpass_rw<64, XT><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, C, Bq, BqE, Bsc, Hout, fpart, s.nchunks, vec4, R, rvec4);
}

hipError_t colpass_carry(const Shape& s, const void* X, int refresh, const void* Cqv, const _Float16* Bq,
                         const _Float16* BqD, const float* Bsc, float* Hout, double* fpart, float* R,
                         hipStream_t st) {
  const f32x4* C = static_cast<const f32x4*>(Cqv);
  if (!refresh) {  // E = R - delta B C, in place
    const int v4 = (s.M % 4 == 0) && ((reinterpret_cast<uintptr_t>(R) & 15) == 0);
    colpass_rw_launch(s, static_cast<const float*>(R), v4, C, Bq, BqD, Bsc, Hout, fpart, R, st);
  } else if (s.xbf16) {  // E = X - B C from the stored data
    colpass_rw_launch(s, static_cast<const __bf16*>(X), 0, C, Bq, Bq, Bsc, Hout, fpart, R, st);
  } else if (s.xtiled) {
    colpass_rw_launch(s, static_cast<const xtf32*>(X), 0, C, Bq, Bq, Bsc, Hout, fpart, R, st);
  } else {
    colpass_rw_launch(s, static_cast<const float*>(X), s.vec4, C, Bq, Bq, Bsc, Hout, fpart, R, st);
  }
  return hipGetLastError();
}

hipError_t colpass(const Shape& s, const void* X, const void* Cqv, const _Float16* Bq, const float* Bsc,
                   float* Hout, double* fpart, int with_h, hipStream_t st) {
  const f32x4* C = static_cast<const f32x4*>(Cqv);
  if (s.xbf16)
    colpass_launch(s, static_cast<const __bf16*>(X), C, Bq, Bsc, Hout, fpart, with_h, st);
  else if (s.xtiled)
    colpass_launch(s, static_cast<const xtf32*>(X), C, Bq, Bsc, Hout, fpart, with_h, st);
  else
    colpass_launch(s, static_cast<const float*>(X), C, Bq, Bsc, Hout, fpart, with_h, st);
  return hipGetLastError();
}

// ------------------------------------------------------------------ coordinate sweep
// One thread per column j.  With h = B^T e_j from the column pass and G = B^T B in LDS, the
// coordinates are updated in ascending order in float64:
//   c_kj := [c_kj + h_k / G_kk]_+,  then h_q -= G_qk (c_kj^new - c_kj^old) for q > k,
// (a true division, so that cancellations the closed form makes exact stay exact),
// which is eq. up:c with b_q^T e_j kept up to date through inner products; a coordinate
// with G_kk = 0 (zero column of B) is skipped.  The block's 256 columns of C (contiguous
// in memory) are staged through LDS so that global loads and stores are coalesced, and
// each updated column is repacked into Cq for the row pass and the next column pass.
// With CqD (the carried-residual form) the block also packs delta C = C' - C (float32
// difference of the stored values) into CqD's E-order units, for the row pass's update of
// the carried residual.
template <int KP, bool G_IN_LDS>
__device__ __forceinline__ void sweep_body(const float* __restrict__ Hin, float* __restrict__ C,
                                           f32x4* __restrict__ Cq, float* __restrict__ Csc, int64_t N, int K,
                                           const double* __restrict__ G, int64_t bid,
                                           f32x4* __restrict__ CqD = nullptr) {
  // G = B^T B (KP x KP, both halves stored) is the same for every lane.  The single-instance
  // kernel reads it directly: uniform addresses into memory the kernel does not write, which
  // the compiler serves with scalar loads, so the FMAs below take G from scalar registers.
  // The grouped kernels (whose pointers come from the descriptor table, after earlier work
  // items stored to memory) stage its strictly lower triangle in LDS instead and read the
  // diagonal from memory: without the diagonal, two blocks of the K > 32 class fit per CU.
  __shared__ double Gs[G_IN_LDS ? KP * (KP - 1) / 2 : 1];  // strictly lower triangle, rows r >= 1
  __shared__ int cs_own[G_IN_LDS ? 1 : 256];                // packing scratch (else in Gs, see below)
  extern __shared__ float Ct[];                             // the block's columns, stride K (256 * K floats)
  const int tid = threadIdx.x;
  if constexpr (G_IN_LDS) {
    for (int q = tid; q < KP * (KP - 1) / 2; q += 256) {
      int a, b;
      pair_of(q, a, b);  // a >= b; entry (a + 1, b) of G
      Gs[q] = G[(a + 1) * KP + b];
    }
  }
  // G[r][c] for r > c
  auto gl = [&](int r, int c) -> double {
    if constexpr (G_IN_LDS)
      return Gs[(r - 1) * r / 2 + c];
    else
      return G[c * KP + r];  // row c of the symmetric G: contiguous in r
  };

  const int64_t j0 = bid * 256;
  const int nv = (int)((N - j0) < 256 ? (N - j0) : 256);
  const int ne = nv * K;
  const int64_t col = j0 + tid;
  // the column's h, loaded while the block stages its columns of C
  float hf[KP];
  if (tid < nv) {
#pragma unroll
    for (int k = 0; k < KP; ++k) hf[k] = Hin[(int64_t)k * N + col];
  }
  block_copy(Ct, C + j0 * K, ne);
  __syncthreads();
  if (tid < nv) {
    double h[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) h[k] = (double)hf[k];
    float* cl = Ct + tid * K;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      if (k < K) {
        const double nk = G[k * KP + k];
        if (nk > 0.0) {
          const double cold = (double)cl[k];
          double cn = cold + h[k] / nk;
          cn = cn > 0.0 ? cn : 0.0;
          const double d = cn - cold;
          cl[k] = (float)cn;
#pragma unroll
          for (int q = k + 1; q < KP; ++q) h[q] -= gl(q, k) * d;
        }
      }
    }
  }
  __syncthreads();
  // the packing scratch reuses Gs once the sweep is done (the barrier above): with its own
  // 1 kB the grouped K > 32 kernel would no longer fit two blocks per CU
  int* cs = G_IN_LDS ? reinterpret_cast<int*>(Gs) : cs_own;
  if (CqD) {  // carried-residual form: C' packed, then Ct := C' - C packed into CqD
    pack_block<KP>(Cq, Csc, j0, nv, Ct, K, (N + 31) / 32, cs);
    __syncthreads();
    constexpr int G = 16;  // loads of the old values issued ahead, as in block_copy
    int e = tid;
    for (; e + (G - 1) * 256 < ne; e += G * 256) {
      float co[G];
#pragma unroll
      for (int u = 0; u < G; ++u) co[u] = C[j0 * K + e + u * 256];
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const float cn = Ct[e + u * 256];
        C[j0 * K + e + u * 256] = cn;
        Ct[e + u * 256] = cn - co[u];
      }
    }
    for (; e < ne; e += 256) {
      const float cn = Ct[e], co = C[j0 * K + e];
      C[j0 * K + e] = cn;
      Ct[e] = cn - co;
    }
    __syncthreads();
    pack_block<KP, true>(CqD, nullptr, j0, nv, Ct, K, (N + 31) / 32, cs);
    return;
  }
  block_copy(C + j0 * K, Ct, ne);
  pack_block<KP>(Cq, Csc, j0, nv, Ct, K, (N + 31) / 32, cs);
}

template <int KP>
__global__ __launch_bounds__(256) void k_sweep(const float* __restrict__ Hin, float* __restrict__ C,
                                               f32x4* __restrict__ Cq, float* __restrict__ Csc, int64_t N, int K,
                                               const double* __restrict__ G, f32x4* __restrict__ CqD) {
  sweep_body<KP, false>(Hin, C, Cq, Csc, N, K, G, blockIdx.x, CqD);
}

// E order of 256 columns of C (block bid), and their contribution to the row maxima.
template <int KP>
__device__ __forceinline__ void packc_body(const float* __restrict__ C, f32x4* __restrict__ Cq,
                                           float* __restrict__ Csc, int64_t N, int K, int64_t bid) {
  extern __shared__ float Ct[];  // 256 * K floats
  __shared__ int cs[256];
  const int64_t j0 = bid * 256;
  const int nv = (int)((N - j0) < 256 ? (N - j0) : 256);
  const int ne = nv * K;
  block_copy(Ct, C + j0 * K, ne);
  __syncthreads();
  pack_block<KP>(Cq, Csc, j0, nv, Ct, K, (N + 31) / 32, cs);
}

template <int KP>
__global__ __launch_bounds__(256) void k_packc(const float* __restrict__ C, f32x4* __restrict__ Cq,
                                               float* __restrict__ Csc, int64_t N, int K) {
  packc_body<KP>(C, Cq, Csc, N, K, blockIdx.x);
}

template <int KP>
__global__ __launch_bounds__(256) void k_packw(const float* __restrict__ C, f32x4* __restrict__ Cq,
                                               float* __restrict__ Csc, int64_t N, int K) {
  packw_body<KP>(C, Cq, Csc, N, K, blockIdx.x);
}

static hipError_t packw(const Shape& s, const float* C, f32x4* Cq, float* Csc, hipStream_t st) {
  const unsigned g = (unsigned)((s.N + 255) / 256);
  if (s.KP == 32)
    k_packw<32><<<g, 256, 0, st>>>(C, Cq, Csc, s.N, s.K);
  else
    k_packw<64><<<g, 256, 0, st>>>(C, Cq, Csc, s.N, s.K);
  return hipGetLastError();
}

hipError_t sweep(const Shape& s, const float* Hin, float* C, void* Cq, float* Csc, const double* G,
                 hipStream_t st, void* CqD) {
  const unsigned g = (unsigned)((s.N + 255) / 256);
  f32x4* q = static_cast<f32x4*>(Cq);
  f32x4* qd = static_cast<f32x4*>(CqD);
  k_zero_f32<<<1, 64, 0, st>>>(Csc, s.KP);
  if (s.KP == 32)
    k_sweep<32><<<g, 256, 256 * s.K * sizeof(float), st>>>(Hin, C, q, Csc, s.N, s.K, G, qd);
  else
    k_sweep<64><<<g, 256, 256 * s.K * sizeof(float), st>>>(Hin, C, q, Csc, s.N, s.K, G, qd);
  return packw(s, C, q, Csc, st);
}

hipError_t packc(const Shape& s, const float* C, void* Cq, float* Csc, hipStream_t st) {
  const unsigned g = (unsigned)((s.N + 255) / 256);
  f32x4* q = static_cast<f32x4*>(Cq);
  k_zero_f32<<<1, 64, 0, st>>>(Csc, s.KP);
  if (s.KP == 32)
    k_packc<32><<<g, 256, 256 * s.K * sizeof(float), st>>>(C, q, Csc, s.N, s.K);
  else
    k_packc<64><<<g, 256, 256 * s.K * sizeof(float), st>>>(C, q, Csc, s.N, s.K);
  return packw(s, C, q, Csc, st);
}

// ------------------------------------------------------------------ V = tril(C C^T)
// V = C C^T from the packed W-order units of C: a W unit holds, for one coordinate kk,
// eight columns of a tile, which is both the A fragment (rows kk, reduction over columns)
// and the B fragment (reduction over columns, columns kk') of the product.  Each block
// takes a contiguous run of tiles; wave w takes every fourth tile of the run and forms the
// lower 32x32 blocks (b1 >= b2) of the tile's contribution with scaled fp16 MFMAs (float32
// within the tile, in units of 2^(w_a + w_b)), adding them to float64 accumulators.  The
// four waves' partials are then unscaled (exactly), added in wave order and written as
// tril pairs.
constexpr int kVBlocks = 256;

template <int KP>
__device__ __forceinline__ void vgram_body(const f32x4* __restrict__ Cq, const float* __restrict__ Csc,
                                           int64_t ntiles, double* __restrict__ Vpart, int64_t bid, int64_t nblk) {
  constexpr int NB = KP / 32;
  constexpr int UE = CqL<KP>::E;  // E-order units and scales of a packed C tile
  constexpr int UT = CqL<KP>::T;
  constexpr int NBL = NB * (NB + 1) / 2;  // lower blocks (b1 >= b2)
  constexpr int NP = KP * (KP + 1) / 2;
  __shared__ double Vs[4][NP];
  // the wave index is uniform: from a scalar register, so that wave-based addresses stay scalar
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, half = l >> 5,
            lc = l & 31;
  const int64_t per = (ntiles + nblk - 1) / nblk;
  const int64_t t0 = bid * per;
  const int64_t t1 = (t0 + per < ntiles) ? t0 + per : ntiles;
  double acc[NBL][16];
#pragma unroll
  for (int k = 0; k < NBL; ++k)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[k][i] = 0.0;
  for (int64_t T = t0 + wave; T < t1; T += 4) {
    const f32x4* wu = Cq + T * UT + UE + l;
    f32x16 v[NBL];
#pragma unroll
    for (int k = 0; k < NBL; ++k)
#pragma unroll
      for (int i = 0; i < 16; ++i) v[k][i] = 0.0f;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      f16x8 w[NB][2];
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int p = 0; p < 2; ++p) w[b][p] = as_f16x8(wu[((b * 2 + q) * 2 + p) * 64]);
      int k = 0;
#pragma unroll
      for (int b1 = 0; b1 < NB; ++b1)
#pragma unroll
        for (int b2 = 0; b2 <= b1; ++b2, ++k) v[k] = mfma_x3(w[b1], w[b2], v[k]);
    }
#pragma unroll
    for (int k = 0; k < NBL; ++k)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[k][i] += (double)v[k][i];
  }
  for (int q = l; q < NP; q += 64) Vs[wave][q] = 0.0;
  __syncthreads();
  {
    const float* inv = Csc + KP;  // 2^-w_kk
    int k = 0;
#pragma unroll
    for (int b1 = 0; b1 < NB; ++b1)
#pragma unroll
      for (int b2 = 0; b2 <= b1; ++b2, ++k)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int a = 32 * b1 + row32(i, half), b = 32 * b2 + lc;
          if (a >= b) Vs[wave][a * (a + 1) / 2 + b] = acc[k][i] * (double)inv[a] * (double)inv[b];
        }
  }
  __syncthreads();
  for (int q = tid; q < NP; q += 256)
    Vpart[bid * NP + q] = ((Vs[0][q] + Vs[1][q]) + Vs[2][q]) + Vs[3][q];
}

template <int KP>
__global__ __launch_bounds__(256) void k_vgram(const f32x4* __restrict__ Cq, const float* __restrict__ Csc,
                                               int64_t ntiles, double* __restrict__ Vpart) {
  vgram_body<KP>(Cq, Csc, ntiles, Vpart, blockIdx.x, gridDim.x);
}

int64_t vgram_blocks(const Shape& s) {
  const int64_t t = n_tiles32(s);
  return t < kVBlocks ? t : kVBlocks;
}

hipError_t vgram(const Shape& s, const void* Cq, const float* Csc, double* Vpart, hipStream_t st) {
  const unsigned g = (unsigned)vgram_blocks(s);
  const f32x4* q = static_cast<const f32x4*>(Cq);
  if (s.KP == 32)
    k_vgram<32><<<g, 256, 0, st>>>(q, Csc, n_tiles32(s), Vpart);
  else
    k_vgram<64><<<g, 256, 0, st>>>(q, Csc, n_tiles32(s), Vpart);
  return hipGetLastError();
}

// ------------------------------------------------------------------ row pass
// Block = 4 waves; wave w owns the 32-row chunk c = 4*sg + w of slab group sg and column
// range r.  Per 32-column tile T of the range (transposed tiles, rows = columns of X):
//   P    = (C[:, tile] 2^t)^T (-B[chunk, :] 2^s)^T  (scaled fp16 steps, as in the column pass)
//   acc  = X[chunk, tile]^T + P 2^-(t_j + s_m)       -> E'^T with E' = X - B C'
//   WT  += (C[:, tile] 2^w) (acc 2^v)                -> (E' C'^T)^T for this chunk, scaled
// where w is the packed per-row scale of C' and v, per row of E' (per lane), the running
// scale of the column pass's H: chosen per tile from the tile's largest |E'| in the row and
// never raised, the running WT being rescaled exactly when it drops.  The packed C' tile
// (both operand orders, already split and scaled) is copied into LDS for the next tile
// (double buffer shared by the four waves; straight from global memory into LDS, with no
// staging registers) and X of the next tile is prefetched into registers.
// Blocks map to (range, slab group) so that all slab groups of a range run on one XCD
// (blocks are dealt to the eight XCDs round-robin): the range's C' tiles are then fetched
// into a single L2.
//
// RW (the carried-residual form): X is the column-major float32 residual R = X - B C of
// the column pass, the E-order operand of each tile comes from CqE (delta C, stride
// CqL<KP>::E units per tile) while the W-order operand comes from Cq, so that
// E' = R - B delta C, and E' is stored back into R in place.
template <int KP, typename XT, bool RW = false>
__device__ __forceinline__ void rowpass_body(const XT* __restrict__ X, int64_t M, int64_t N, int K,
                                             const f32x4* __restrict__ Cq, const float* __restrict__ Csc,
                                             const _Float16* __restrict__ Bq,
                                             float* __restrict__ Wpart, int64_t Mpad, int64_t nchunks,
                                             const int64_t* __restrict__ tb, int R, int nsg, int64_t bid,
                                             const f32x4* __restrict__ CqE = nullptr, float* Rout = nullptr) {
  constexpr int NB = KP / 32;
  constexpr int KS = KP / 16;
  constexpr int UE0 = CqL<KP>::E0;     // 16-byte units of the E'^T A operand per tile
  constexpr int UE = CqL<KP>::E;       // ... followed by the tile's inverse column scales
  constexpr int UT = CqL<KP>::T;       // then the W A operand
  constexpr int NV = (UT + 255) / 256;
  constexpr int64_t UC = BqL<KP>::C;   // units per packed B chunk
  constexpr int UBS = BqL<KP>::S;      // the chunk's 32 row scales
  __shared__ f32x4 sc[2][UT];
  const int id = (int)bid, xcd = id & 7, local = id >> 3;
  const int r = xcd + 8 * (local / nsg), sg = local % nsg;
  if (r >= R) return;  // whole block
  // the wave index is uniform: from a scalar register, so that wave-based addresses stay scalar
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, half = l >> 5,
            lc = l & 31;
  const int64_t c = (int64_t)sg * 4 + wave;
  const bool active = c < nchunks;  // inactive waves still take part in staging and barriers
  const int64_t tlo = tb[r], thi = tb[r + 1];
  const int64_t hi = (thi * 32 < N) ? thi * 32 : N;  // column end of the range
  const int64_t m0 = (active ? c : 0) * 32, mrow = m0 + lc;
  const bool rowok = active && mrow < M;

  f16x8 bP[KS][2];  // pieces of -B[m0 + l%32][16s + 8*half + t] 2^s_m
  float bs;         // 2^-s_m of this lane's row
  {
    const f32x4* pe = reinterpret_cast<const f32x4*>(Bq) + (active ? c : 0) * UC;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int p = 0; p < 2; ++p) bP[s][p] = as_f16x8(pe[(s * 2 + p) * 64 + l]);
    bs = fabsf(reinterpret_cast<const float*>(pe + UBS)[lc]);  // row 0's may carry the uniform flag
  }
  f32x16 WT[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int i = 0; i < 16; ++i) WT[b][i] = 0.0f;
  int vcur = 126;  // current scale exponent of this row's E' operand (never raised)

  // tile T's packed C units straight from global memory into LDS buffer buf (no staging
  // registers): lane l of wave w writes unit w*64 + 256 v + l, the unit it loads
  auto cdma = [&](int64_t T, int buf) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int u = tid + 256 * v;
      if (u < UT) {
        const f32x4* src = Cq + T * UT + u;
        if constexpr (RW)
          if (u < UE) src = CqE + T * UE + u;
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                         (__attribute__((address_space(3))) void*)&sc[buf][wave * 64 + 256 * v], 16, 0,
                                         0);
      }
    }
  };
  const uint32_t loff = (uint32_t)(4 * half * M + mrow);  // lane offset within a tile
  const bool rowsfull = active && m0 + 32 <= M;            // wave-uniform
  auto xload = [&](int64_t T) {
    f32x16 v;
    if constexpr (x_is_tiled<XT>::value) {  // tiled copy XR
      return ld_tile(X + ((active ? c : 0) * ((N + 31) / 32) + T) * 1024, l);
    } else {  // column-major float32 X
      const int64_t j0 = T * 32;
      const float* xt = X + j0 * M;  // wave-uniform
      if (rowsfull && j0 + 32 <= hi) {  // wave-uniform
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = xt[(int64_t)(8 * (i >> 2) + (i & 3)) * M + loff];
      } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int64_t j = j0 + row32(i, half);
          v[i] = (rowok && j < hi) ? X[j * M + mrow] : 0.0f;
        }
      }
      return v;
    }
  };

  // One tile: compute tile T from the X tile in xc (loaded one tile earlier) and the
  // staged C' operands in LDS buffer buf; meanwhile stage tile T+1 and load its X tile
  // into xn.
  auto step = [&](int64_t T, int buf, const f32x16& xc, f32x16& xn) {
    const int64_t Tn = T + 1 < thi ? T + 1 : T;
    cdma(Tn, buf ^ 1);
    xn = xload(Tn);
    if (active) {
      f32x16 acc;  // E' of the tile (the X tile in xc stays as loaded)
      {
        const f32x4* ue = &sc[buf][0] + l;
        f16x8 a[2], an[2];
        f32x16 P;
#pragma unroll
        for (int i = 0; i < 16; ++i) P[i] = 0.0f;
#pragma unroll
        for (int p = 0; p < 2; ++p) a[p] = as_f16x8(ue[p * 64]);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          if (s + 1 < KS) {
#pragma unroll
            for (int p = 0; p < 2; ++p) an[p] = as_f16x8(ue[((s + 1) * 2 + p) * 64]);
          }
          P = mfma_x3(a, bP[s], P);
          if (s + 1 < KS) {
#pragma unroll
            for (int p = 0; p < 2; ++p) a[p] = an[p];
          }
        }
        // rows row32(4q + e, half) = 8q + 4 half + e of the tile: inverse scales in unit 2q + half.
        // A negative first scale flags a tile whose columns share one scale (the C packing):
        // one multiplier for the whole tile.
        const f32x4* ts = &sc[buf][UE0];
        const float t0 =
            __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, ts[0][0])));
        if (t0 < 0.0f) {
          const float mu = -t0 * bs;
#pragma unroll
          for (int i = 0; i < 16; ++i) acc[i] = fmaf(P[i], mu, xc[i]);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const f32x4 t4 = ts[2 * q + half];
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[4 * q + e] = fmaf(P[4 * q + e], t4[e] * bs, xc[4 * q + e]);
          }
        }
      }
      if constexpr (RW) {  // E' back into the residual, where it was read
        const int64_t j0 = T * 32;
        float* rt = Rout + j0 * M;
        if (rowsfull && j0 + 32 <= hi) {
#pragma unroll
          for (int i = 0; i < 16; ++i) rt[(int64_t)(8 * (i >> 2) + (i & 3)) * M + loff] = acc[i];
        } else {
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int64_t j = j0 + row32(i, half);
            if (rowok && j < hi) Rout[j * M + mrow] = acc[i];
          }
        }
      }
      // scale of this tile's E' operand: the largest |E'| of the row over the tile (the
      // lane and its partner l ^ 32 hold the row's 32 columns)
      float em = 0.0f;
#pragma unroll
      for (int i = 0; i < 16; ++i) em = fmaxf(em, fabsf(acc[i]));
      em = fmaxf(em, __shfl_xor(em, 32, 64));
      int v = scale_exp(em);
      v = (em > 0.0f && v < vcur) ? v : vcur;
      if (__ballot(v != vcur)) {  // wave-uniform: rescale only when some row's scale drops
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int i = 0; i < 16; ++i) WT[b][i] = ldexpf(WT[b][i], v - vcur);
        vcur = v;
      }
      const f32x4* uw = &sc[buf][UE] + l;
      f16x8 w[2], wn[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) w[p] = as_f16x8(uw[p * 64]);
      f16x8 eP[2][2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        float y[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) y[t] = ldexpf(acc[8 * q + t], v);
        const Split2 sp = split2(y);
#pragma unroll
        for (int p = 0; p < 2; ++p) eP[q][p] = sp.p[p];
      }
#pragma unroll
      for (int gg = 0; gg < NB * 2; ++gg) {  // accumulators alternate, as in the column pass
        if (gg + 1 < NB * 2) {
          const int un = (((gg + 1) % NB) * 2 + (gg + 1) / NB) * 2;
#pragma unroll
          for (int p = 0; p < 2; ++p) wn[p] = as_f16x8(uw[(un + p) * 64]);
        }
        WT[gg % NB] = mfma_x3(w, eP[gg / NB], WT[gg % NB]);
        if (gg + 1 < NB * 2) {
#pragma unroll
          for (int p = 0; p < 2; ++p) w[p] = wn[p];
        }
      }
    }
    __syncthreads();
  };

  if (tlo < thi) {
    f32x16 x0 = xload(tlo);
    cdma(tlo, 0);
    __syncthreads();
    f32x16 x1;
    for (int64_t T = tlo; T < thi; T += 2) {
      step(T, 0, x0, x1);
      if (T + 1 < thi) step(T + 1, 1, x1, x0);
    }
  }
  if (active) {
    float* wp = Wpart + (int64_t)r * KP * Mpad;
    const float* inv = Csc + KP;  // 2^-w_kk
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int kk = 32 * b + row32(i, half);
        wp[(int64_t)kk * Mpad + m0 + lc] = ldexpf(WT[b][i], -vcur) * inv[kk];
      }
  }
}

template <int KP, typename XT>
__global__ __launch_bounds__(256, 2) void k_rowpass(const XT* __restrict__ X, int64_t M, int64_t N, int K,
                                                    const f32x4* __restrict__ Cq, const float* __restrict__ Csc,
                                                    const _Float16* __restrict__ Bq, float* __restrict__ Wpart,
                                                    int64_t Mpad, int64_t nchunks, const int64_t* __restrict__ tb,
                                                    int R, int nsg) {
  rowpass_body<KP, XT>(X, M, N, K, Cq, Csc, Bq, Wpart, Mpad, nchunks, tb, R, nsg, blockIdx.x);
}

template <int KP>
__global__ __launch_bounds__(256, 2) void k_rowpass_rw(float* Rr, int64_t M, int64_t N, int K,
                                                       const f32x4* __restrict__ Cq, const f32x4* __restrict__ CqD,
                                                       const float* __restrict__ Csc,
                                                       const _Float16* __restrict__ Bq, float* __restrict__ Wpart,
                                                       int64_t Mpad, int64_t nchunks, const int64_t* __restrict__ tb,
                                                       int R, int nsg) {
  rowpass_body<KP, float, true>(Rr, M, N, K, Cq, Csc, Bq, Wpart, Mpad, nchunks, tb, R, nsg, blockIdx.x, CqD, Rr);
}

hipError_t rowpass_carry(const Shape& s, float* Rr, const void* Cqv, const void* CqDv, const float* Csc,
                         const _Float16* Bq, float* Wpart, const int64_t* tb, int R, hipStream_t st) {
  const f32x4* Cq = static_cast<const f32x4*>(Cqv);
  const f32x4* CqD = static_cast<const f32x4*>(CqDv);
  const int nsg = (int)((s.nchunks + 3) / 4);
  const int R8 = (R + 7) / 8 * 8;
  const unsigned g = (unsigned)((int64_t)nsg * R8);
  if (s.KP == 32)
    k_rowpass_rw<32><<<g, 256, 0, st>>>(Rr, s.M, s.N, s.K, Cq, CqD, Csc, Bq, Wpart, s.Mpad, s.nchunks, tb, R, nsg);
  else
    k_rowpass_rw<64><<<g, 256, 0, st>>>(Rr, s.M, s.N, s.K, Cq, CqD, Csc, Bq, Wpart, s.Mpad, s.nchunks, tb, R, nsg);
  return hipGetLastError();
}

template <typename XT>
static void rowpass_launch(const Shape& s, const XT* X, const f32x4* Cq, const float* Csc, const _Float16* Bq,
                           float* Wpart, const int64_t* tb, int R, hipStream_t st) {
  const int nsg = (int)((s.nchunks + 3) / 4);
  const int R8 = (R + 7) / 8 * 8;
  const unsigned g = (unsigned)((int64_t)nsg * R8);
  if (s.KP == 32)
    k_rowpass<32, XT><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, Cq, Csc, Bq, Wpart, s.Mpad, s.nchunks, tb, R, nsg);
  else
    k_rowpass<64, XT><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, Cq, Csc, Bq, Wpart, s.Mpad, s.nchunks, tb, R, nsg);
}

hipError_t rowpass(const Shape& s, const void* X, const void* Cqv, const float* Csc, const _Float16* Bq,
                   float* Wpart, const int64_t* tb, int R, hipStream_t st) {
  const f32x4* Cq = static_cast<const f32x4*>(Cqv);
  if (s.xbf16)
    rowpass_launch(s, static_cast<const __bf16*>(X), Cq, Csc, Bq, Wpart, tb, R, st);
  else if (s.xtiled)
    rowpass_launch(s, static_cast<const xtf32*>(X), Cq, Csc, Bq, Wpart, tb, R, st);
  else
    rowpass_launch(s, static_cast<const float*>(X), Cq, Csc, Bq, Wpart, tb, R, st);
  return hipGetLastError();
}

// ------------------------------------------------------------------ reductions
// The fixed-order sums below issue the loads of their terms in groups ahead of the
// additions, which still take the terms one at a time in order: a thread then waits for one
// memory round trip per group instead of one per term (a plain loop over a run-time count
// is compiled as load, wait, add).

// W[kk][m] = sum_r Wpart[r][kk][m], r ascending, float64 (blocks of 256 entries).
__device__ __forceinline__ void reduce_w_body(const float* __restrict__ Wpart, int R, int64_t n,
                                              double* __restrict__ W, int64_t bid) {
  const int64_t i = bid * 256 + threadIdx.x;
  if (i >= n) return;
  constexpr int G = 16;
  const float* wp = Wpart + i;
  double s = 0.0;
  int r = 0;
  for (; r + G <= R; r += G) {
    float v[G];
#pragma unroll
    for (int u = 0; u < G; ++u) v[u] = wp[(int64_t)(r + u) * n];
#pragma unroll
    for (int u = 0; u < G; ++u) s += (double)v[u];
  }
  for (; r < R; ++r) s += (double)wp[(int64_t)r * n];
  W[i] = s;
}

__global__ __launch_bounds__(256) void k_reduce_w(const float* __restrict__ Wpart, int R, int64_t n,
                                                  double* __restrict__ W) {
  reduce_w_body(Wpart, R, n, W, blockIdx.x);
}

hipError_t reduce_w(const Shape& s, const float* Wpart, int R, double* W, hipStream_t st) {
  const int64_t n = (int64_t)s.KP * s.Mpad;
  k_reduce_w<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(Wpart, R, n, W);
  return hipGetLastError();
}

// full[i] = sum_p part[p][i] over KP*KP entries, p ascending.
__global__ void k_reduce_full(const double* __restrict__ part, int64_t P, int n, double* __restrict__ full) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  double s = 0.0;
  for (int64_t p = 0; p < P; ++p) s += part[p * n + q];
  full[q] = s;
}

hipError_t reduce_full(const double* part, int64_t P, int KP, double* full, hipStream_t st) {
  const int n = KP * KP;
  k_reduce_full<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(part, P, n, full);
  return hipGetLastError();
}

// full[a][b] = full[b][a] = sum_p part[p][pair(a,b)] in a fixed order.  A block of 256
// threads takes kSymPairs consecutive pairs with 32 threads each: thread (t, qi) =
// (tid / 8, tid % 8) adds the partials p = t, t + 32, t + 64, ... in turn, then the 32
// sums of a pair are combined by a fixed tree (xor shuffles within each wave, then the
// four waves in order).  Every thread reaches the barrier.
constexpr int kSymPairs = 8;
__device__ __forceinline__ void reduce_sym_body(const double* __restrict__ part, int64_t P, int KP,
                                                double* __restrict__ full, int64_t bid) {
  __shared__ double ws[4][kSymPairs];
  const int NP = KP * (KP + 1) / 2;
  const int tid = threadIdx.x, qi = tid & (kSymPairs - 1), t = tid / kSymPairs, wave = tid >> 6;
  const int q = (int)bid * kSymPairs + qi;
  double s = 0.0;
  if (q < NP) {
    constexpr int64_t D = 256 / kSymPairs;  // stride between a thread's partials
    constexpr int G = 8;
    int64_t p = t;
    for (; p + (G - 1) * D < P; p += G * D) {
      double v[G];
#pragma unroll
      for (int u = 0; u < G; ++u) v[u] = part[(p + u * D) * NP + q];
#pragma unroll
      for (int u = 0; u < G; ++u) s += v[u];
    }
    for (; p < P; p += D) s += part[p * NP + q];
  }
  // lanes qi + 8 t' of a wave (t' = t % 8) hold the same pair
  s += __shfl_xor(s, 8, 64);
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  if ((tid & 63) < kSymPairs) ws[wave][qi] = s;
  __syncthreads();
  if (tid < kSymPairs && q < NP) {
    const double v = (ws[0][qi] + ws[1][qi]) + (ws[2][qi] + ws[3][qi]);
    int a, b;
    pair_of(q, a, b);
    full[a * KP + b] = v;
    full[b * KP + a] = v;
  }
}

__global__ __launch_bounds__(256) void k_reduce_sym(const double* __restrict__ part, int64_t P, int KP,
                                                    double* __restrict__ full) {
  reduce_sym_body(part, P, KP, full, blockIdx.x);
}

hipError_t reduce_sym(const double* part, int64_t P, int KP, double* full, hipStream_t st) {
  const int NP = KP * (KP + 1) / 2;
  k_reduce_sym<<<(unsigned)((NP + kSymPairs - 1) / kSymPairs), 256, 0, st>>>(part, P, KP, full);
  return hipGetLastError();
}

// scale * sum_p part[p]: each thread sums a strided subset in order, then a fixed tree over
// the block; the result is returned to every thread.
__device__ __forceinline__ double reduce_f_body(const double* __restrict__ part, int64_t P, double scale) {
  __shared__ double s[256];
  constexpr int G = 8;
  double a = 0.0;
  int64_t p = threadIdx.x;
  for (; p + (G - 1) * 256 < P; p += G * 256) {
    double v[G];
#pragma unroll
    for (int u = 0; u < G; ++u) v[u] = part[p + u * 256];
#pragma unroll
    for (int u = 0; u < G; ++u) a += v[u];
  }
  for (; p < P; p += 256) a += part[p];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  const double r = scale * s[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_reduce_f(const double* __restrict__ part, int64_t P, double* out,
                                                  double scale) {
  const double r = reduce_f_body(part, P, scale);
  if (threadIdx.x == 0) *out = r;
}

hipError_t reduce_f(const double* part, int64_t P, double* out, double scale, hipStream_t st) {
  k_reduce_f<<<1, 256, 0, st>>>(part, P, out, scale);
  return hipGetLastError();
}

// The objective of an iteration into the history ring at the device iteration counter,
// which then advances: no host value is baked into the launch, so a captured iteration
// can be replayed.
__global__ __launch_bounds__(256) void k_reduce_f_hist(const double* __restrict__ part, int64_t P,
                                                       double* __restrict__ fhist, int64_t cap,
                                                       int64_t* __restrict__ tdev, double scale) {
  const double r = reduce_f_body(part, P, scale);
  if (threadIdx.x == 0) {
    const int64_t t = *tdev;
    fhist[t % cap] = r;
    *tdev = t + 1;
  }
}

hipError_t reduce_f_hist(const double* part, int64_t P, double* fhist, int64_t cap, int64_t* tdev, double scale,
                         hipStream_t st) {
  k_reduce_f_hist<<<1, 256, 0, st>>>(part, P, fhist, cap, tdev, scale);
  return hipGetLastError();
}

__global__ void k_set_i64(int64_t* p, int64_t v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}

hipError_t set_i64(int64_t* p, int64_t v, hipStream_t st) {
  k_set_i64<<<1, 64, 0, st>>>(p, v);
  return hipGetLastError();
}

// ------------------------------------------------------------------ batched form
// Grouped persistent kernels: block b takes items b, b + grid, b + 2 grid, ... of the
// stage's concatenated item list, finds the owning instance by binary search over the
// item prefix, and runs the stage's device code for that instance and local block index.
// The row pass's items of each instance start at a multiple of 8 and every grid is a
// multiple of 8, so an item's XCD (block index mod 8) is the same as in the instance's
// own launch.
__device__ __forceinline__ int ginst_find(const GTable* __restrict__ g, int st, int64_t w) {
  int lo = 0, hi = g->n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g->begin[st][mid] <= w)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

#define DID_GROUP_LOOP(ST)                                                     \
  const int64_t total_ = g->total[ST];                                        \
  for (int64_t w_ = blockIdx.x; w_ < total_; w_ += gridDim.x) {               \
    const int i_ = ginst_find(g, ST, w_);                                      \
    const GInst& d = g->inst[i_];                                              \
    const int64_t bid = w_ - g->begin[ST][i_];

#define DID_GROUP_END \
  __syncthreads();    \
  }

template <int KP, typename XT, int WPB>
__global__ __launch_bounds__(64 * WPB, 8 / WPB) void kg_colpass(const GTable* __restrict__ g) {
  DID_GROUP_LOOP(GS_COL)
  colpass_body<KP, true, XT, false, WPB>(static_cast<const XT*>(d.X), d.M, d.N, d.K, static_cast<const f32x4*>(d.Cq),
                                         d.Bq, d.Bsc, d.H, d.fpart, d.nchunks, d.vec4, bid);
  DID_GROUP_END
}

__global__ __launch_bounds__(256) void kg_reduce_f(const GTable* __restrict__ g) {
  DID_GROUP_LOOP(GS_REDF)
  (void)bid;
  // the row maxima of C start from zero for the sweep that follows
  if ((int)threadIdx.x < d.K) d.Csc[threadIdx.x] = 0.0f;
  const double r = reduce_f_body(d.fpart, d.colblocks, 0.5);
  if (threadIdx.x == 0) {
    const int64_t t = *d.tdev;
    d.fhist[t % d.hist_cap] = r;
    *d.fcur = r;
  }
  DID_GROUP_END
}

template <int KP>
__global__ __launch_bounds__(256) void kg_sweep(const GTable* __restrict__ g) {
  DID_GROUP_LOOP(GS_SWEEP)
  sweep_body<KP, true>(d.H, d.C, static_cast<f32x4*>(d.Cq), d.Csc, d.N, d.K, d.G, bid);
  DID_GROUP_END
}

template <int KP>
__global__ __launch_bounds__(256) void kg_packw(const GTable* __restrict__ g) {
  DID_GROUP_LOOP(GS_PACKW)
  packw_body<KP>(d.C, static_cast<f32x4*>(d.Cq), d.Csc, d.N, d.K, bid);
  DID_GROUP_END
}

template <int KP>
__global__ __launch_bounds__(256) void kg_vgram(const GTable* __restrict__ g) {
  DID_GROUP_LOOP(GS_VGRAM)
  vgram_body<KP>(static_cast<const f32x4*>(d.Cq), d.Csc, (d.N + 31) / 32, d.Vpart, bid, d.vblocks);
  DID_GROUP_END
}

template <int KP>
__global__ __launch_bounds__(256) void kg_reduce_v(const GTable* __restrict__ g) {
  DID_GROUP_LOOP(GS_REDV)
  reduce_sym_body(d.Vpart, d.vblocks, KP, d.V, bid);
  DID_GROUP_END
}

template <int KP, typename XT>
__global__ __launch_bounds__(256, 2) void kg_rowpass(const GTable* __restrict__ g) {
  DID_GROUP_LOOP(GS_ROW)
  rowpass_body<KP, XT>(static_cast<const XT*>(d.XR), d.M, d.N, d.K, static_cast<const f32x4*>(d.Cq), d.Csc, d.Bq,
                       d.Wpart,
                       d.Mpad, d.nchunks, d.tb, d.R, d.nsg, bid);
  DID_GROUP_END
}

template <int KP>
__global__ __launch_bounds__(256) void kg_reduce_w(const GTable* __restrict__ g) {
  DID_GROUP_LOOP(GS_REDW)
  // the column maxima of B start from zero for the B update that follows
  if (bid == 0 && threadIdx.x < KP) d.Bsc[threadIdx.x] = 0.0f;
  reduce_w_body(d.Wpart, d.R, (int64_t)KP * d.Mpad, d.W, bid);
  DID_GROUP_END
}

template <int KP>
__global__ __launch_bounds__(kBupThreads) void kg_bupdate(const GTable* __restrict__ g) {
  DID_GROUP_LOOP(GS_BUP)
  bupdate_body<KP, false, false>(d.B, d.M, d.K, d.W, d.Mpad, d.V, d.Bq, d.Bsc, d.Gpart, 1, bid);
  DID_GROUP_END
}

template <int KP>
__global__ __launch_bounds__(256) void kg_reduce_g(const GTable* __restrict__ g) {
  DID_GROUP_LOOP(GS_REDG)
  // the G reduction, then the H-order packing of B: both need only the B update
  const int64_t ng = (KP * (KP + 1) / 2 + kSymPairs - 1) / kSymPairs;
  if (bid < ng)
    reduce_sym_body(d.Gpart, d.bupblocks, KP, d.G, bid);
  else
    packh_body<KP>(d.B, d.M, d.K, d.nchunks, d.Bq, d.Bsc, bid - ng);
  DID_GROUP_END
}

__global__ __launch_bounds__(64) void kg_advance(const GTable* __restrict__ g) {
  DID_GROUP_LOOP(GS_ADV)
  (void)bid;
  if (threadIdx.x == 0) *d.tdev = *d.tdev + 1;
  DID_GROUP_END
}

#undef DID_GROUP_LOOP
#undef DID_GROUP_END

void ginst_items(const Shape& s, int R, int64_t items[GS_N]) {
  const int64_t np = n_pairs(s.KP);
  const int64_t nsg = (s.nchunks + 3) / 4;
  const int64_t R8 = ((int64_t)R + 7) / 8 * 8;
  items[GS_COL] = colpass_blocks(s);
  items[GS_REDF] = 1;
  items[GS_SWEEP] = (s.N + 255) / 256;
  items[GS_PACKW] = (s.N + 255) / 256;
  items[GS_VGRAM] = vgram_blocks(s);
  items[GS_REDV] = (np + kSymPairs - 1) / kSymPairs;
  items[GS_ROW] = nsg * R8;
  items[GS_REDW] = ((int64_t)s.KP * s.Mpad + 255) / 256;
  items[GS_BUP] = bupdate_blocks(s);
  items[GS_REDG] = (np + kSymPairs - 1) / kSymPairs + bupdate_blocks(s);
  items[GS_ADV] = 1;
}

template <int KP, typename XT, int WPB>
static hipError_t group_grids_t(int64_t grids[GS_N]) {
  int dev = 0, cus = 0;
  hipError_t e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  auto occ = [&](const void* fn, int threads, size_t lds, int64_t* out) {
    int per = 0;
    hipError_t r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, lds);
    // multiple of 8 (one block per XCD round), at least one round
    *out = ((int64_t)std::max(per, 1) * cus + 7) / 8 * 8;
    return r;
  };
  if ((e = occ((const void*)kg_colpass<KP, XT, WPB>, 64 * WPB, 0, &grids[GS_COL])) != hipSuccess) return e;
  if ((e = occ((const void*)kg_reduce_f, 256, 0, &grids[GS_REDF])) != hipSuccess) return e;
  if ((e = occ((const void*)kg_sweep<KP>, 256, 256 * KP * sizeof(float), &grids[GS_SWEEP])) != hipSuccess) return e;
  if ((e = occ((const void*)kg_packw<KP>, 256, 0, &grids[GS_PACKW])) != hipSuccess) return e;
  if ((e = occ((const void*)kg_vgram<KP>, 256, 0, &grids[GS_VGRAM])) != hipSuccess) return e;
  if ((e = occ((const void*)kg_reduce_v<KP>, 256, 0, &grids[GS_REDV])) != hipSuccess) return e;
  if ((e = occ((const void*)kg_rowpass<KP, XT>, 256, 0, &grids[GS_ROW])) != hipSuccess) return e;
  if ((e = occ((const void*)kg_reduce_w<KP>, 256, 0, &grids[GS_REDW])) != hipSuccess) return e;
  if ((e = occ((const void*)kg_bupdate<KP>, kBupThreads, 0, &grids[GS_BUP])) != hipSuccess) return e;
  if ((e = occ((const void*)kg_reduce_g<KP>, 256, 0, &grids[GS_REDG])) != hipSuccess) return e;
  if ((e = occ((const void*)kg_advance, 64, 0, &grids[GS_ADV])) != hipSuccess) return e;
  return hipSuccess;
}

template <int KP, typename XT>
static hipError_t group_grids_k(int cwpb, int64_t grids[GS_N]) {
  return cwpb == 8 ? group_grids_t<KP, XT, 8>(grids) : group_grids_t<KP, XT, 4>(grids);
}

hipError_t group_grids(int KP, int xkind, int cwpb, int64_t grids[GS_N]) {
  if (KP == 32) {
    if (xkind == XK_BF16) return group_grids_k<32, __bf16>(cwpb, grids);
    if (xkind == XK_F32_TILED) return group_grids_k<32, xtf32>(cwpb, grids);
    return group_grids_k<32, float>(cwpb, grids);
  }
  if (xkind == XK_BF16) return group_grids_k<64, __bf16>(cwpb, grids);
  if (xkind == XK_F32_TILED) return group_grids_k<64, xtf32>(cwpb, grids);
  return group_grids_k<64, float>(cwpb, grids);
}

template <int KP, typename XT, int WPB>
static void group_iteration_t(const GTable* t, const int64_t* gr, hipStream_t st) {
  kg_colpass<KP, XT, WPB><<<(unsigned)gr[GS_COL], 64 * WPB, 0, st>>>(t);
  kg_reduce_f<<<(unsigned)gr[GS_REDF], 256, 0, st>>>(t);
  kg_sweep<KP><<<(unsigned)gr[GS_SWEEP], 256, 256 * KP * sizeof(float), st>>>(t);
  kg_packw<KP><<<(unsigned)gr[GS_PACKW], 256, 0, st>>>(t);
  kg_vgram<KP><<<(unsigned)gr[GS_VGRAM], 256, 0, st>>>(t);
  kg_reduce_v<KP><<<(unsigned)gr[GS_REDV], 256, 0, st>>>(t);
  kg_rowpass<KP, XT><<<(unsigned)gr[GS_ROW], 256, 0, st>>>(t);
  kg_reduce_w<KP><<<(unsigned)gr[GS_REDW], 256, 0, st>>>(t);
  kg_bupdate<KP><<<(unsigned)gr[GS_BUP], kBupThreads, 0, st>>>(t);
  kg_reduce_g<KP><<<(unsigned)gr[GS_REDG], 256, 0, st>>>(t);
  kg_advance<<<(unsigned)gr[GS_ADV], 64, 0, st>>>(t);
}

template <int KP, typename XT>
static void group_iteration_k(int cwpb, const GTable* t, const int64_t* gr, hipStream_t st) {
  if (cwpb == 8)
    group_iteration_t<KP, XT, 8>(t, gr, st);
  else
    group_iteration_t<KP, XT, 4>(t, gr, st);
}

hipError_t group_iteration(int KP, int xkind, int cwpb, const GTable* dtab, const int64_t grids[GS_N],
                           hipStream_t st) {
  if (KP == 32) {
    if (xkind == XK_BF16)
      group_iteration_k<32, __bf16>(cwpb, dtab, grids, st);
    else if (xkind == XK_F32_TILED)
      group_iteration_k<32, xtf32>(cwpb, dtab, grids, st);
    else
      group_iteration_k<32, float>(cwpb, dtab, grids, st);
  } else {
    if (xkind == XK_BF16)
      group_iteration_k<64, __bf16>(cwpb, dtab, grids, st);
    else if (xkind == XK_F32_TILED)
      group_iteration_k<64, xtf32>(cwpb, dtab, grids, st);
    else
      group_iteration_k<64, float>(cwpb, dtab, grids, st);
  }
  return hipGetLastError();
}

}  // namespace didk
