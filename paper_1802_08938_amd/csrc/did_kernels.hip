// gfx950 kernels of the DID engine.
//
// One DID iteration (Alg. 3 of Gao & Chu, AAAI-18) is carried out as
//   pass1   column pass over X: E = X - B C (MFMA), f partial = sum E^2 (float64),
//           H = B^T E (MFMA) and the coordinate sweep over the rows of C,
//   vgram   V = tril(C C^T) partials of the updated C (float64),
//   pass2   row pass over X: E' = X - B C' (MFMA) and W = E' C'^T per column range (MFMA),
//   reduce  fixed-order sums of the V, W and f partials (the paper's one Allreduce),
//   bupdate incremental update of the columns of B, one thread per row of B.
//
// The coordinate sweep over c_j is written in inner-product form.  With the residual
// e_j of the column at the start of the sweep and h = B^T e_j, the running inner product
// b_i^T e_j after coordinates k < i moved by delta c_k is h_i - sum_{k<i} (b_i^T b_k)
// delta c_k, so eq. up:c becomes c_ij := [c_ij + (h_i - sum_{k<i} G_ik delta c_kj) / G_ii]_+
// with G = B^T B.  This is the same identity Section 4 uses for the columns of B (the
// v_ik delta b_k term); it turns the K dependent length-M reductions of the sweep into
// one MFMA contraction plus O(K^2) float64 work per column.
//
// MFMA lane layouts used (v_mfma_f32_32x32x2_f32, one block): lane l supplies A[l%32][l/32]
// and B[l/32][l%32]; accumulator register i of lane l holds D[row32(i, l/32)][l%32] with
// row32(i, h) = 8*(i/4) + 4*h + i%4.  Because the accumulator's row index pairs with
// l/32, accumulator register i can be fed back directly as the B operand of a second
// 32x32x2 MFMA that reduces over those two rows; no lane shuffles are needed.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "did_kernels.h"

namespace didk {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int row32(int i, int h) { return 8 * (i >> 2) + 4 * h + (i & 3); }

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
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
// Packed operand buffers of B (rows >= M and columns >= K stay zero from allocation):
//   BpE[((c*(KP/8) + s/4)*64 + l)*4 + s%4] = -B[32c + l%32][2s + l/32]
//       (A operand of E = X - B C in the column pass; B operand of E' in the row pass)
//   BpH[((c*(KP/32)*4 + b*4 + i/4)*64 + l)*4 + i%4] = B[32c + row32(i, l/32)][32b + l%32]
//       (A operand of H = B^T E in the column pass)
// so that each lane fetches four consecutive MFMA steps with one 16-byte load.
template <int KP>
__device__ __forceinline__ void pack_entry(float* BpE, float* BpH, int64_t m, int kk, float v) {
  constexpr int NB = KP / 32;
  const int64_t c = m >> 5;
  const int r = (int)(m & 31);
  {
    const int s = kk >> 1, l = r + 32 * (kk & 1);
    BpE[((c * (KP / 8) + (s >> 2)) * 64 + l) * 4 + (s & 3)] = -v;
  }
  {
    const int b = kk >> 5, l = 32 * ((r >> 2) & 1) + (kk & 31), i = 4 * (r >> 3) + (r & 3);
    BpH[((c * NB * 4 + b * 4 + (i >> 2)) * 64 + l) * 4 + (i & 3)] = v;
  }
}

// One thread per row m of B.  With update=1 the row follows the incremental rule of
// Section 4 (Alg. 3, 'Update B'):
//   b_mi := [b_mi + (w_mi - sum_{k<i} v_ik delta b_mk) / v_ii]_+,  delta b_mi := new - old,
// for i = 1..K in order, in float64; a column with v_ii = 0 is left unchanged.  Rows are
// independent because V couples only the columns of one row.
template <int KP>
__global__ __launch_bounds__(256) void k_bupdate(float* __restrict__ B, int64_t M, int K,
                                                 const double* __restrict__ W, int64_t Mpad,
                                                 const double* __restrict__ V, float* __restrict__ BpE,
                                                 float* __restrict__ BpH, double* __restrict__ Gpart,
                                                 int update) {
  __shared__ double Vs[KP * KP];
  __shared__ float Bt[256 * (KP + 1)];
  const int tid = threadIdx.x;
  if (update)
    for (int q = tid; q < KP * KP; q += 256) Vs[q] = V[q];
  __syncthreads();
  const int64_t m = (int64_t)blockIdx.x * 256 + tid;
  const bool ok = m < M;
  double db[KP];
#pragma unroll
  for (int i = 0; i < KP; ++i) {
    db[i] = 0.0;
    float bnew = 0.0f;
    if (i < K && ok) {
      const double bold = (double)B[(int64_t)i * M + m];
      double bn = bold;
      if (update) {
        const double vii = Vs[i * KP + i];
        if (vii > 0.0) {
          double s = W[(int64_t)i * Mpad + m];
#pragma unroll
          for (int k = 0; k < KP; ++k)
            if (k < i) s -= Vs[i * KP + k] * db[k];
          bn = bold + s / vii;
          bn = bn > 0.0 ? bn : 0.0;
        }
        db[i] = bn - bold;
      }
      bnew = (float)bn;
      if (update) B[(int64_t)i * M + m] = bnew;
      pack_entry<KP>(BpE, BpH, m, i, bnew);
    }
    Bt[tid * (KP + 1) + i] = bnew;
  }
  __syncthreads();
  // Partial of G = B^T B over this block's rows, float64, pairs (a >= b).
  constexpr int NP = KP * (KP + 1) / 2;
  for (int q = tid; q < NP; q += 256) {
    int a, b;
    pair_of(q, a, b);
    double s0 = 0.0, s1 = 0.0;
    for (int r = 0; r < 256; r += 2) {
      s0 += (double)Bt[r * (KP + 1) + a] * (double)Bt[r * (KP + 1) + b];
      s1 += (double)Bt[(r + 1) * (KP + 1) + a] * (double)Bt[(r + 1) * (KP + 1) + b];
    }
    Gpart[(int64_t)blockIdx.x * NP + q] = s0 + s1;
  }
}

int bupdate_blocks(const Shape& s) { return (int)((s.M + 255) / 256); }

hipError_t bupdate(const Shape& s, float* B, const double* W, const double* V, float* BpE, float* BpH,
                   double* Gpart, int update, hipStream_t st) {
  const unsigned g = (unsigned)bupdate_blocks(s);
  if (s.KP == 32)
    k_bupdate<32><<<g, 256, 0, st>>>(B, s.M, s.K, W, s.Mpad, V, BpE, BpH, Gpart, update);
  else
    k_bupdate<64><<<g, 256, 0, st>>>(B, s.M, s.K, W, s.Mpad, V, BpE, BpH, Gpart, update);
  return hipGetLastError();
}

// ------------------------------------------------------------------ column pass
// Block = 4 waves = 128 consecutive columns; wave w owns columns j0 = 128*blockIdx + 32w
// .. j0+31 and walks all M rows in 32-row chunks:
//   acc  = X[chunk, cols]                        (E tile, accumulator layout)
//   acc += (-B[chunk, :]) C[:, cols]             (K/2 MFMA steps)   -> E = X - B C
//   fsum += sum acc^2                            (float64)
//   H   += B[chunk, :]^T acc                     (16 MFMA steps per 32 rows of H)
// then the sweep over c_j in float64 with G = B^T B staged in LDS, writing C in place.
template <int KP, bool SWEEP>
__global__ __launch_bounds__(256, 2) void k_pass1(const float* __restrict__ X, int64_t M, int64_t N, int K,
                                                  float* __restrict__ C, const float* __restrict__ BpE,
                                                  const float* __restrict__ BpH, const double* __restrict__ G,
                                                  double* __restrict__ fpart, int64_t nchunks, int vec4) {
  constexpr int NB = KP / 32;
  constexpr int KS2 = KP / 2;
  __shared__ double Gs[SWEEP ? KP * KP : 1];
  __shared__ float Hs[SWEEP ? 4 * KP * 33 : 1];
  __shared__ double fw[4];
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, half = l >> 5, lc = l & 31;
  if (SWEEP)
    for (int q = tid; q < KP * KP; q += 256) Gs[q] = G[q];
  const int KSr = (K + 1) >> 1;
  const int64_t col = (int64_t)blockIdx.x * 128 + wave * 32 + lc;
  const bool colok = col < N;
  const float* xcol = X + (colok ? col : 0) * M;

  float creg[KS2];
#pragma unroll
  for (int s = 0; s < KS2; ++s) {
    const int kk = 2 * s + half;
    creg[s] = (colok && kk < K) ? C[col * K + kk] : 0.0f;
  }
  f32x16 H[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int i = 0; i < 16; ++i) H[b][i] = 0.0f;
  double fs0 = 0.0, fs1 = 0.0;

  for (int64_t c = 0; c < nchunks; ++c) {
    const int64_t m0 = c * 32;
    f32x16 acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t rb = m0 + 8 * q + 4 * half;
      if (colok && vec4 && rb + 3 < M) {
        const f32x4 v = *reinterpret_cast<const f32x4*>(xcol + rb);
        acc[4 * q + 0] = v[0];
        acc[4 * q + 1] = v[1];
        acc[4 * q + 2] = v[2];
        acc[4 * q + 3] = v[3];
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[4 * q + e] = (colok && rb + e < M) ? xcol[rb + e] : 0.0f;
      }
    }
    const f32x4* pe = reinterpret_cast<const f32x4*>(BpE + c * (int64_t)KP * 32) + l;
#pragma unroll
    for (int s4 = 0; s4 < KP / 8; ++s4) {
      if (4 * s4 < KSr) {
        const f32x4 a = pe[s4 * 64];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (4 * s4 + u < KSr) acc = mfma32(a[u], creg[4 * s4 + u], acc);
      }
    }
#pragma unroll
    for (int i = 0; i < 16; i += 2) {
      fs0 += (double)acc[i] * (double)acc[i];
      fs1 += (double)acc[i + 1] * (double)acc[i + 1];
    }
    if (SWEEP) {
      const f32x4* ph = reinterpret_cast<const f32x4*>(BpH + c * (int64_t)KP * 32) + l;
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i4 = 0; i4 < 4; ++i4) {
          const f32x4 a = ph[(b * 4 + i4) * 64];
#pragma unroll
          for (int u = 0; u < 4; ++u) H[b] = mfma32(a[u], acc[4 * i4 + u], H[b]);
        }
    }
  }

  if (SWEEP) {
    float* hs = Hs + wave * KP * 33;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) hs[(32 * b + row32(i, half)) * 33 + lc] = H[b][i];
    __syncthreads();  // Gs and this wave's Hs visible
    if (half == 0 && colok) {
      double h[KP];
#pragma unroll
      for (int k = 0; k < KP; ++k) h[k] = (double)hs[k * 33 + lc];
      float* ccol = C + col * K;
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        if (k < K) {
          const double nk = Gs[k * KP + k];
          if (nk > 0.0) {
            const double cold = (double)ccol[k];
            double cn = cold + h[k] / nk;
            cn = cn > 0.0 ? cn : 0.0;
            const double d = cn - cold;
            ccol[k] = (float)cn;
#pragma unroll
            for (int q = k + 1; q < KP; ++q) h[q] -= Gs[q * KP + k] * d;
          }
        }
      }
    }
  }

  double fsum = fs0 + fs1;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) fsum += __shfl_xor(fsum, off, 64);
  if (l == 0) fw[wave] = fsum;
  __syncthreads();
  if (tid == 0) fpart[blockIdx.x] = (fw[0] + fw[1]) + (fw[2] + fw[3]);
}

int64_t pass1_blocks(const Shape& s) { return (s.N + 127) / 128; }

hipError_t pass1(const Shape& s, const float* X, float* C, const float* BpE, const float* BpH, const double* G,
                 double* fpart, int sweep, hipStream_t st) {
  const unsigned g = (unsigned)pass1_blocks(s);
  if (s.KP == 32) {
    if (sweep)
      k_pass1<32, true><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, C, BpE, BpH, G, fpart, s.nchunks, s.vec4);
    else
      k_pass1<32, false><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, C, BpE, BpH, G, fpart, s.nchunks, s.vec4);
  } else {
    if (sweep)
      k_pass1<64, true><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, C, BpE, BpH, G, fpart, s.nchunks, s.vec4);
    else
      k_pass1<64, false><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, C, BpE, BpH, G, fpart, s.nchunks, s.vec4);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ row pass
// Block = 4 waves; wave w owns the 32-row chunk c = 4*blockIdx.x + w and column range r =
// blockIdx.y.  Per 32 columns of the range (transposed tiles, rows = columns of X):
//   acc  = X[chunk, cols]^T
//   acc += C[:, cols]^T (-B[chunk, :])^T          -> E'^T with E' = X - B C'
//   WT  += C[:, cols] acc                          -> (E' C'^T)^T for this chunk
template <int KP>
__global__ __launch_bounds__(256, 2) void k_pass2(const float* __restrict__ X, int64_t M, int K,
                                                  const float* __restrict__ C, const float* __restrict__ BpE,
                                                  float* __restrict__ Wpart, int64_t Mpad, int64_t nchunks,
                                                  const int64_t* __restrict__ rbounds) {
  constexpr int NB = KP / 32;
  constexpr int KS2 = KP / 2;
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, half = l >> 5, lc = l & 31;
  const int64_t c = (int64_t)blockIdx.x * 4 + wave;
  if (c >= nchunks) return;
  const int r = blockIdx.y;
  const int64_t lo = rbounds[r], hi = rbounds[r + 1];
  const int64_t m0 = c * 32, mrow = m0 + lc;
  const bool rowok = mrow < M;
  const int KSr = (K + 1) >> 1;

  float bneg[KS2];
  {
    const f32x4* pe = reinterpret_cast<const f32x4*>(BpE + c * (int64_t)KP * 32) + l;
#pragma unroll
    for (int s4 = 0; s4 < KP / 8; ++s4) {
      const f32x4 a = pe[s4 * 64];
#pragma unroll
      for (int u = 0; u < 4; ++u) bneg[4 * s4 + u] = a[u];
    }
  }
  f32x16 WT[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int i = 0; i < 16; ++i) WT[b][i] = 0.0f;

  for (int64_t j0 = lo; j0 < hi; j0 += 32) {
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int64_t j = j0 + row32(i, half);
      acc[i] = (rowok && j < hi) ? X[j * M + mrow] : 0.0f;
    }
    const int64_t ja = j0 + lc;
    const bool jaok = ja < hi;
#pragma unroll
    for (int s = 0; s < KS2; ++s) {
      if (s < KSr) {
        const int kk = 2 * s + half;
        const float a = (jaok && kk < K) ? C[ja * K + kk] : 0.0f;
        acc = mfma32(a, bneg[s], acc);
      }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int kk = 32 * b + lc;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int64_t jj = j0 + row32(i, half);
        const float a = (jj < hi && kk < K) ? C[jj * K + kk] : 0.0f;
        WT[b] = mfma32(a, acc[i], WT[b]);
      }
    }
  }
  float* wp = Wpart + (int64_t)r * KP * Mpad;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int i = 0; i < 16; ++i) wp[(int64_t)(32 * b + row32(i, half)) * Mpad + m0 + lc] = WT[b][i];
}

hipError_t pass2(const Shape& s, const float* X, const float* C, const float* BpE, float* Wpart,
                 const int64_t* rbounds, int R, hipStream_t st) {
  dim3 g((unsigned)((s.nchunks + 3) / 4), (unsigned)R);
  if (s.KP == 32)
    k_pass2<32><<<g, 256, 0, st>>>(X, s.M, s.K, C, BpE, Wpart, s.Mpad, s.nchunks, rbounds);
  else
    k_pass2<64><<<g, 256, 0, st>>>(X, s.M, s.K, C, BpE, Wpart, s.Mpad, s.nchunks, rbounds);
  return hipGetLastError();
}

// ------------------------------------------------------------------ V = tril(C C^T)
// Block b owns VG tiles of 256 consecutive columns; a tile of C is contiguous in memory.
constexpr int kVTiles = 16;

template <int KP>
__global__ __launch_bounds__(256) void k_vgram(const float* __restrict__ C, int64_t N, int K,
                                               double* __restrict__ Vpart) {
  constexpr int NP = KP * (KP + 1) / 2;
  constexpr int NQ = (NP + 255) / 256;
  __shared__ float Cs[256 * KP];
  const int tid = threadIdx.x;
  int qa[NQ], qb[NQ];
  double acc[NQ];
#pragma unroll
  for (int t = 0; t < NQ; ++t) {
    const int q = tid + 256 * t;
    if (q < NP) pair_of(q, qa[t], qb[t]);
    else qa[t] = qb[t] = 0;
    acc[t] = 0.0;
  }
  for (int vt = 0; vt < kVTiles; ++vt) {
    const int64_t j0 = ((int64_t)blockIdx.x * kVTiles + vt) * 256;
    if (j0 >= N) break;  // uniform across the block
    const int64_t nv = (N - j0) < 256 ? (N - j0) : 256;
    __syncthreads();
    for (int64_t t = tid; t < nv * K; t += 256) Cs[t] = C[j0 * K + t];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
      const int q = tid + 256 * t;
      if (q < NP && qa[t] < K) {
        const int a = qa[t], b = qb[t];
        double s = 0.0;
        for (int j = 0; j < nv; ++j) s += (double)Cs[j * K + a] * (double)Cs[j * K + b];
        acc[t] += s;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NQ; ++t) {
    const int q = tid + 256 * t;
    if (q < NP) Vpart[(int64_t)blockIdx.x * NP + q] = acc[t];
  }
}

int64_t vgram_blocks(const Shape& s) { return (s.N + 256 * kVTiles - 1) / (256 * kVTiles); }

hipError_t vgram(const Shape& s, const float* C, double* Vpart, hipStream_t st) {
  const unsigned g = (unsigned)vgram_blocks(s);
  if (s.KP == 32)
    k_vgram<32><<<g, 256, 0, st>>>(C, s.N, s.K, Vpart);
  else
    k_vgram<64><<<g, 256, 0, st>>>(C, s.N, s.K, Vpart);
  return hipGetLastError();
}

// ------------------------------------------------------------------ reductions
// W[kk][m] = sum_r Wpart[r][kk][m], r ascending, float64.
__global__ void k_reduce_w(const float* __restrict__ Wpart, int R, int64_t n, double* __restrict__ W) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int r = 0; r < R; ++r) s += (double)Wpart[(int64_t)r * n + i];
  W[i] = s;
}

hipError_t reduce_w(const Shape& s, const float* Wpart, int R, double* W, hipStream_t st) {
  const int64_t n = (int64_t)s.KP * s.Mpad;
  k_reduce_w<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(Wpart, R, n, W);
  return hipGetLastError();
}

// full[a][b] = full[b][a] = sum_p part[p][pair(a,b)], p ascending.
__global__ void k_reduce_sym(const double* __restrict__ part, int64_t P, int KP, double* __restrict__ full) {
  const int NP = KP * (KP + 1) / 2;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= NP) return;
  double s = 0.0;
  for (int64_t p = 0; p < P; ++p) s += part[p * NP + q];
  int a, b;
  pair_of(q, a, b);
  full[a * KP + b] = s;
  full[b * KP + a] = s;
}

hipError_t reduce_sym(const double* part, int64_t P, int KP, double* full, hipStream_t st) {
  const int NP = KP * (KP + 1) / 2;
  k_reduce_sym<<<(unsigned)((NP + 255) / 256), 256, 0, st>>>(part, P, KP, full);
  return hipGetLastError();
}

// *out = scale * sum_p part[p]: each thread sums a strided subset in order, then a fixed
// tree over the block.
__global__ __launch_bounds__(256) void k_reduce_f(const double* __restrict__ part, int64_t P, double* out,
                                                  double scale) {
  __shared__ double s[256];
  double a = 0.0;
  for (int64_t p = threadIdx.x; p < P; p += 256) a += part[p];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = scale * s[0];
}

hipError_t reduce_f(const double* part, int64_t P, double* out, double scale, hipStream_t st) {
  k_reduce_f<<<1, 256, 0, st>>>(part, P, out, scale);
  return hipGetLastError();
}

}  // namespace didk
