// gfx950 kernels of the DID engine.
//
// One DID iteration (Alg. 3 of Gao & Chu, AAAI-18) is carried out as
//   colpass column pass over X: E = X - B C (MFMA), f partial = sum E^2 (float64),
//           H = B^T E (MFMA),
//   sweep   the coordinate sweep over the rows of C (float64, one thread per column) and
//           V = C C^T partials of the updated C,
//   rowpass row pass over X: E' = X - B C' (MFMA) and W = E' C'^T per column range (MFMA),
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
// Block = 4 waves = 128 consecutive columns; wave w owns columns 128*blockIdx + 32w ..+31
// and walks all M rows in 32-row chunks:
//   acc  = X[chunk, cols]                        (E tile, accumulator layout)
//   acc += (-B[chunk, :]) C[:, cols]             (ceil(K/2) MFMA steps) -> E = X - B C
//   fsum += sum acc^2                            (float64)
//   H   += B[chunk, :]^T acc                     (16 MFMA steps per 32 rows of H)
// The packed B operands of chunk c+1 are staged into LDS (double buffer shared by the four
// waves) and the X tile of chunk c+1 is loaded into registers while chunk c is computed.
// H is written as KP x N (ld KP) for the sweep kernel.
template <int KP, bool WITH_H>
__global__ __launch_bounds__(256, 2) void k_colpass(const float* __restrict__ X, int64_t M, int64_t N, int K,
                                                    const float* __restrict__ C, const float* __restrict__ BpE,
                                                    const float* __restrict__ BpH, float* __restrict__ Hout,
                                                    double* __restrict__ fpart, int64_t nchunks, int vec4) {
  constexpr int NB = KP / 32;
  constexpr int KS2 = KP / 2;
  constexpr int CH = KP * 32;                    // floats of one packed operand chunk
  constexpr int STG4 = (WITH_H ? 2 * CH : CH) / 4;  // float4 staged per chunk
  constexpr int NV4 = STG4 / 256;                 // float4 per thread per chunk
  __shared__ f32x4 sb[2][STG4];
  __shared__ double fw[4];
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, half = l >> 5, lc = l & 31;
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

  f32x4 stg[NV4];
  auto gload = [&](int64_t c) {
#pragma unroll
    for (int v = 0; v < NV4; ++v) {
      const int idx = tid + 256 * v;
      if (!WITH_H || idx < CH / 4)
        stg[v] = reinterpret_cast<const f32x4*>(BpE + c * (int64_t)CH)[idx];
      else
        stg[v] = reinterpret_cast<const f32x4*>(BpH + c * (int64_t)CH)[idx - CH / 4];
    }
  };
  auto xload = [&](int64_t c) {
    f32x16 v;
    const int64_t m0 = c * 32;
    if (colok && vec4 && m0 + 32 <= M) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 t = *reinterpret_cast<const f32x4*>(xcol + m0 + 8 * q + 4 * half);
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
          v[4 * q + e] = (colok && r < M) ? xcol[r] : 0.0f;
        }
    }
    return v;
  };

  gload(0);
  f32x16 xn = xload(0);
#pragma unroll
  for (int v = 0; v < NV4; ++v) sb[0][tid + 256 * v] = stg[v];
  __syncthreads();

  for (int64_t c = 0; c < nchunks; ++c) {
    const int buf = (int)(c & 1);
    f32x16 acc = xn;
    const bool more = c + 1 < nchunks;
    if (more) {
      gload(c + 1);
      xn = xload(c + 1);
    }
    const f32x4* pe = &sb[buf][0] + l;
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
    if (WITH_H) {
      const f32x4* ph = &sb[buf][CH / 4] + l;
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i4 = 0; i4 < 4; ++i4) {
          const f32x4 a = ph[(b * 4 + i4) * 64];
#pragma unroll
          for (int u = 0; u < 4; ++u) H[b] = mfma32(a[u], acc[4 * i4 + u], H[b]);
        }
    }
    if (more) {
#pragma unroll
      for (int v = 0; v < NV4; ++v) sb[buf ^ 1][tid + 256 * v] = stg[v];
    }
    __syncthreads();
  }

  if (WITH_H && colok) {
    float* hcol = Hout + col * KP;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        f32x4 v;
        v[0] = H[b][4 * q + 0];
        v[1] = H[b][4 * q + 1];
        v[2] = H[b][4 * q + 2];
        v[3] = H[b][4 * q + 3];
        *reinterpret_cast<f32x4*>(hcol + 32 * b + 8 * q + 4 * half) = v;
      }
  }

  double fsum = fs0 + fs1;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) fsum += __shfl_xor(fsum, off, 64);
  if (l == 0) fw[wave] = fsum;
  __syncthreads();
  if (tid == 0) fpart[blockIdx.x] = (fw[0] + fw[1]) + (fw[2] + fw[3]);
}

int64_t colpass_blocks(const Shape& s) { return (s.N + 127) / 128; }

hipError_t colpass(const Shape& s, const float* X, const float* C, const float* BpE, const float* BpH, float* Hout,
                   double* fpart, int with_h, hipStream_t st) {
  const unsigned g = (unsigned)colpass_blocks(s);
  if (s.KP == 32) {
    if (with_h)
      k_colpass<32, true><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, C, BpE, BpH, Hout, fpart, s.nchunks, s.vec4);
    else
      k_colpass<32, false><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, C, BpE, BpH, Hout, fpart, s.nchunks, s.vec4);
  } else {
    if (with_h)
      k_colpass<64, true><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, C, BpE, BpH, Hout, fpart, s.nchunks, s.vec4);
    else
      k_colpass<64, false><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, C, BpE, BpH, Hout, fpart, s.nchunks, s.vec4);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ coordinate sweep
// One thread per column j.  With h = B^T e_j from the column pass and G = B^T B in LDS, the
// coordinates are updated in ascending order in float64:
//   c_kj := [c_kj + h_k / G_kk]_+,  then h_q -= G_qk (c_kj^new - c_kj^old) for q > k,
// which is eq. up:c with b_q^T e_j kept up to date through inner products; a coordinate
// with G_kk = 0 (zero column of B) is skipped.  The updated column is written back to C
// and staged in LDS, where the block adds its columns' outer products c_j c_j^T to its V
// partial (thread t owns the 4x4 block (t / (KP/4), t % (KP/4)) of V).
constexpr int kSweepTiles = 1024;  // upper bound on blocks (V partials) of the sweep

template <int KP>
__global__ __launch_bounds__(256) void k_sweep(const float* __restrict__ Hin, float* __restrict__ C, int64_t N, int K,
                                               const double* __restrict__ G, double* __restrict__ Vpart) {
  constexpr int CS = KP + 4;  // LDS row stride of the staged columns
  constexpr int NBL = KP / 4;
  __shared__ double Gs[KP * KP];
  __shared__ float Ct[256 * CS];
  const int tid = threadIdx.x;
  for (int q = tid; q < KP * KP; q += 256) Gs[q] = G[q];
  const int ab = tid / NBL, bb = tid % NBL;
  const bool vown = tid < NBL * NBL;
  double vacc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) vacc[q] = 0.0;
  const int64_t ntiles = (N + 255) / 256;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();  // Gs ready (first pass); Ct free (later passes)
    const int64_t col = tile * 256 + tid;
    const bool colok = col < N;
    double h[KP];
    if (colok) {
      const f32x4* hp = reinterpret_cast<const f32x4*>(Hin + col * KP);
#pragma unroll
      for (int q = 0; q < KP / 4; ++q) {
        const f32x4 v = hp[q];
        h[4 * q + 0] = v[0];
        h[4 * q + 1] = v[1];
        h[4 * q + 2] = v[2];
        h[4 * q + 3] = v[3];
      }
    } else {
#pragma unroll
      for (int k = 0; k < KP; ++k) h[k] = 0.0;
    }
    float* ccol = C + (colok ? col : 0) * K;
    float* crow = Ct + tid * CS;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      float cnew = 0.0f;
      if (k < K && colok) {
        const double cold = (double)ccol[k];
        double cn = cold;
        const double nk = Gs[k * KP + k];
        if (nk > 0.0) {
          cn = cold + h[k] / nk;
          cn = cn > 0.0 ? cn : 0.0;
          const double d = cn - cold;
#pragma unroll
          for (int q = k + 1; q < KP; ++q) h[q] -= Gs[q * KP + k] * d;
        }
        cnew = (float)cn;
        ccol[k] = cnew;
      }
      crow[k] = cnew;
    }
    __syncthreads();
    if (vown) {
      for (int j = 0; j < 256; ++j) {
        const f32x4 ca = *reinterpret_cast<const f32x4*>(Ct + j * CS + 4 * ab);
        const f32x4 cb = *reinterpret_cast<const f32x4*>(Ct + j * CS + 4 * bb);
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) vacc[4 * r + q] += (double)ca[r] * (double)cb[q];
      }
    }
  }
  if (vown) {
    double* vp = Vpart + (int64_t)blockIdx.x * KP * KP;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) vp[(4 * ab + r) * KP + 4 * bb + q] = vacc[4 * r + q];
  } else {
    // threads without a V block (KP = 32 uses 64 of 256) have nothing to write
  }
}

int64_t sweep_blocks(const Shape& s) {
  const int64_t t = (s.N + 255) / 256;
  return t < kSweepTiles ? t : kSweepTiles;
}

hipError_t sweep(const Shape& s, const float* Hin, float* C, const double* G, double* Vpart, hipStream_t st) {
  const unsigned g = (unsigned)sweep_blocks(s);
  if (s.KP == 32)
    k_sweep<32><<<g, 256, 0, st>>>(Hin, C, s.N, s.K, G, Vpart);
  else
    k_sweep<64><<<g, 256, 0, st>>>(Hin, C, s.N, s.K, G, Vpart);
  return hipGetLastError();
}

// ------------------------------------------------------------------ row pass
// Block = 4 waves; wave w owns the 32-row chunk c = 4*blockIdx.x + w and column range r =
// blockIdx.y.  Per 32 columns of the range (transposed tiles, rows = columns of X):
//   acc  = X[chunk, cols]^T
//   acc += C[:, cols]^T (-B[chunk, :])^T          -> E'^T with E' = X - B C'
//   WT  += C[:, cols] acc                          -> (E' C'^T)^T for this chunk
// The C' tile of the next 32 columns is staged into LDS in both MFMA operand orders
// (double buffer shared by the four waves); X of the next tile is prefetched.
template <int KP>
__global__ __launch_bounds__(256, 2) void k_rowpass(const float* __restrict__ X, int64_t M, int K,
                                                    const float* __restrict__ C, const float* __restrict__ BpE,
                                                    float* __restrict__ Wpart, int64_t Mpad, int64_t nchunks,
                                                    const int64_t* __restrict__ rbounds) {
  constexpr int NB = KP / 32;
  constexpr int KS2 = KP / 2;
  constexpr int TE = KP * 32;      // floats of the E-operand tile
  constexpr int TT = 2 * KP * 32;  // floats of both tiles
  constexpr int NEL = KP / 8;      // tile elements per thread (32 * KP / 256)
  __shared__ float sc[2][TT];
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, half = l >> 5, lc = l & 31;
  const int64_t c = (int64_t)blockIdx.x * 4 + wave;
  const bool active = c < nchunks;  // inactive waves still take part in staging and barriers
  const int r = blockIdx.y;
  const int64_t lo = rbounds[r], hi = rbounds[r + 1];
  const int64_t m0 = (active ? c : 0) * 32, mrow = m0 + lc;
  const bool rowok = active && mrow < M;
  const int KSr = (K + 1) >> 1;

  float bneg[KS2];
  {
    const f32x4* pe = reinterpret_cast<const f32x4*>(BpE + (active ? c : 0) * (int64_t)KP * 32) + l;
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

  // staging of tile elements e = tid + 256 v: jj = e / KP (column in tile), kk = e % KP
  float stv[NEL];
  auto cload = [&](int64_t j0) {
#pragma unroll
    for (int v = 0; v < NEL; ++v) {
      const int e = tid + 256 * v, jj = e / KP, kk = e % KP;
      stv[v] = (j0 + jj < hi && kk < K) ? C[(j0 + jj) * K + kk] : 0.0f;
    }
  };
  auto cstore = [&](int buf) {
#pragma unroll
    for (int v = 0; v < NEL; ++v) {
      const int e = tid + 256 * v, jj = e / KP, kk = e % KP;
      {  // A operand of E'^T: lane l, step s -> C'[2s + l/32][j0 + l%32]
        const int s = kk >> 1, hh = kk & 1, ln = jj + 32 * hh;
        sc[buf][((s >> 2) * 64 + ln) * 4 + (s & 3)] = stv[v];
      }
      {  // A operand of W^T: block b, step i -> C'[32b + l%32][j0 + row32(i, l/32)]
        const int b = kk >> 5, i4 = jj >> 3, hh = (jj >> 2) & 1, u = jj & 3, ln = (kk & 31) + 32 * hh;
        sc[buf][TE + ((b * 4 + i4) * 64 + ln) * 4 + u] = stv[v];
      }
    }
  };
  const float* xrow = X + mrow;
  auto xload = [&](int64_t j0) {
    f32x16 v;
    if (rowok && j0 + 32 <= hi) {
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = xrow[(j0 + row32(i, half)) * M];
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int64_t j = j0 + row32(i, half);
        v[i] = (rowok && j < hi) ? xrow[j * M] : 0.0f;
      }
    }
    return v;
  };

  if (lo < hi) {
    cload(lo);
    f32x16 xn = xload(lo);
    cstore(0);
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = lo; j0 < hi; j0 += 32) {
      f32x16 acc = xn;
      const bool more = j0 + 32 < hi;
      if (more) {
        cload(j0 + 32);
        xn = xload(j0 + 32);
      }
      if (active) {
        const f32x4* pe = reinterpret_cast<const f32x4*>(&sc[buf][0]) + l;
#pragma unroll
        for (int s4 = 0; s4 < KP / 8; ++s4) {
          if (4 * s4 < KSr) {
            const f32x4 a = pe[s4 * 64];
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (4 * s4 + u < KSr) acc = mfma32(a[u], bneg[4 * s4 + u], acc);
          }
        }
        const f32x4* pw = reinterpret_cast<const f32x4*>(&sc[buf][TE]) + l;
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int i4 = 0; i4 < 4; ++i4) {
            const f32x4 a = pw[(b * 4 + i4) * 64];
#pragma unroll
            for (int u = 0; u < 4; ++u) WT[b] = mfma32(a[u], acc[4 * i4 + u], WT[b]);
          }
      }
      if (more) cstore(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  if (active) {
    float* wp = Wpart + (int64_t)r * KP * Mpad;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) wp[(int64_t)(32 * b + row32(i, half)) * Mpad + m0 + lc] = WT[b][i];
  }
}

hipError_t rowpass(const Shape& s, const float* X, const float* C, const float* BpE, float* Wpart,
                   const int64_t* rbounds, int R, hipStream_t st) {
  dim3 g((unsigned)((s.nchunks + 3) / 4), (unsigned)R);
  if (s.KP == 32)
    k_rowpass<32><<<g, 256, 0, st>>>(X, s.M, s.K, C, BpE, Wpart, s.Mpad, s.nchunks, rbounds);
  else
    k_rowpass<64><<<g, 256, 0, st>>>(X, s.M, s.K, C, BpE, Wpart, s.Mpad, s.nchunks, rbounds);
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
