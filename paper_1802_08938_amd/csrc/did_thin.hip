// Thin-matrix path of the DID engine (M <= 16 rows, K <= 8 coordinates), e.g. the
// experiments' synthetic sets with M = 5, K = 3 and up to 10^8 samples.
//
// With so few rows a whole column x_j, its residual e_j and its coordinates c_j fit in
// registers, so one thread carries out, for its columns, exactly the per-column work of
// Alg. 3 in a single pass over X:
//   e_j := x_j - B c_j,
//   for i = 1..K: c_ij := [c_ij + b_i^T e_j / (b_i^T b_i)]_+, e_j := e_j - b_i (c_ij^new - c_ij^old)
//       (eq. sol:c_ij with the running residual of eq. up:c),
//   W_j = e_j c_j^T and V_j = c_j c_j^T (eqs. W_j, V_j), and |e_j|^2 of the iterate it
//   started from,
// all in float64, accumulated per thread and then summed over the block in a fixed order
// (the block partials are the paper's per-node messages; their fixed-order sum is the
// single Allreduce).  The B update itself is the shared per-row kernel of the main path.
//
// The same path also runs DBCD (Alg. 2) as an ablation: the same C half, then for every
// i = 1..K one pass over X forms y_j = (e_j + b_i c_ij) c_ij and z_j = c_ij^2 with e_j
// recomputed for the current B, one reduction, and b_i := [y / z]_+ -- K reductions per
// iteration where DID needs one.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "did_kernels.h"

namespace didk {

namespace {

// Deterministic wave-level sum (butterfly with a fixed lane pattern).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int kThinBlocks = 1024;

}  // namespace

int thin_slots(int MM, int KK) { return MM * KK + KK * KK + 1; }

// MODE 0: DID column work (sweep, W/V/f partials, C written back)
// MODE 1: objective only (f partial)
// MODE 2: DBCD C half (sweep, f partial, C written back)
template <int MM, int KK, int MODE>
__global__ __launch_bounds__(256) void k_thin(const float* __restrict__ X, int64_t M, int64_t N, int K,
                                             const float* __restrict__ B, const double* __restrict__ G, int KP,
                                             float* __restrict__ C, double* __restrict__ part) {
  constexpr int NS = MM * KK + KK * KK + 1;
  __shared__ double Bs[MM * KK];
  __shared__ double nk[KK];
  __shared__ double red[4][NS];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int q = tid; q < MM * KK; q += 256) {
    const int m = q % MM, k = q / MM;
    Bs[q] = (m < M && k < K) ? (double)B[(int64_t)k * M + m] : 0.0;
  }
  if (tid < KK) nk[tid] = tid < K ? G[tid * KP + tid] : 0.0;
  __syncthreads();
  double Wacc[MM][KK], Vacc[KK][KK], facc = 0.0;
#pragma unroll
  for (int m = 0; m < MM; ++m)
#pragma unroll
    for (int k = 0; k < KK; ++k) Wacc[m][k] = 0.0;
#pragma unroll
  for (int a = 0; a < KK; ++a)
#pragma unroll
    for (int b = 0; b < KK; ++b) Vacc[a][b] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t j = (int64_t)blockIdx.x * 256 + tid; j < N; j += stride) {
    double e[MM], c[KK];
    const float* xj = X + j * M;
    float* cj = C + j * K;
#pragma unroll
    for (int k = 0; k < KK; ++k) c[k] = k < K ? (double)cj[k] : 0.0;
#pragma unroll
    for (int m = 0; m < MM; ++m) {
      double v = m < M ? (double)xj[m] : 0.0;
#pragma unroll
      for (int k = 0; k < KK; ++k) v -= Bs[k * MM + m] * c[k];
      e[m] = v;
      facc += v * v;
    }
    if (MODE != 1) {
#pragma unroll
      for (int k = 0; k < KK; ++k) {
        if (k < K && nk[k] > 0.0) {
          double g = 0.0;
#pragma unroll
          for (int m = 0; m < MM; ++m) g += Bs[k * MM + m] * e[m];
          double cn = c[k] + g / nk[k];
          cn = cn > 0.0 ? cn : 0.0;
          const double cf = (double)(float)cn;  // the stored (float32) coordinate
          const double d = cf - c[k];
#pragma unroll
          for (int m = 0; m < MM; ++m) e[m] -= Bs[k * MM + m] * d;
          c[k] = cf;
        }
      }
#pragma unroll
      for (int k = 0; k < KK; ++k)
        if (k < K) cj[k] = (float)c[k];
    }
    if (MODE == 0) {
#pragma unroll
      for (int m = 0; m < MM; ++m)
#pragma unroll
        for (int k = 0; k < KK; ++k) Wacc[m][k] += e[m] * c[k];
#pragma unroll
      for (int a = 0; a < KK; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) Vacc[a][b] += c[a] * c[b];
    }
  }
  // block partials: wave butterflies, then the four waves in order
  auto put = [&](int slot, double v) {
    v = wave_sum(v);
    if (lane == 0) red[wave][slot] = v;
  };
  if (MODE == 0) {
#pragma unroll
    for (int m = 0; m < MM; ++m)
#pragma unroll
      for (int k = 0; k < KK; ++k) put(k * MM + m, Wacc[m][k]);
#pragma unroll
    for (int a = 0; a < KK; ++a)
#pragma unroll
      for (int b = 0; b < KK; ++b) put(MM * KK + a * KK + b, b <= a ? Vacc[a][b] : 0.0);
  } else if (lane == 0) {
    for (int q = 0; q < NS - 1; ++q) red[wave][q] = 0.0;
  }
  put(NS - 1, facc);
  __syncthreads();
  for (int q = tid; q < NS; q += 256)
    part[(int64_t)blockIdx.x * NS + q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
}

// Sum the block partials in block order into W (KP x Mpad, float64, row kk), V (KP x KP,
// symmetric) and scale * f; with_wv = 0 sums only f.
template <int MM, int KK>
__global__ __launch_bounds__(256) void k_thin_reduce(const double* __restrict__ part, int64_t P, int KP,
                                                    int64_t Mpad, double* __restrict__ W, double* __restrict__ V,
                                                    double* __restrict__ fout, double scale, int with_wv) {
  constexpr int NS = MM * KK + KK * KK + 1;
  for (int q = threadIdx.x; q < NS; q += 256) {
    if (!with_wv && q != NS - 1) continue;
    double s = 0.0;
    for (int64_t p = 0; p < P; ++p) s += part[p * NS + q];
    if (q < MM * KK) {
      const int m = q % MM, k = q / MM;
      W[(int64_t)k * Mpad + m] = s;
    } else if (q < NS - 1) {
      const int r = q - MM * KK, a = r / KK, b = r % KK;
      if (b <= a) {
        V[a * KP + b] = s;
        V[b * KP + a] = s;
      }
    } else {
      *fout = scale * s;
    }
  }
}

// DBCD, step i: block partials of y = sum_j (e_j + b_i c_ij) c_ij and z = sum_j c_ij^2 with
// e_j = x_j - B c_j for the current B.
template <int MM, int KK>
__global__ __launch_bounds__(256) void k_dbcd_yz(const float* __restrict__ X, int64_t M, int64_t N, int K, int i,
                                                const float* __restrict__ B, const float* __restrict__ C,
                                                double* __restrict__ part) {
  __shared__ double Bs[MM * KK];
  __shared__ double red[4][MM + 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int q = tid; q < MM * KK; q += 256) {
    const int m = q % MM, k = q / MM;
    Bs[q] = (m < M && k < K) ? (double)B[(int64_t)k * M + m] : 0.0;
  }
  __syncthreads();
  double y[MM], z = 0.0;
#pragma unroll
  for (int m = 0; m < MM; ++m) y[m] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t j = (int64_t)blockIdx.x * 256 + tid; j < N; j += stride) {
    double c[KK];
    const float* cj = C + j * K;
#pragma unroll
    for (int k = 0; k < KK; ++k) c[k] = k < K ? (double)cj[k] : 0.0;
    double ci = 0.0;
#pragma unroll
    for (int k = 0; k < KK; ++k)
      if (k == i) ci = c[k];
    const float* xj = X + j * M;
#pragma unroll
    for (int m = 0; m < MM; ++m) {
      double v = m < M ? (double)xj[m] : 0.0;
#pragma unroll
      for (int k = 0; k < KK; ++k)
        if (k != i) v -= Bs[k * MM + m] * c[k];  // e_j + b_i c_ij
      y[m] += v * ci;
    }
    z += ci * ci;
  }
#pragma unroll
  for (int m = 0; m < MM; ++m) {
    const double v = wave_sum(y[m]);
    if (lane == 0) red[wave][m] = v;
  }
  {
    const double v = wave_sum(z);
    if (lane == 0) red[wave][MM] = v;
  }
  __syncthreads();
  for (int q = tid; q <= MM; q += 256)
    part[(int64_t)blockIdx.x * (MM + 1) + q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
}

// DBCD, step i: b_i := [y / z]_+ from the block partials (summed in block order); a zero
// row of C (z = 0) leaves b_i unchanged.
template <int MM>
__global__ void k_dbcd_b(const double* __restrict__ part, int64_t P, int64_t M, int i, float* __restrict__ B) {
  __shared__ double zs;
  const int t = threadIdx.x;
  if (t == 0) {
    double z = 0.0;
    for (int64_t p = 0; p < P; ++p) z += part[p * (MM + 1) + MM];
    zs = z;
  }
  __syncthreads();
  if (t < M && zs > 0.0) {
    double y = 0.0;
    for (int64_t p = 0; p < P; ++p) y += part[p * (MM + 1) + t];
    const double b = y / zs;
    B[(int64_t)i * M + t] = (float)(b > 0.0 ? b : 0.0);
  }
}

int64_t thin_blocks(const Shape& s) {
  const int64_t t = (s.N + 255) / 256;
  return t < kThinBlocks ? t : kThinBlocks;
}

template <int MM, int KK>
static void thin_dispatch(const Shape& s, const float* X, const float* B, const double* G, float* C, double* part,
                          int mode, hipStream_t st) {
  const unsigned g = (unsigned)thin_blocks(s);
  if (mode == 0)
    k_thin<MM, KK, 0><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, B, G, s.KP, C, part);
  else if (mode == 1)
    k_thin<MM, KK, 1><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, B, G, s.KP, C, part);
  else
    k_thin<MM, KK, 2><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, B, G, s.KP, C, part);
}

hipError_t thin_pass(const Shape& s, const float* X, const float* B, const double* G, float* C, double* part,
                     int mode, hipStream_t st) {
  if (s.M <= 8 && s.K <= 4)
    thin_dispatch<8, 4>(s, X, B, G, C, part, mode, st);
  else if (s.M <= 8)
    thin_dispatch<8, 8>(s, X, B, G, C, part, mode, st);
  else if (s.K <= 4)
    thin_dispatch<16, 4>(s, X, B, G, C, part, mode, st);
  else
    thin_dispatch<16, 8>(s, X, B, G, C, part, mode, st);
  return hipGetLastError();
}

hipError_t thin_reduce(const Shape& s, const double* part, double* W, double* V, double* fout, double scale,
                       int with_wv, hipStream_t st) {
  const int64_t P = thin_blocks(s);
  if (s.M <= 8 && s.K <= 4)
    k_thin_reduce<8, 4><<<1, 256, 0, st>>>(part, P, s.KP, s.Mpad, W, V, fout, scale, with_wv);
  else if (s.M <= 8)
    k_thin_reduce<8, 8><<<1, 256, 0, st>>>(part, P, s.KP, s.Mpad, W, V, fout, scale, with_wv);
  else if (s.K <= 4)
    k_thin_reduce<16, 4><<<1, 256, 0, st>>>(part, P, s.KP, s.Mpad, W, V, fout, scale, with_wv);
  else
    k_thin_reduce<16, 8><<<1, 256, 0, st>>>(part, P, s.KP, s.Mpad, W, V, fout, scale, with_wv);
  return hipGetLastError();
}

hipError_t dbcd_b_step(const Shape& s, const float* X, float* B, const float* C, double* part, int i, hipStream_t st) {
  const unsigned g = (unsigned)thin_blocks(s);
  if (s.M <= 8) {
    if (s.K <= 4)
      k_dbcd_yz<8, 4><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, i, B, C, part);
    else
      k_dbcd_yz<8, 8><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, i, B, C, part);
    k_dbcd_b<8><<<1, 64, 0, st>>>(part, g, s.M, i, B);
  } else {
    if (s.K <= 4)
      k_dbcd_yz<16, 4><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, i, B, C, part);
    else
      k_dbcd_yz<16, 8><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, i, B, C, part);
    k_dbcd_b<16><<<1, 64, 0, st>>>(part, g, s.M, i, B);
  }
  return hipGetLastError();
}

}  // namespace didk
