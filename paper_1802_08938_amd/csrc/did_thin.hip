// Thin-matrix path of the DID engine (M <= 16 rows, K <= 8 coordinates, M <= 8 or K <= 4),
// e.g. the experiments' synthetic sets with M = 5, K = 3 and up to 10^8 samples.
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

// columns in flight per thread: fewer for the larger shapes, whose float64 accumulators
// already take most of the registers
constexpr int thin_pf(int MM, int KK) { return MM * KK <= 16 ? 3 : (MM * KK <= 32 ? 2 : 1); }

}  // namespace

int thin_slots(int MM, int KK) { return MM * KK + KK * KK + 1; }

// One column's data as loaded: x_j (MM rows) and c_j (KK coordinates), float32.
template <int MM, int KK>
struct ThinCol {
  float x[MM];
  float c[KK];
};

// MODE 0: DID column work (sweep, W/V/f partials, C written back)
// MODE 1: objective only (f partial)
// MODE 2: DBCD C half (sweep, f partial, C written back)
// EXACT: M == MM and K == KK (no padding rows or coordinates).
// Each thread takes columns j, j + S, j + 2S, ... (S = threads in the grid) and keeps the
// next thin_pf(MM, KK) of its columns in flight while it works on the current one.
template <int MM, int KK, int MODE, bool EXACT>
__global__ __launch_bounds__(256) void k_thin(const float* __restrict__ X, int64_t M, int64_t N, int K,
                                             const float* __restrict__ B, const double* __restrict__ G, int KP,
                                             float* __restrict__ C, double* __restrict__ part) {
  constexpr int NS = MM * KK + KK * KK + 1;
  constexpr int PF = thin_pf(MM, KK);
  const int Mr = EXACT ? MM : (int)M;
  const int Kr = EXACT ? KK : K;
  __shared__ double Bs[MM * KK];
  __shared__ double nk[KK];
  __shared__ double red[4][NS];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int q = tid; q < MM * KK; q += 256) {
    const int m = q % MM, k = q / MM;
    Bs[q] = (m < Mr && k < Kr) ? (double)B[(int64_t)k * M + m] : 0.0;
  }
  if (tid < KK) nk[tid] = tid < Kr ? G[tid * KP + tid] : 0.0;
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

  auto load = [&](int64_t j) {
    ThinCol<MM, KK> v;
    if (j < N) {
      const float* xj = X + j * M;
      const float* cj = C + j * K;
#pragma unroll
      for (int m = 0; m < MM; ++m) v.x[m] = m < Mr ? xj[m] : 0.0f;
#pragma unroll
      for (int k = 0; k < KK; ++k) v.c[k] = k < Kr ? cj[k] : 0.0f;
    } else {
#pragma unroll
      for (int m = 0; m < MM; ++m) v.x[m] = 0.0f;
#pragma unroll
      for (int k = 0; k < KK; ++k) v.c[k] = 0.0f;
    }
    return v;
  };
  auto process = [&](int64_t j, const ThinCol<MM, KK>& v) {
    double e[MM], c[KK];
#pragma unroll
    for (int k = 0; k < KK; ++k) c[k] = (double)v.c[k];
#pragma unroll
    for (int m = 0; m < MM; ++m) {
      double r = (double)v.x[m];
#pragma unroll
      for (int k = 0; k < KK; ++k) r -= Bs[k * MM + m] * c[k];
      e[m] = r;
      facc += r * r;
    }
    if (MODE != 1) {
#pragma unroll
      for (int k = 0; k < KK; ++k) {
        if (k < Kr && nk[k] > 0.0) {
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
      float* cj = C + j * K;
#pragma unroll
      for (int k = 0; k < KK; ++k)
        if (k < Kr) cj[k] = (float)c[k];
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
  };

  const int64_t stride = (int64_t)gridDim.x * 256;
  const int64_t j0 = (int64_t)blockIdx.x * 256 + tid;
  ThinCol<MM, KK> ring[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) ring[p] = load(j0 + p * stride);
  for (int64_t j = j0; j < N; j += PF * stride) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int64_t jj = j + p * stride;
      if (jj >= N) break;
      const ThinCol<MM, KK> cur = ring[p];
      ring[p] = load(jj + PF * stride);
      process(jj, cur);
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

// Sum of slot q over the P block partials (stride NS), by one wave: lane l adds partials
// l, l + 64, ... in order (their loads issued eight at a time ahead of the additions), then
// a fixed butterfly.  Same result on every call.
__device__ __forceinline__ double slot_sum(const double* __restrict__ part, int64_t P, int NS, int q, int lane) {
  constexpr int G = 8;
  double s = 0.0;
  int64_t p = lane;
  for (; p + (G - 1) * 64 < P; p += G * 64) {
    double v[G];
#pragma unroll
    for (int u = 0; u < G; ++u) v[u] = part[(p + u * 64) * NS + q];
#pragma unroll
    for (int u = 0; u < G; ++u) s += v[u];
  }
  for (; p < P; p += 64) s += part[p * NS + q];
  return wave_sum(s);
}

// One wave (block of 64) per slot: W (KP x Mpad, float64, row kk), V (KP x KP, symmetric)
// and scale * f from the block partials; with_wv = 0 sums only f.
template <int MM, int KK>
__global__ __launch_bounds__(64) void k_thin_reduce(const double* __restrict__ part, int64_t P, int KP,
                                                   int64_t Mpad, double* __restrict__ W, double* __restrict__ V,
                                                   double* __restrict__ fout, double scale, int with_wv) {
  constexpr int NS = MM * KK + KK * KK + 1;
  const int q = with_wv ? (int)blockIdx.x : NS - 1;
  const int lane = threadIdx.x;
  if (q < MM * KK) {
    const double s = slot_sum(part, P, NS, q, lane);
    const int m = q % MM, k = q / MM;
    if (lane == 0) W[(int64_t)k * Mpad + m] = s;
  } else if (q < NS - 1) {
    const int r = q - MM * KK, a = r / KK, b = r % KK;
    if (b > a) return;
    const double s = slot_sum(part, P, NS, q, lane);
    if (lane == 0) {
      V[a * KP + b] = s;
      V[b * KP + a] = s;
    }
  } else {
    const double s = slot_sum(part, P, NS, q, lane);
    if (lane == 0) *fout = scale * s;
  }
}

// DBCD, step i: block partials of y = sum_j (e_j + b_i c_ij) c_ij and z = sum_j c_ij^2 with
// e_j = x_j - B c_j for the current B.
template <int MM, int KK, bool EXACT>
__global__ __launch_bounds__(256) void k_dbcd_yz(const float* __restrict__ X, int64_t M, int64_t N, int K, int i,
                                                const float* __restrict__ B, const float* __restrict__ C,
                                                double* __restrict__ part) {
  constexpr int PF = thin_pf(MM, KK);
  const int Mr = EXACT ? MM : (int)M;
  const int Kr = EXACT ? KK : K;
  __shared__ double Bs[MM * KK];
  __shared__ double red[4][MM + 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int q = tid; q < MM * KK; q += 256) {
    const int m = q % MM, k = q / MM;
    Bs[q] = (m < Mr && k < Kr) ? (double)B[(int64_t)k * M + m] : 0.0;
  }
  __syncthreads();
  double y[MM], z = 0.0;
#pragma unroll
  for (int m = 0; m < MM; ++m) y[m] = 0.0;
  auto load = [&](int64_t j) {
    ThinCol<MM, KK> v;
    if (j < N) {
      const float* xj = X + j * M;
      const float* cj = C + j * K;
#pragma unroll
      for (int m = 0; m < MM; ++m) v.x[m] = m < Mr ? xj[m] : 0.0f;
#pragma unroll
      for (int k = 0; k < KK; ++k) v.c[k] = k < Kr ? cj[k] : 0.0f;
    } else {
#pragma unroll
      for (int m = 0; m < MM; ++m) v.x[m] = 0.0f;
#pragma unroll
      for (int k = 0; k < KK; ++k) v.c[k] = 0.0f;
    }
    return v;
  };
  auto process = [&](const ThinCol<MM, KK>& v) {
    double c[KK], ci = 0.0;
#pragma unroll
    for (int k = 0; k < KK; ++k) {
      c[k] = (double)v.c[k];
      if (k == i) ci = c[k];
    }
#pragma unroll
    for (int m = 0; m < MM; ++m) {
      double r = (double)v.x[m];
#pragma unroll
      for (int k = 0; k < KK; ++k)
        if (k != i) r -= Bs[k * MM + m] * c[k];  // e_j + b_i c_ij
      y[m] += r * ci;
    }
    z += ci * ci;
  };
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int64_t j0 = (int64_t)blockIdx.x * 256 + tid;
  ThinCol<MM, KK> ring[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) ring[p] = load(j0 + p * stride);
  for (int64_t j = j0; j < N; j += PF * stride) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int64_t jj = j + p * stride;
      if (jj >= N) break;
      const ThinCol<MM, KK> cur = ring[p];
      ring[p] = load(jj + PF * stride);
      process(cur);
    }
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

// DBCD, step i: the MM + 1 sums (y, then z) over the block partials, one wave per slot.
template <int MM>
__global__ __launch_bounds__(64) void k_dbcd_sum(const double* __restrict__ part, int64_t P,
                                                double* __restrict__ yz) {
  const double s = slot_sum(part, P, MM + 1, (int)blockIdx.x, threadIdx.x);
  if (threadIdx.x == 0) yz[blockIdx.x] = s;
}

// DBCD, step i: b_i := [y / z]_+; a zero row of C (z = 0) leaves b_i unchanged.
template <int MM>
__global__ __launch_bounds__(64) void k_dbcd_b(const double* __restrict__ yz, int64_t M, int i,
                                              float* __restrict__ B) {
  const int t = threadIdx.x;
  const double z = yz[MM];
  if (t < M && z > 0.0) {
    const double b = yz[t] / z;
    B[(int64_t)i * M + t] = (float)(b > 0.0 ? b : 0.0);
  }
}

int64_t thin_blocks(const Shape& s) { return s.thin_grid; }

// Instances: the experiments' shape (5 x 3) exactly, and padded 8 x 4, 8 x 8, 16 x 4
// (the thin path takes M <= 16, K <= 8 with M <= 8 or K <= 4).
#define DID_THIN_SHAPES(X_) \
  if (s.M == 5 && s.K == 3) { X_(5, 3, true); }        \
  else if (s.M <= 8 && s.K <= 4) { X_(8, 4, false); }  \
  else if (s.M <= 8) { X_(8, 8, false); }              \
  else { X_(16, 4, false); }

// Partial slots per block of the instance the shape runs (the size of its block partials).
int thin_slots_for(const Shape& s) {
  int n = 0;
#define DID_THIN_NS(MM, KK, EX) n = thin_slots(MM, KK);
  DID_THIN_SHAPES(DID_THIN_NS)
#undef DID_THIN_NS
  return n;
}

// One full wave of resident blocks of the DID column kernel (blocks per CU from the
// occupancy calculator times the CU count), at most one block per 256 columns.
int64_t thin_grid_for(const Shape& s) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -1;
  hipError_t e = hipSuccess;
#define DID_THIN_OCC(MM, KK, EX) \
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_thin<MM, KK, 0, EX>, 256, 0);
  DID_THIN_SHAPES(DID_THIN_OCC)
#undef DID_THIN_OCC
  if (e != hipSuccess) return -1;
  int64_t g = (int64_t)(per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
  const int64_t need = (s.N + 255) / 256;
  return g < need ? g : need;
}

hipError_t thin_pass(const Shape& s, const float* X, const float* B, const double* G, float* C, double* part,
                     int mode, hipStream_t st) {
  const unsigned g = (unsigned)thin_blocks(s);
#define DID_THIN_PASS(MM, KK, EX)                                                                \
  if (mode == 0)                                                                                 \
    k_thin<MM, KK, 0, EX><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, B, G, s.KP, C, part);             \
  else if (mode == 1)                                                                            \
    k_thin<MM, KK, 1, EX><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, B, G, s.KP, C, part);             \
  else                                                                                           \
    k_thin<MM, KK, 2, EX><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, B, G, s.KP, C, part);
  DID_THIN_SHAPES(DID_THIN_PASS)
#undef DID_THIN_PASS
  return hipGetLastError();
}

hipError_t thin_reduce(const Shape& s, const double* part, double* W, double* V, double* fout, double scale,
                       int with_wv, hipStream_t st) {
  const int64_t P = thin_blocks(s);
#define DID_THIN_RED(MM, KK, EX)                                                                   \
  k_thin_reduce<MM, KK><<<with_wv ? thin_slots(MM, KK) : 1, 64, 0, st>>>(part, P, s.KP, s.Mpad, W, V, fout, \
                                                                         scale, with_wv);
  DID_THIN_SHAPES(DID_THIN_RED)
#undef DID_THIN_RED
  return hipGetLastError();
}

hipError_t dbcd_b_step(const Shape& s, const float* X, float* B, const float* C, double* part, double* yz, int i,
                       hipStream_t st) {
  const unsigned g = (unsigned)thin_blocks(s);
#define DID_DBCD(MM, KK, EX)                                                   \
  k_dbcd_yz<MM, KK, EX><<<g, 256, 0, st>>>(X, s.M, s.N, s.K, i, B, C, part); \
  k_dbcd_sum<MM><<<MM + 1, 64, 0, st>>>(part, g, yz);                        \
  k_dbcd_b<MM><<<1, 64, 0, st>>>(yz, s.M, i, B);
  DID_THIN_SHAPES(DID_DBCD)
#undef DID_DBCD
  return hipGetLastError();
}

}  // namespace didk
