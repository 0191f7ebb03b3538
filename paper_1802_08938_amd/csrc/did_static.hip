// Allocation-free form of did_iterate: did_iterate_static (include/did.h).
//
// For callers that cannot allocate device memory.  The instance's intermediate buffers
// (packed operands, partials, the per-range W partials, H, ...) are carved from one fixed
// device array, `scratch`, instead of hipMalloc'd buffers; the caller passes X, B and C.
// In host code the array's name is only a stand-in for its device address: that address
// is taken once per device with hipGetSymbolAddress and kept per device, and only that
// address reaches kernels and fill launches.  The iteration itself is the engine's own
// (iterate_mfma), so the iterates equal those of did_init_from_factors + did_iterate.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "../../include/did.h"
#include "did_engine.h"
#include "did_kernels.h"

using didk::Shape;
using namespace didengine;

// Every call on a device shares this array and it keeps the last call's contents.
static __device__ __align__(256) unsigned char scratch[DID_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int static_workspace(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(DID_EDEVICE, "device index out of range for the static workspace");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(DID_EDEVICE, std::string("hipGetSymbolAddress of the static workspace: ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return DID_OK;
}

// Bump allocator over the static workspace (base == nullptr: only counts bytes).
struct Carve {
  unsigned char* base;
  int64_t off = 0;
  template <class T>
  T* take(int64_t count) {
    const int64_t bytes = ((std::max<int64_t>(count, 1) * (int64_t)sizeof(T)) + 255) / 256 * 256;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += bytes;
    return p;
  }
};

// Lay the buffers of one MFMA-path instance out in the workspace; returns the bytes used.
int64_t carve_static(did_ctx& c, unsigned char* base, int64_t R) {
  const Shape& s = c.s;
  Carve w{base};
  const int NP = didk::n_pairs(s.KP);
  c.Bq = w.take<_Float16>(didk::packed_b_elems(s));
  c.Bsc = w.take<float>(didk::bsc_floats(s.KP));
  c.G = w.take<double>((int64_t)s.KP * s.KP);
  c.Gpart = w.take<double>((int64_t)didk::bupdate_blocks(s) * NP);
  c.V = w.take<double>((int64_t)s.KP * s.KP);
  c.W = w.take<double>((int64_t)s.KP * s.Mpad);
  c.Vpart = w.take<double>(didk::vgram_blocks(s) * NP);
  c.H = w.take<float>((int64_t)s.KP * s.N);
  c.Cq = w.take<unsigned char>(didk::cq_bytes(s));
  c.Csc = w.take<float>(didk::bsc_floats(s.KP));
  c.Wpart = w.take<float>(R * s.KP * s.Mpad);
  c.rbounds = w.take<int64_t>(R + 1);
  c.fpart = w.take<double>(didk::colpass_blocks(s));
  c.fobj = w.take<double>(1);  // objective slot when the caller passes no f
  c.tdev = w.take<int64_t>(1);  // device iteration counter (index into the history)
  return w.off;
}

}  // namespace

extern "C" {

int did_iterate_static(const float* X, int64_t M, int64_t N, int32_t K, float* B, float* C, int32_t n,
                       const did_opts* opts, double* f) {
  if (!X || !B || !C) return fail(DID_EINVAL, "X, B and C must not be NULL");
  if (n < 0) return fail(DID_EINVAL, "n must be >= 0");
  int rc = check_shape(M, N, K);
  if (rc) return rc;
  did_opts o;
  did_default_opts(&o);
  if (opts) o = *opts;
  if (o.x_dtype != DID_F32 || o.x_tiled != 0 || o.algorithm != DID_ALG_DID || o.refresh_every != 1)
    return fail(DID_EINVAL,
                "did_iterate_static takes float32 X read as given (x_dtype DID_F32, x_tiled 0, DID_ALG_DID, refresh_every 1)");
  did_ctx c;
  if ((rc = make_shape(c.s, M, N, K, o))) return rc;
  if (c.s.thin) return fail(DID_EINVAL, "did_iterate_static runs the MFMA path only (not M <= 16, K <= 8 shapes)");
  int64_t T, P, S;
  range_params(N, c.s.nchunks, o.n_blocks, row_target(c.s, o), &T, &P, &S);
  const int64_t R = didk::range_bounds(T, P, S, nullptr);
  const int64_t need = carve_static(c, nullptr, R);
  if (need > (int64_t)DID_STATIC_SCRATCH_BYTES)
    return fail(DID_EINVAL, "instance needs " + std::to_string(need) + " bytes of workspace, more than the static " +
                                std::to_string((int64_t)DID_STATIC_SCRATCH_BYTES) +
                                " (fewer row-pass ranges, opts.row_blocks, or a smaller N)");
  if (hipGetDevice(&c.dev) != hipSuccess) return fail(DID_EDEVICE, "no HIP device");
  unsigned char* base = nullptr;
  if ((rc = static_workspace(c.dev, &base))) return rc;
  (void)carve_static(c, base, R);
  c.st = static_cast<hipStream_t>(o.stream);
  c.own_stream = false;
  c.use_graph = false;  // a graph would allocate
  c.may_create_st2 = false;
  c.X = const_cast<float*>(X);
  c.XR = c.X;
  c.s.vec4 = (M % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  c.B = B;
  c.C = C;
  c.R = (int)R;
  c.fhist = f ? f : c.fobj;
  c.hist_cap = f ? std::max<int64_t>(n, 1) : 1;
  const Shape& s = c.s;
  hipError_t e;
  // the workspace keeps the last call's contents: clear the zero-padded packed operands
  // and the maxima (fill kernels, no memset nodes, so that the call can be captured)
  if ((e = didk::zero16(c.Bq, didk::packed_b_elems(s) * 2, c.st)) != hipSuccess ||
      (e = didk::zero16(c.Cq, didk::cq_bytes(s), c.st)) != hipSuccess ||
      (e = didk::zero16(c.Bsc, (int64_t)didk::bsc_floats(s.KP) * 4, c.st)) != hipSuccess ||
      (e = didk::zero16(c.Csc, (int64_t)didk::bsc_floats(s.KP) * 4, c.st)) != hipSuccess ||
      (e = didk::zero16(c.V, (int64_t)s.KP * s.KP * 8, c.st)) != hipSuccess ||
      (e = didk::zero16(c.W, (int64_t)s.KP * s.Mpad * 8, c.st)) != hipSuccess ||
      (e = didk::ranges_on_device(c.rbounds, T, P, S, c.st)) != hipSuccess ||
      (e = didk::set_i64(c.tdev, 0, c.st)) != hipSuccess ||
      (e = refresh_b_derived(&c)) != hipSuccess || (e = pack_c(&c)) != hipSuccess)
    return dev_fail(nullptr, e, "did_iterate_static setup");
  rc = iterate_mfma(&c, n);
  if (rc) return rc;
  g_err.clear();
  return DID_OK;
}


}  // extern "C"
