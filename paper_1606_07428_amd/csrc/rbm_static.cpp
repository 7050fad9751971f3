// rbm_far_traction_static: the off-body traction sum of rbm_far_traction for callers that
// cannot allocate device memory.  Its scratch (packed sources, the split's partial sums,
// float32 copies of the targets) lives in a file-scope device array of fixed size instead of
// a context workspace, so the call needs no context and allocates nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/rbm.h"
#include "kernels.h"
#include "far_plan.h"

namespace rbm {
rbm_status set_last_error(rbm_status s, const char* msg);
}  // namespace rbm

using namespace rbm;

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // per GPU
constexpr int kMaxDevices = 64;

// Every GPU the library runs on holds its own copy until the process ends.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

// Device address of this device's copy of `scratch`, looked up once per device with that
// device current (the name itself is a host-side stand-in, not a device address).
rbm_status scratch_address(unsigned char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_last_error(RBM_E_DEVICE, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_last_error(RBM_E_DEVICE, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_last_error(RBM_E_DEVICE, (std::string("hipGetSymbolAddress: ") + hipGetErrorString(e)).c_str());
    g_scratch[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch[dev];
  return RBM_OK;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Bytes of scratch for N points, `split` source chunks, precision prec.
size_t scratch_bytes(size_t N, int split, int prec) {
  const size_t src = align256(N * (prec == 0 ? 64 : 32));
  const size_t part = align256((size_t)split * 3 * N * sizeof(double));
  const size_t f32 = prec == 0 ? 0 : 2 * align256(3 * N * sizeof(float));
  return src + part + f32;
}

}  // namespace

extern "C" rbm_status rbm_far_traction_static(int n_points, int M, const double* X, const double* Nrm,
                                              const double* q, const double* add, double* y, int precision,
                                              void* stream) {
  if (!X || !Nrm || !q || !y) return set_last_error(RBM_E_INVAL, "null argument");
  if (n_points < 1 || M < 1) return set_last_error(RBM_E_INVAL, "sizes must be >= 1");
  if (precision != 0 && precision != 1) return set_last_error(RBM_E_INVAL, "precision must be 0 or 1");
  const size_t N = (size_t)n_points;
  if (scratch_bytes(N, 1, precision) > kScratchBytes)
    return set_last_error(RBM_E_NOMEM, "more points than the 64 MiB static scratch holds (about 762,000 in "
                                       "float64, 838,000 in float32)");
  // the split of the context path, lowered until the partial sums fit
  int split = far_split(n_points);
  while (split > 1 && scratch_bytes(N, split, precision) > kScratchBytes) --split;
  unsigned char* base = nullptr;
  rbm_status s = scratch_address(&base);
  if (s != RBM_OK) return s;
  void* src = base;
  double* part = reinterpret_cast<double*>(base + align256(N * (precision == 0 ? 64 : 32)));
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (precision == 0) {
    if ((e = launch_pack_sources<double>(n_points, M, X, nullptr, nullptr, q, 0, nullptr, src, st)) != hipSuccess ||
        (e = launch_far<double>(0, n_points, M, X, Nrm, src, part, split, st)) != hipSuccess)
      return set_last_error(RBM_E_DEVICE, hipGetErrorString(e));
  } else {
    unsigned char* f = reinterpret_cast<unsigned char*>(part) + align256((size_t)split * 3 * N * sizeof(double));
    float* Xf = reinterpret_cast<float*>(f);
    float* Nf = reinterpret_cast<float*>(f + align256(3 * N * sizeof(float)));
    if ((e = launch_cast_f32(3 * N, X, Xf, st)) != hipSuccess || (e = launch_cast_f32(3 * N, Nrm, Nf, st)) != hipSuccess ||
        (e = launch_pack_sources<float>(n_points, M, X, nullptr, nullptr, q, 0, nullptr, src, st)) != hipSuccess ||
        (e = launch_far<float>(0, n_points, M, Xf, Nf, src, part, split, st)) != hipSuccess)
      return set_last_error(RBM_E_DEVICE, hipGetErrorString(e));
  }
  if ((e = launch_combine(n_points, M, split, part, 1.0, add, 1.0, nullptr, nullptr, 0.0, y, st)) != hipSuccess)
    return set_last_error(RBM_E_DEVICE, hipGetErrorString(e));
  return RBM_OK;
}
