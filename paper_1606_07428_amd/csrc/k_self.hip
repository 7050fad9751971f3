// Per-body dense operator apply (the self part of the matvec, §3.1-§3.2):
// y_body = A_{s(i)} (R_i^T x_lab) for every body i, with A column-major
// [n_shapes][3M][3M] in the body frame (rotation covariance of §3.1 applied to the
// vector, not to the operator).  Distinct shapes make this a batched GEMV bound by
// HBM bandwidth: lanes own consecutive rows, so each column read is one coalesced
// 64-row segment; four waves split the columns and are summed through LDS.
#include "common.h"
#include "kernels.h"

namespace rbm {

template <typename TM> struct AccOf { using T = float; };
template <> struct AccOf<double> { using T = double; };

__device__ __forceinline__ float load_as_f(const float* p) { return *p; }
__device__ __forceinline__ double load_as_f(const double* p) { return *p; }
__device__ __forceinline__ float load_as_f(const uint16_t* p) {
  return __uint_as_float(((uint32_t)(*p)) << 16);
}

template <typename TM>
__global__ __launch_bounds__(256) void k_self_apply(int M, int N, const int* __restrict__ sid,
                                                    const TM* __restrict__ A_all,
                                                    const double* __restrict__ Rm,
                                                    const double* __restrict__ x_lab,
                                                    double* __restrict__ y_body) {
  using TA = typename AccOf<TM>::T;
  extern __shared__ double smem[];
  const int M3 = 3 * M;
  TA* xs = reinterpret_cast<TA*>(smem);               // [3M] body-frame input
  TA* red = xs + ((M3 + 63) / 64) * 64;               // [4][64]
  const int i = blockIdx.y, tid = threadIdx.x;
  const double* R = Rm + 9 * i;
  for (int a = tid; a < M; a += 256) {
    const size_t g = (size_t)i * M + a;
    const double v0 = x_lab[g], v1 = x_lab[N + g], v2 = x_lab[2 * (size_t)N + g];
    xs[a] = (TA)(R[0] * v0 + R[3] * v1 + R[6] * v2);
    xs[M + a] = (TA)(R[1] * v0 + R[4] * v1 + R[7] * v2);
    xs[2 * M + a] = (TA)(R[2] * v0 + R[5] * v1 + R[8] * v2);
  }
  __syncthreads();
  const TM* A = A_all + (size_t)sid[i] * M3 * M3;
  const int lane = tid & 63, w = tid >> 6;
  const int row = blockIdx.x * 64 + lane;
  const int cq = (M3 + 3) / 4;
  const int c0 = w * cq, c1 = min(M3, c0 + cq);
  TA acc = 0;
  if (row < M3) {
    const TM* Ar = A + row;
    int col = c0;
    TA a1 = 0, a2 = 0, a3 = 0;
    for (; col + 4 <= c1; col += 4) {
      acc += (TA)load_as_f(Ar + (size_t)col * M3) * xs[col];
      a1 += (TA)load_as_f(Ar + (size_t)(col + 1) * M3) * xs[col + 1];
      a2 += (TA)load_as_f(Ar + (size_t)(col + 2) * M3) * xs[col + 2];
      a3 += (TA)load_as_f(Ar + (size_t)(col + 3) * M3) * xs[col + 3];
    }
    for (; col < c1; ++col) acc += (TA)load_as_f(Ar + (size_t)col * M3) * xs[col];
    acc += (a1 + a2) + a3;
  }
  red[w * 64 + lane] = acc;
  __syncthreads();
  if (w == 0 && row < M3) {
    const TA v = (red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane]);
    const int c = row / M, a = row % M;
    y_body[(size_t)c * N + (size_t)i * M + a] = (double)v;
  }
}

template <typename TM>
hipError_t launch_self_apply(int n, int M, const int* sid, const TM* A, const double* Rm,
                             const double* x_lab, double* y_body, hipStream_t st) {
  using TA = typename AccOf<TM>::T;
  const int M3 = 3 * M;
  dim3 grid((M3 + 63) / 64, n);
  const size_t lds = (((M3 + 63) / 64) * 64 + 256) * sizeof(TA);
  k_self_apply<TM><<<grid, 256, lds, st>>>(M, n * M, sid, A, Rm, x_lab, y_body);
  return hipGetLastError();
}

template hipError_t launch_self_apply<double>(int, int, const int*, const double*, const double*,
                                              const double*, double*, hipStream_t);
template hipError_t launch_self_apply<float>(int, int, const int*, const float*, const double*,
                                             const double*, double*, hipStream_t);
template hipError_t launch_self_apply<uint16_t>(int, int, const int*, const uint16_t*,
                                                const double*, const double*, double*,
                                                hipStream_t);

}  // namespace rbm
