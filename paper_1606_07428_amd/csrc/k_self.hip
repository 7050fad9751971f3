// Per-body dense operator apply (the self part of the matvec, §3.1-§3.2):
// y_body = A_{s(i)} (R_i^T x_lab) for every body i, with A column-major
// [n_shapes][3M][3M] in the body frame (rotation covariance of §3.1 applied to the
// vector, not to the operator).  Distinct shapes make this a batched GEMV bound by
// HBM bandwidth: lanes own consecutive rows, so each column read is one coalesced
// segment of 64 lanes' rows; four waves split the columns and are summed through LDS.
#include "common.h"
#include "kernels.h"

namespace rbm {

template <typename TM> struct AccOf { using T = float; };
template <> struct AccOf<double> { using T = double; };

__device__ __forceinline__ float as_f(float v) { return v; }
__device__ __forceinline__ double as_f(double v) { return v; }
__device__ __forceinline__ float as_f(uint16_t v) { return __uint_as_float(((uint32_t)v) << 16); }

// RPL consecutive matrix entries of one column, read as one vector load (RPL * sizeof(TM)
// bytes, aligned because 3M and the lane's first row are multiples of RPL).
template <typename TM, int RPL> struct alignas(RPL * sizeof(TM)) RowVec { TM v[RPL]; };

// Lanes own RPL consecutive rows each (one row in float64, where a lane's 8-byte loads
// already stream at the HBM rate; 2 or 4 in float32 and bf16, whose 4- and 2-byte
// loads would otherwise leave too few bytes in flight per wave).  WAVES waves split the
// columns.  The float64 blocks are read once per apply and do not fit in the 256 MB
// Infinity Cache at the sizes where this kernel matters, so they are loaded
// non-temporally (NT) with 16 waves per workgroup: 77.7 -> 75.4 us at 64 bodies x 936
// rows, 154 -> 134 us at 1000 x 336.
template <typename TM, int RPL, int WAVES, bool NT>
__global__ __launch_bounds__(64 * WAVES) void k_self_apply(int M, int N, const int* __restrict__ sid,
                                                           const TM* __restrict__ A_all,
                                                           const double* __restrict__ Rm,
                                                           const double* __restrict__ x_lab,
                                                           double* __restrict__ y_body) {
  using TA = typename AccOf<TM>::T;
  using V = RowVec<TM, RPL>;
  extern __shared__ double smem[];
  const int M3 = 3 * M;
  TA* xs = reinterpret_cast<TA*>(smem);               // [3M] body-frame input
  TA* red = xs + ((M3 + 63) / 64) * 64;               // [WAVES][64 RPL]
  const int i = blockIdx.y, tid = threadIdx.x;
  const double* R = Rm + 9 * i;
  for (int a = tid; a < M; a += 64 * WAVES) {
    const size_t g = (size_t)i * M + a;
    const double v0 = x_lab[g], v1 = x_lab[N + g], v2 = x_lab[2 * (size_t)N + g];
    xs[a] = (TA)(R[0] * v0 + R[3] * v1 + R[6] * v2);
    xs[M + a] = (TA)(R[1] * v0 + R[4] * v1 + R[7] * v2);
    xs[2 * M + a] = (TA)(R[2] * v0 + R[5] * v1 + R[8] * v2);
  }
  __syncthreads();
  const TM* A = A_all + (size_t)sid[i] * M3 * M3;
  const int lane = tid & 63, w = tid >> 6;
  const int row = (blockIdx.x * 64 + lane) * RPL;
  const int cq = (M3 + WAVES - 1) / WAVES;
  const int c0 = w * cq, c1 = min(M3, c0 + cq);
  TA acc[4][RPL];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int r = 0; r < RPL; ++r) acc[u][r] = 0;
  auto load = [&](const TM* p) -> V {
    if constexpr (NT && RPL == 1) {
      V v;
      v.v[0] = __builtin_nontemporal_load(p);
      return v;
    } else if constexpr (NT) {
      typedef TM VT __attribute__((ext_vector_type(RPL)));
      const VT x = __builtin_nontemporal_load(reinterpret_cast<const VT*>(p));
      V v;
#pragma unroll
      for (int r = 0; r < RPL; ++r) v.v[r] = x[r];
      return v;
    } else {
      return *reinterpret_cast<const V*>(p);
    }
  };
  if (row < M3) {
    const TM* Ar = A + row;
    int col = c0;
    for (; col + 4 <= c1; col += 4) {
      V a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = load(Ar + (size_t)(col + u) * M3);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int r = 0; r < RPL; ++r) acc[u][r] += (TA)as_f(a[u].v[r]) * xs[col + u];
    }
    for (; col < c1; ++col) {
      const V a = load(Ar + (size_t)col * M3);
#pragma unroll
      for (int r = 0; r < RPL; ++r) acc[0][r] += (TA)as_f(a.v[r]) * xs[col];
    }
  }
#pragma unroll
  for (int r = 0; r < RPL; ++r)
    red[w * 64 * RPL + lane * RPL + r] = (acc[0][r] + acc[1][r]) + (acc[2][r] + acc[3][r]);
  __syncthreads();
  if (w == 0 && row < M3) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int q = lane * RPL + r;
      TA v = 0;
      for (int ww = 0; ww < WAVES; ++ww) v += red[ww * 64 * RPL + q];
      const int c = (row + r) / M, a = (row + r) % M;
      y_body[(size_t)c * N + (size_t)i * M + a] = (double)v;
    }
  }
}

template <typename TM, int RPL, int WAVES, bool NT>
static hipError_t self_apply_rpl(int n, int M, const int* sid, const TM* A, const double* Rm,
                                 const double* x_lab, double* y_body, hipStream_t st) {
  using TA = typename AccOf<TM>::T;
  const int M3 = 3 * M;
  dim3 grid((M3 + 64 * RPL - 1) / (64 * RPL), n);
  const size_t lds = (((M3 + 63) / 64) * 64 + 64 * WAVES * RPL) * sizeof(TA);
  k_self_apply<TM, RPL, WAVES, NT><<<grid, 64 * WAVES, lds, st>>>(M, n * M, sid, A, Rm, x_lab, y_body);
  return hipGetLastError();
}

template <typename TM>
hipError_t launch_self_apply(int n, int M, const int* sid, const TM* A, const double* Rm,
                             const double* x_lab, double* y_body, hipStream_t st) {
  const int M3 = 3 * M;
  if constexpr (sizeof(TM) == 8) {
    return self_apply_rpl<TM, 1, 16, true>(n, M, sid, A, Rm, x_lab, y_body, st);
  } else {
    // blocks beyond the 256 MB Infinity Cache are streamed once per apply: non-temporal loads
    // and 8 waves per workgroup (4000 bodies x 936 rows in float32: 7 % less time per apply)
    const bool stream = (double)n * M3 * M3 * sizeof(TM) > 256.0 * (1 << 20);
    if (M3 % 4 == 0 && M3 >= 768) {
      if (stream) return self_apply_rpl<TM, 4, 8, true>(n, M, sid, A, Rm, x_lab, y_body, st);
      return self_apply_rpl<TM, 4, 4, false>(n, M, sid, A, Rm, x_lab, y_body, st);
    }
    if (M3 % 2 == 0) return self_apply_rpl<TM, 2, 4, false>(n, M, sid, A, Rm, x_lab, y_body, st);
    return self_apply_rpl<TM, 1, 4, false>(n, M, sid, A, Rm, x_lab, y_body, st);
  }
}

template hipError_t launch_self_apply<double>(int, int, const int*, const double*, const double*,
                                              const double*, double*, hipStream_t);
template hipError_t launch_self_apply<float>(int, int, const int*, const float*, const double*,
                                             const double*, double*, hipStream_t);
template hipError_t launch_self_apply<uint16_t>(int, int, const int*, const uint16_t*,
                                                const double*, const double*, double*,
                                                hipStream_t);

}  // namespace rbm

namespace rbm {

// ---- one shape shared by every body: the self apply is a GEMM ------------------------
// Z (3M x n) = A (3M x 3M, column-major) . B (3M x n),  B[:, i] = R_i^T x_i (body frame),
// on MFMA: v_mfma_f64_16x16x4_f64 (float64) or v_mfma_f32_16x16x4_f32 (float32).  A 64x64
// output tile per workgroup (4 waves of 32x32 = 2x2 MFMA tiles), K staged by 16 through
// LDS.  Operand layout (16x16x4): lane l holds A[l%16][l/16] and B[l/16][l%16]; it
// receives D[4(l/16)+e][l%16] from the f32 instruction but D[(l/16)+4e][l%16] from the
// f64 one (e = 0..3; both measured on gfx950 with a known product).

// B[i*3M + c*M + a] = (R_i^T x_lab)[c] at node a, in the GEMM's operand type
template <typename TB>
__global__ void k_rotate_in(int n, int M, const double* __restrict__ Rm,
                            const double* __restrict__ x_lab, TB* __restrict__ B) {
  const size_t N = (size_t)n * M;
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int i = (int)(g / M), a = (int)(g % M);
  const double* R = Rm + 9 * i;
  const double v0 = x_lab[g], v1 = x_lab[N + g], v2 = x_lab[2 * N + g];
  TB* o = B + (size_t)i * 3 * M;
  o[a] = (TB)(R[0] * v0 + R[3] * v1 + R[6] * v2);
  o[M + a] = (TB)(R[1] * v0 + R[4] * v1 + R[7] * v2);
  o[2 * M + a] = (TB)(R[2] * v0 + R[5] * v1 + R[8] * v2);
}

__global__ void k_rotate_in_bf16(int n, int M, const double* __restrict__ Rm,
                                 const double* __restrict__ x_lab, uint16_t* __restrict__ B) {
  const size_t N = (size_t)n * M;
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int i = (int)(g / M), a = (int)(g % M);
  const double* R = Rm + 9 * i;
  const double v0 = x_lab[g], v1 = x_lab[N + g], v2 = x_lab[2 * N + g];
  uint16_t* o = B + (size_t)i * 3 * M;
  const double b[3] = {R[0] * v0 + R[3] * v1 + R[6] * v2, R[1] * v0 + R[4] * v1 + R[7] * v2,
                       R[2] * v0 + R[5] * v1 + R[8] * v2};
  for (int c = 0; c < 3; ++c) {
    uint32_t u = __float_as_uint((float)b[c]);
    u += 0x7fffu + ((u >> 16) & 1u);
    o[c * M + a] = (uint16_t)(u >> 16);
  }
}

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v_ __attribute__((ext_vector_type(4)));

template <typename T> struct MfmaAcc;
template <> struct MfmaAcc<double> {
  using V = d4v;
  __device__ static V mfma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lk, int e) { return lk + 4 * e; }
};
template <> struct MfmaAcc<float> {
  using V = f4v_;
  __device__ static V mfma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lk, int e) { return 4 * lk + e; }
};

// y_body[(row/M)*N + i*M + row%M] = Z[row][i], Z = A B (A: 3M x 3M column-major, B: one body
// per column).  Tiles of 64 rows x 32 bodies, 832 workgroups at 1000 bodies and p = 16 (64 x 64
// tiles left 416 for 256 CUs); four waves of 32 x 16; K staged by 32 through LDS, the next
// slice loaded into registers while the MFMAs use the current one.
template <typename T>
__global__ __launch_bounds__(256) void k_self_gemm(int M3, int n, int M, const T* __restrict__ A,
                                                   const T* __restrict__ B,
                                                   double* __restrict__ y_body) {
  constexpr int BM = 64, BN = 32, BK = 32;
  __shared__ T As[BM][BK + 1];
  __shared__ T Bs[BK][BN + 1];
  using V = typename MfmaAcc<T>::V;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int bm = blockIdx.y * BM, bn = blockIdx.x * BN;
  const int wr = (wid >> 1) * 32, wc = (wid & 1) * 16;
  V acc[2];
  for (int a = 0; a < 2; ++a)
    for (int e = 0; e < 4; ++e) acc[a][e] = 0;
  const int lr = lane & 15, lk = lane >> 4;
  // slice elements of this thread: A (BM x BK) e = tid + 256 u, row e % BM (consecutive rows
  // contiguous in the column-major A); B (BK x BN) e = tid + 256 u, k e % BK (one body's k
  // contiguous)
  constexpr int UA = BM * BK / 256, UB = BK * BN / 256;
  T ra[UA], rb[UB];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      const int e = tid + 256 * u, r = e % BM, kk = e / BM;
      const int gi = bm + r, gk = k0 + kk;
      ra[u] = (gi < M3 && gk < M3) ? A[(size_t)gk * M3 + gi] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int e = tid + 256 * u, kk = e % BK, c = e / BK;
      const int gk = k0 + kk, gj = bn + c;
      rb[u] = (gk < M3 && gj < n) ? B[(size_t)gj * M3 + gk] : (T)0;
    }
  };
  load(0);
  for (int k0 = 0; k0 < M3; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      const int e = tid + 256 * u;
      As[e % BM][e / BM] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int e = tid + 256 * u;
      Bs[e % BK][e / BK] = rb[u];
    }
    __syncthreads();
    if (k0 + BK < M3) load(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const T bv = Bs[ks + lk][wc + lr];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti) acc[ti] = MfmaAcc<T>::mfma(As[wr + ti * 16 + lr][ks + lk], bv, acc[ti]);
    }
  }
  const size_t N = (size_t)n * M;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = bm + wr + ti * 16 + MfmaAcc<T>::row(lk, e), i = bn + wc + lr;
      if (row < M3 && i < n)
        y_body[(size_t)(row / M) * N + (size_t)i * M + row % M] = (double)acc[ti][e];
    }
}

// scatter of a float32 (3M x n, row-major [row][i]) product into y_body
__global__ void k_scatter_f32(int M3, int n, int M, const float* __restrict__ Z,
                              double* __restrict__ y_body) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)M3 * n) return;
  const int row = (int)(e / n), i = (int)(e % n);
  const size_t N = (size_t)n * M;
  y_body[(size_t)(row / M) * N + (size_t)i * M + row % M] = (double)Z[e];
}

template <typename TM>
hipError_t launch_self_apply_shared(int n, int M, const TM* A, const double* Rm,
                                    const double* x_lab, void* scratchB, void* scratchZ,
                                    double* y_body, hipStream_t st) {
  const int M3 = 3 * M;
  const size_t N = (size_t)n * M;
  const unsigned gblocks = (unsigned)((N + 255) / 256);
  if constexpr (sizeof(TM) == 2) {
    uint16_t* B = reinterpret_cast<uint16_t*>(scratchB);
    float* Z = reinterpret_cast<float*>(scratchZ);
    k_rotate_in_bf16<<<gblocks, 256, 0, st>>>(n, M, Rm, x_lab, B);
    // Z[row][i] = sum_k A[k*M3 + row] B[i*M3 + k]
    hipError_t e = launch_gemm_bf16(M3, n, M3, reinterpret_cast<const uint16_t*>(A), 1, M3, B, 1,
                                    M3, Z, n, nullptr, 1.f, 0.f, st);
    if (e != hipSuccess) return e;
    k_scatter_f32<<<(unsigned)(((size_t)M3 * n + 255) / 256), 256, 0, st>>>(M3, n, M, Z, y_body);
  } else {
    TM* B = reinterpret_cast<TM*>(scratchB);
    k_rotate_in<TM><<<gblocks, 256, 0, st>>>(n, M, Rm, x_lab, B);
    dim3 grid((n + 31) / 32, (M3 + 63) / 64);
    k_self_gemm<TM><<<grid, 256, 0, st>>>(M3, n, M, A, B, y_body);
  }
  return hipGetLastError();
}

template hipError_t launch_self_apply_shared<double>(int, int, const double*, const double*,
                                                     const double*, void*, void*, double*,
                                                     hipStream_t);
template hipError_t launch_self_apply_shared<float>(int, int, const float*, const double*,
                                                    const double*, void*, void*, double*,
                                                    hipStream_t);
template hipError_t launch_self_apply_shared<uint16_t>(int, int, const uint16_t*, const double*,
                                                       const double*, void*, void*, double*,
                                                       hipStream_t);

}  // namespace rbm
