// GMRES building blocks in float64 (§3.2): classical Gram-Schmidt dot products and
// updates (applied twice, CGS2), Givens rotations of the Hessenberg column, and the
// triangular solve.  Reductions are two-stage with a fixed order (deterministic).
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace rbm {

// partial[j*nblk + blk] = sum over the block's slice of V[j] . w, j < kk
__global__ __launch_bounds__(256) void k_dots(int kk, size_t len, const double* __restrict__ V,
                                              size_t ldv, const double* __restrict__ w,
                                              double* __restrict__ partial, int nblk) {
  __shared__ double red[4];
  const size_t stride = (size_t)nblk * 256;
  for (int j = 0; j < kk; ++j) {
    const double* v = V + (size_t)j * ldv;
    double acc = 0.0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < len; e += stride) acc += v[e] * w[e];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[(size_t)j * nblk + blockIdx.x] = s;
  }
}

hipError_t launch_dots(int kk, size_t len, const double* V, size_t ldv, const double* w,
                       double* partial, int nblk, hipStream_t st) {
  k_dots<<<nblk, 256, 0, st>>>(kk, len, V, ldv, w, partial, nblk);
  return hipGetLastError();
}

// h[j] = sum_blk partial (fixed order); optional hacc[j] += h[j]; take_sqrt -> h = sqrt(h)
__global__ __launch_bounds__(256) void k_dots_final(int nblk, const double* partial, double* h,
                                                    double* hacc, int take_sqrt) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) acc += partial[(size_t)j * nblk + b];
  double s = block_sum(acc, red);
  if (threadIdx.x == 0) {
    if (take_sqrt) s = sqrt(s);
    if (h) h[j] = s;
    if (hacc) hacc[j] += s;
  }
}

hipError_t launch_dots_final_sqrt(int nblk, const double* partial, double* h, hipStream_t st) {
  k_dots_final<<<1, 256, 0, st>>>(nblk, partial, h, nullptr, 1);
  return hipGetLastError();
}

// w -= sum_j V[j] h[j]   or   w = sum_j V[j] h[j]
__global__ void k_vupdate(int kk, size_t len, const double* __restrict__ V, size_t ldv,
                          const double* __restrict__ h, double* __restrict__ w, int overwrite) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double acc = 0.0;
  for (int j = 0; j < kk; ++j) acc += V[(size_t)j * ldv + e] * h[j];
  w[e] = overwrite ? acc : w[e] - acc;
}

hipError_t launch_vupdate(int kk, size_t len, const double* V, size_t ldv, const double* h,
                          double* w, int overwrite, hipStream_t st) {
  k_vupdate<<<(unsigned)((len + 255) / 256), 256, 0, st>>>(kk, len, V, ldv, h, w, overwrite);
  return hipGetLastError();
}

__global__ void k_axpby(size_t len, double a, const double* x, double b, const double* y,
                        double* out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  out[e] = a * x[e] + (y ? b * y[e] : 0.0);
}

hipError_t launch_axpby(size_t len, double a, const double* x, double b, const double* y,
                        double* out, hipStream_t st) {
  k_axpby<<<(unsigned)((len + 255) / 256), 256, 0, st>>>(len, a, x, b, y, out);
  return hipGetLastError();
}

// Start of a GMRES cycle: V0 = r / rnorm (0 if rnorm = 0), g = (rnorm, 0, ..., 0) over ng
// entries, H = 0 over nh entries; one launch in place of two fills, a copy and a scale.
__global__ void k_gmres_init(size_t len, const double* __restrict__ r, double rnorm,
                             double* __restrict__ V0, int ng, double* __restrict__ g, size_t nh,
                             double* __restrict__ H) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double f = rnorm != 0.0 ? 1.0 / rnorm : 0.0;
  for (size_t e = i0; e < len; e += stride) V0[e] = r[e] * f;
  for (size_t e = i0; e < nh; e += stride) H[e] = 0.0;
  for (size_t e = i0; e < (size_t)ng; e += stride) g[e] = e == 0 ? rnorm : 0.0;
}

hipError_t launch_gmres_init(size_t len, const double* r, double rnorm, double* V0, int ng, double* g,
                             size_t nh, double* H, hipStream_t st) {
  const size_t n = std::max(len, nh);
  k_gmres_init<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(len, r, rnorm, V0, ng, g, nh, H);
  return hipGetLastError();
}

// ---- fused Arnoldi step ------------------------------------------------------------
// The Gram-Schmidt tail of one GMRES iteration in four launches instead of eleven.  Each
// kernel writes per-block partial sums, and every block of the next kernel sums all of
// them itself in the same fixed order (kk x nblk values from L2), so no kernel waits on
// another block and every block holds the same sums.  Block 0 alone writes the
// Hessenberg column and the rotation state, which no other block reads in the same
// launch.  Partial buffers: P1 and P2 hold kk x nblk sums, P3 nblk.

// hs[j] = sum over b of P[j * nblk + b], j < kk, in a fixed order: wave j mod 4 takes row
// j, lane l sums b = l, l + 64, ..., then a butterfly over the wave.
__device__ __forceinline__ void sum_partial_rows(int kk, const double* P, int nblk, double* hs) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = wv; j < kk; j += 4) {
    double a = 0.0;
    for (int b = lane; b < nblk; b += 64) a += P[(size_t)j * nblk + b];
    a = wave_sum(a);
    if (lane == 0) hs[j] = a;
  }
  __syncthreads();
}

// P1[j][blk] = block's part of V[j] . w, j < kk.
__global__ __launch_bounds__(256) void k_arnoldi_dots(int kk, size_t len, const double* __restrict__ V,
                                                      size_t ldv, const double* __restrict__ w,
                                                      double* __restrict__ P1, int nblk) {
  __shared__ double red[4];
  const size_t stride = (size_t)nblk * 256;
  for (int j = 0; j < kk; ++j) {
    const double* v = V + (size_t)j * ldv;
    double acc = 0.0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < len; e += stride) acc += v[e] * w[e];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) P1[(size_t)j * nblk + blockIdx.x] = s;
  }
}

// h = sums of P1 (into hcol by block 0); w -= V h; P2 = block parts of V^T w.
__global__ __launch_bounds__(256) void k_arnoldi_update_dots(int kk, size_t len,
                                                             const double* __restrict__ V, size_t ldv,
                                                             const double* __restrict__ P1,
                                                             double* __restrict__ P2, int nblk,
                                                             double* __restrict__ hcol,
                                                             double* __restrict__ w) {
  extern __shared__ double hs[];
  __shared__ double red[4];
  sum_partial_rows(kk, P1, nblk, hs);
  if (blockIdx.x == 0)
    for (int j = threadIdx.x; j < kk; j += 256) hcol[j] = hs[j];
  const size_t stride = (size_t)nblk * 256;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < len; e += stride) {
    double acc = 0.0;
    for (int j = 0; j < kk; ++j) acc += V[(size_t)j * ldv + e] * hs[j];
    w[e] -= acc;
  }
  for (int j = 0; j < kk; ++j) {
    const double* v = V + (size_t)j * ldv;
    double acc = 0.0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < len; e += stride) acc += v[e] * w[e];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) P2[(size_t)j * nblk + blockIdx.x] = s;
  }
}

// h2 = sums of P2 (added to hcol by block 0); w -= V h2; P3 = block parts of w . w.
__global__ __launch_bounds__(256) void k_arnoldi_update_norm(int kk, size_t len,
                                                             const double* __restrict__ V, size_t ldv,
                                                             const double* __restrict__ P2,
                                                             double* __restrict__ P3, int nblk,
                                                             double* __restrict__ hcol,
                                                             double* __restrict__ w) {
  extern __shared__ double hs[];
  __shared__ double red[4];
  sum_partial_rows(kk, P2, nblk, hs);
  if (blockIdx.x == 0)
    for (int j = threadIdx.x; j < kk; j += 256) hcol[j] += hs[j];
  const size_t stride = (size_t)nblk * 256;
  double acc2 = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < len; e += stride) {
    double acc = 0.0;
    for (int j = 0; j < kk; ++j) acc += V[(size_t)j * ldv + e] * hs[j];
    const double v = w[e] - acc;
    w[e] = v;
    acc2 += v * v;
  }
  const double s = block_sum(acc2, red);
  if (threadIdx.x == 0) P3[blockIdx.x] = s;
}

// ||w|| = sqrt(sum of P3); w /= ||w|| (0 if ||w|| = 0); block 0: ||w|| into column k
// of H, previous rotations and a new one on that column, g updated, |g_{k+1}| to resid.
__global__ __launch_bounds__(256) void k_arnoldi_normalize(size_t len, const double* __restrict__ P3,
                                                           int nblk, double* __restrict__ w, int k,
                                                           int ldh, double* H, double* cs, double* sn,
                                                           double* g, double* resid) {
  __shared__ double nsq;
  sum_partial_rows(1, P3, nblk, &nsq);
  const double nv = sqrt(nsq);
  const double f = nv != 0.0 ? 1.0 / nv : 0.0;
  const size_t stride = (size_t)nblk * 256;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < len; e += stride) w[e] *= f;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double* h = H + (size_t)k * ldh;
    h[k + 1] = nv;
    for (int j = 0; j < k; ++j) {
      const double u = cs[j] * h[j] + sn[j] * h[j + 1];
      h[j + 1] = -sn[j] * h[j] + cs[j] * h[j + 1];
      h[j] = u;
    }
    const double p = h[k], q = h[k + 1];
    const double den = hypot(p, q);
    const double c = den > 0.0 ? p / den : 1.0, sv = den > 0.0 ? q / den : 0.0;
    cs[k] = c;
    sn[k] = sv;
    h[k] = den;
    h[k + 1] = 0.0;
    g[k + 1] = -sv * g[k];
    g[k] = c * g[k];
    resid[0] = fabs(g[k + 1]);
  }
}

hipError_t launch_arnoldi(int k, size_t len, double* V, size_t ldv, double* partial, size_t pstride,
                          int nblk, int ldh, double* H, double* cs, double* sn, double* g,
                          double* resid, hipStream_t st) {
  const int kk = k + 1;
  double* w = V + (size_t)kk * ldv;
  double* hcol = H + (size_t)k * ldh;
  double *P1 = partial, *P2 = partial + pstride, *P3 = partial + 2 * pstride;
  const size_t hs = (size_t)kk * sizeof(double);
  k_arnoldi_dots<<<nblk, 256, 0, st>>>(kk, len, V, ldv, w, P1, nblk);
  k_arnoldi_update_dots<<<nblk, 256, hs, st>>>(kk, len, V, ldv, P1, P2, nblk, hcol, w);
  k_arnoldi_update_norm<<<nblk, 256, hs, st>>>(kk, len, V, ldv, P2, P3, nblk, hcol, w);
  k_arnoldi_normalize<<<nblk, 256, 0, st>>>(len, P3, nblk, w, k, ldh, H, cs, sn, g, resid);
  return hipGetLastError();
}

// Solve the m x m upper triangle of H y = g.
__global__ void k_backsolve(int m, int ldh, const double* H, const double* g, double* y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = m - 1; i >= 0; --i) {
    double v = g[i];
    for (int j = i + 1; j < m; ++j) v -= H[(size_t)j * ldh + i] * y[j];
    y[i] = v / H[(size_t)i * ldh + i];
  }
}

hipError_t launch_backsolve(int m, int ldh, const double* H, const double* g, double* y,
                            hipStream_t st) {
  k_backsolve<<<1, 64, 0, st>>>(m, ldh, H, g, y);
  return hipGetLastError();
}

}  // namespace rbm
