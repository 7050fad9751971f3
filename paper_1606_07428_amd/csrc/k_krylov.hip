// GMRES building blocks in float64 (§3.2): classical Gram-Schmidt dot products and
// updates (applied twice, CGS2), Givens rotations of the Hessenberg column, and the
// triangular solve.  Reductions are two-stage with a fixed order (deterministic).
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

hipError_t launch_dots_final(int kk, int nblk, const double* partial, double* h, double* hacc,
                             hipStream_t st) {
  k_dots_final<<<kk, 256, 0, st>>>(nblk, partial, h, hacc, 0);
  return hipGetLastError();
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

// y = x * s (or x / s if invert; 0 if s == 0)
__global__ void k_scale_copy(size_t len, const double* x, const double* s, int invert, double* y) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const double sv = *s;
  double f = sv;
  if (invert) f = sv != 0.0 ? 1.0 / sv : 0.0;
  y[e] = x[e] * f;
}

hipError_t launch_scale_copy(size_t len, const double* x, const double* s, int invert, double* y,
                             hipStream_t st) {
  k_scale_copy<<<(unsigned)((len + 255) / 256), 256, 0, st>>>(len, x, s, invert, y);
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

// Column k of H (ldh rows, column-major) holds h_0..h_{k+1}; apply the previous
// rotations, form the new one, update g, write |g_{k+1}| to resid.
__global__ void k_givens(int k, int ldh, double* H, double* cs, double* sn, double* g,
                         double* resid) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double* h = H + (size_t)k * ldh;
  for (int j = 0; j < k; ++j) {
    const double t = cs[j] * h[j] + sn[j] * h[j + 1];
    h[j + 1] = -sn[j] * h[j] + cs[j] * h[j + 1];
    h[j] = t;
  }
  const double a = h[k], b = h[k + 1];
  const double den = hypot(a, b);
  const double c = den > 0.0 ? a / den : 1.0, s = den > 0.0 ? b / den : 0.0;
  cs[k] = c;
  sn[k] = s;
  h[k] = den;
  h[k + 1] = 0.0;
  g[k + 1] = -s * g[k];
  g[k] = c * g[k];
  resid[0] = fabs(g[k + 1]);
}

hipError_t launch_givens(int k, int ldh, double* H, double* cs, double* sn, double* g,
                         const double*, const double*, double* resid, hipStream_t st) {
  k_givens<<<1, 64, 0, st>>>(k, ldh, H, cs, sn, g, resid);
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
