// Learned GMRES warm start: per-body features, band synthesis/analysis of the density
// correction, and a small MLP trained and run with bf16 MFMA (fp32 accumulation).
#include "common.h"
#include "kernels.h"

namespace rbm {

typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite values)
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// C(i,j) = alpha * sum_kk A(i,kk) B(kk,j) + bias[j] + beta * C(i,j);  A(i,kk) = A[i*sa0 + kk*sa1],
// B(kk,j) = B[kk*sb0 + j*sb1], bf16 operands, fp32 accumulation with v_mfma_f32_16x16x16_bf16.
// 64x64 output tile per workgroup, 4 waves of 32x32 (2x2 MFMA tiles), K staged by 16 in LDS.
// MFMA operand layout (16x16x16): lane l holds A[l%16][4(l/16)+j] and B[4(l/16)+j][l%16],
// j = 0..3, and receives D[4(l/16)+e][l%16], e = 0..3.
__global__ __launch_bounds__(256) void k_gemm_bf16(int m, int n, int k, const uint16_t* __restrict__ A,
                                                   long sa0, long sa1, const uint16_t* __restrict__ B,
                                                   long sb0, long sb1, float* __restrict__ C, int ldc,
                                                   const float* __restrict__ bias, float alpha,
                                                   float beta) {
  __shared__ uint16_t As[64][20];
  __shared__ uint16_t Bs[16][68];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int bm = blockIdx.y * 64, bn = blockIdx.x * 64;
  const int wr = (wid >> 1) * 32, wc = (wid & 1) * 32;
  f4v acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = (f4v){0.f, 0.f, 0.f, 0.f};
  const int lr = lane & 15, lk = 4 * (lane >> 4);
  for (int k0 = 0; k0 < k; k0 += 16) {
    for (int e = tid; e < 1024; e += 256) {
      const int r = e >> 4, kk = e & 15;
      const int gi = bm + r, gk = k0 + kk;
      As[r][kk] = (gi < m && gk < k) ? A[(long)gi * sa0 + (long)gk * sa1] : (uint16_t)0;
    }
    for (int e = tid; e < 1024; e += 256) {
      const int kk = e >> 6, c = e & 63;
      const int gk = k0 + kk, gj = bn + c;
      Bs[kk][c] = (gk < k && gj < n) ? B[(long)gk * sb0 + (long)gj * sb1] : (uint16_t)0;
    }
    __syncthreads();
#pragma unroll
    for (int ti = 0; ti < 2; ++ti) {
      s4v av;
#pragma unroll
      for (int j = 0; j < 4; ++j) av[j] = (short)As[wr + ti * 16 + lr][lk + j];
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        s4v bv;
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = (short)Bs[lk + j][wc + tj * 16 + lr];
        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[ti][tj], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = bm + wr + ti * 16 + lk + e, j = bn + wc + tj * 16 + lr;
        if (i < m && j < n) {
          float v = alpha * acc[ti][tj][e];
          if (bias) v += bias[j];
          if (beta != 0.f) v += beta * C[(long)i * ldc + j];
          C[(long)i * ldc + j] = v;
        }
      }
}

// Few rows (the per-body network at inference, small batches): one workgroup per 16x16
// output tile, its four waves taking every fourth K step of 16 with operands read
// straight from global memory (the same MFMA layout, no LDS staging), then summed in LDS
// in wave order; a 64 x 256 product runs on 64 workgroups instead of 4 that each wait on
// every K step.
__global__ __launch_bounds__(256) void k_gemm_bf16_tile16(int m, int n, int k,
                                                          const uint16_t* __restrict__ A, long sa0,
                                                          long sa1, const uint16_t* __restrict__ B,
                                                          long sb0, long sb1, float* __restrict__ C,
                                                          int ldc, const float* __restrict__ bias,
                                                          float alpha, float beta) {
  __shared__ f4v part[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tiles_n = (n + 15) / 16;
  const int ti = blockIdx.x / tiles_n, tj = blockIdx.x - ti * tiles_n;
  const int lr = lane & 15, lk = 4 * (lane >> 4);
  const int ia = ti * 16 + lr, jb = tj * 16 + lr;
  f4v acc = (f4v){0.f, 0.f, 0.f, 0.f};
  for (int k0 = 16 * w; k0 < k; k0 += 64) {
    s4v av, bv;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = k0 + lk + j;
      av[j] = (short)((ia < m && kk < k) ? A[(long)ia * sa0 + (long)kk * sa1] : (uint16_t)0);
      bv[j] = (short)((kk < k && jb < n) ? B[(long)kk * sb0 + (long)jb * sb1] : (uint16_t)0);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
  }
  part[w][lane] = acc;
  __syncthreads();
  if (w != 0) return;
  const f4v s = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = ti * 16 + lk + e, j = jb;
    if (i < m && j < n) {
      float v = alpha * s[e];
      if (bias) v += bias[j];
      if (beta != 0.f) v += beta * C[(long)i * ldc + j];
      C[(long)i * ldc + j] = v;
    }
  }
}

hipError_t launch_gemm_bf16(int m, int n, int k, const uint16_t* A, long sa0, long sa1,
                            const uint16_t* B, long sb0, long sb1, float* C, int ldc,
                            const float* bias, float alpha, float beta, hipStream_t st) {
  // The network's products (at most a few thousand 16x16 output tiles: inference, and the
  // training batches' forward, weight-gradient and input-gradient products) take one
  // workgroup per 16x16 tile, so that even a 256 x 256 x 256 product fills 256 workgroups;
  // larger ones the 64x64-tile kernel.
  const long tiles16 = (long)((m + 15) / 16) * ((n + 15) / 16);
  if (tiles16 <= 8192) {
    const long tiles = (long)((m + 15) / 16) * ((n + 15) / 16);
    k_gemm_bf16_tile16<<<(unsigned)tiles, 256, 0, st>>>(m, n, k, A, sa0, sa1, B, sb0, sb1, C, ldc, bias,
                                                         alpha, beta);
    return hipGetLastError();
  }
  dim3 grid((n + 63) / 64, (m + 63) / 64);
  k_gemm_bf16<<<grid, 256, 0, st>>>(m, n, k, A, sa0, sa1, B, sb0, sb1, C, ldc, bias, alpha, beta);
  return hipGetLastError();
}

// H = silu(Z) (fp32 and bf16 copies)
__global__ void k_silu_fwd(size_t cnt, const float* Z, float* H, uint16_t* Hb) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const float z = Z[i];
  const float h = z / (1.f + expf(-z));
  H[i] = h;
  Hb[i] = f2bf(h);
}

hipError_t launch_silu_fwd(size_t cnt, const float* Z, float* H, uint16_t* Hb, hipStream_t st) {
  k_silu_fwd<<<(unsigned)((cnt + 255) / 256), 256, 0, st>>>(cnt, Z, H, Hb);
  return hipGetLastError();
}

// dZ = dH * silu'(Z), silu'(z) = s (1 + z (1 - s)), s = sigmoid(z)
__global__ void k_silu_bwd(size_t cnt, const float* dH, const float* Z, float* dZ, uint16_t* dZb) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const float z = Z[i];
  const float s = 1.f / (1.f + expf(-z));
  const float g = dH[i] * s * (1.f + z * (1.f - s));
  dZ[i] = g;
  dZb[i] = f2bf(g);
}

hipError_t launch_silu_bwd(size_t cnt, const float* dH, const float* Z, float* dZ, uint16_t* dZb,
                           hipStream_t st) {
  k_silu_bwd<<<(unsigned)((cnt + 255) / 256), 256, 0, st>>>(cnt, dH, Z, dZ, dZb);
  return hipGetLastError();
}

// Mean-squared error over rows x cols: dY = 2 (Y - T) / (rows cols); per-block partial
// sums of (Y - T)^2 in part[blockIdx.x].
__global__ __launch_bounds__(256) void k_mse(size_t cnt, float inv, const float* Y, const float* T,
                                             float* dY, uint16_t* dYb, double* part) {
  __shared__ double red[4];
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e2 = 0.0;
  if (i < cnt) {
    const float d = Y[i] - T[i];
    const float g = 2.f * d * inv;
    dY[i] = g;
    dYb[i] = f2bf(g);
    e2 = (double)d * d;
  }
  const double s = block_sum(e2, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

hipError_t launch_mse(size_t cnt, float inv, const float* Y, const float* T, float* dY,
                      uint16_t* dYb, double* part, hipStream_t st) {
  k_mse<<<(unsigned)((cnt + 255) / 256), 256, 0, st>>>(cnt, inv, Y, T, dY, dYb, part);
  return hipGetLastError();
}

// out[0] = scale * sum(part); with accumulate, out[1] += out[0] as well (a running sum of
// the batch losses of an epoch, read once at its end).
__global__ __launch_bounds__(256) void k_sum_parts(int nparts, const double* part, double scale,
                                                   double* out, int accumulate) {
  __shared__ double red[4];
  double a = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) a += part[i];
  const double s = block_sum(a, red);
  if (threadIdx.x == 0) {
    out[0] = s * scale;
    if (accumulate) out[1] += s * scale;
  }
}

hipError_t launch_sum_parts(int nparts, const double* part, double scale, double* out, int accumulate,
                            hipStream_t st) {
  k_sum_parts<<<1, 256, 0, st>>>(nparts, part, scale, out, accumulate);
  return hipGetLastError();
}

// db[j] = sum_i dZ[i][j] in a fixed order.  A workgroup takes 16 columns; its 256 threads
// are 16 row groups x 16 columns, row group g summing rows g, g + 16, ... (four independent
// accumulators, so eight loads of each lane are in flight), and the 16 group sums of a
// column are added in group order through LDS.
__global__ __launch_bounds__(256) void k_colsum(int rows, int cols, const float* __restrict__ dZ,
                                                float* __restrict__ db) {
  __shared__ float red[16][17];
  const int c = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int j = blockIdx.x * 16 + c;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  if (j < cols) {
    int i = g;
    for (; i + 48 < rows; i += 64) {
      a0 += dZ[(size_t)i * cols + j];
      a1 += dZ[(size_t)(i + 16) * cols + j];
      a2 += dZ[(size_t)(i + 32) * cols + j];
      a3 += dZ[(size_t)(i + 48) * cols + j];
    }
    for (; i < rows; i += 16) a0 += dZ[(size_t)i * cols + j];
  }
  red[g][c] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (g == 0 && j < cols) {
    float v = 0.f;
    for (int k = 0; k < 16; ++k) v += red[k][c];
    db[j] = v;
  }
}

hipError_t launch_colsum(int rows, int cols, const float* dZ, float* db, hipStream_t st) {
  k_colsum<<<(cols + 15) / 16, 256, 0, st>>>(rows, cols, dZ, db);
  return hipGetLastError();
}

// Adam with bias correction; fp32 master weights, optional bf16 copy.
__global__ void k_adam(size_t cnt, float* P, const float* G, float* m, float* v, float lr, float b1,
                       float b2, float eps, float c1, float c2, uint16_t* Pb) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const float g = G[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float p = P[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  P[i] = p;
  if (Pb) Pb[i] = f2bf(p);
}

hipError_t launch_adam(size_t cnt, float* P, const float* G, float* m, float* v, float lr, float b1,
                       float b2, float eps, int t, uint16_t* Pb, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  k_adam<<<(unsigned)((cnt + 255) / 256), 256, 0, st>>>(cnt, P, G, m, v, lr, b1, b2, eps, c1, c2, Pb);
  return hipGetLastError();
}

__global__ void k_to_bf16(size_t cnt, const float* x, uint16_t* y) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) y[i] = f2bf(x[i]);
}

hipError_t launch_to_bf16(size_t cnt, const float* x, uint16_t* y, hipStream_t st) {
  k_to_bf16<<<(unsigned)((cnt + 255) / 256), 256, 0, st>>>(cnt, x, y);
  return hipGetLastError();
}

// Per body i: body-frame features (own load, shape descriptor, k nearest neighbours:
// R^T d/|d|^2, first two columns of R_i^T R_j, R^T F_j, R^T T_j; zero padding).
// One wave per body.  The k nearest other bodies in (squared distance, index) order are
// picked in k rounds, each a wave-wide argmin over the pairs after the previous pick
// (the order an insertion sort over increasing j keeps, ties included); lane s then
// writes the 15 features of neighbour slot s.
__global__ __launch_bounds__(64) void k_features(int n, int k, int S, const double* cen, const double* Rm,
                                                 const double* FT, const int* sid, const double* desc,
                                                 float* X) {
  const int i = blockIdx.x, lane = threadIdx.x;
  const double ci0 = cen[3 * i], ci1 = cen[3 * i + 1], ci2 = cen[3 * i + 2];
  double pd = -1.0;
  int pj = -1, myj = -1;
  for (int s = 0; s < k; ++s) {
    double bd = 1e300;
    int bj = 0x7fffffff;
    for (int j = lane; j < n; j += 64) {
      if (j == i) continue;
      const double d0 = cen[3 * j] - ci0, d1 = cen[3 * j + 1] - ci1, d2 = cen[3 * j + 2] - ci2;
      const double dd = d0 * d0 + d1 * d1 + d2 * d2;
      const bool after = dd > pd || (dd == pd && j > pj);
      if (after && (dd < bd || (dd == bd && j < bj))) {
        bd = dd;
        bj = j;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double od = __shfl_xor(bd, o, 64);
      const int oj = __shfl_xor(bj, o, 64);
      if (od < bd || (od == bd && oj < bj)) {
        bd = od;
        bj = oj;
      }
    }
    if (bj == 0x7fffffff) break;  // fewer than k other bodies
    if (lane == s) myj = bj;
    pd = bd;
    pj = bj;
  }
  const int F = 6 + S + 15 * k;
  float* x = X + (size_t)i * F;
  const double* R = Rm + 9 * i;
  auto rt = [&](double a0, double a1, double a2, float* o) {  // R^T a
    o[0] = (float)(R[0] * a0 + R[3] * a1 + R[6] * a2);
    o[1] = (float)(R[1] * a0 + R[4] * a1 + R[7] * a2);
    o[2] = (float)(R[2] * a0 + R[5] * a1 + R[8] * a2);
  };
  if (lane == 0) {
    const double* f = FT + 6 * i;
    rt(f[0], f[1], f[2], x);
    rt(f[3], f[4], f[5], x + 3);
  }
  for (int q = lane; q < S; q += 64) x[6 + q] = (float)desc[(size_t)sid[i] * S + q];
  if (lane < k) {
    float* o = x + 6 + S + 15 * lane;
    const int j = myj;
    if (j < 0) {
      for (int e = 0; e < 15; ++e) o[e] = 0.f;
    } else {
      const double d0 = cen[3 * j] - ci0, d1 = cen[3 * j + 1] - ci1, d2 = cen[3 * j + 2] - ci2;
      const double id2 = 1.0 / (d0 * d0 + d1 * d1 + d2 * d2);
      rt(d0 * id2, d1 * id2, d2 * id2, o);
      const double* Rj = Rm + 9 * j;
      rt(Rj[0], Rj[3], Rj[6], o + 3);   // first column of R_j
      rt(Rj[1], Rj[4], Rj[7], o + 6);   // second column of R_j
      const double* fj = FT + 6 * j;
      rt(fj[0], fj[1], fj[2], o + 9);
      rt(fj[3], fj[4], fj[5], o + 12);
    }
  }
}

hipError_t launch_features(int n, int k, int S, const double* cen, const double* Rm,
                           const double* FT, const int* sid, const double* desc, float* X,
                           hipStream_t st) {
  if (k > 16) return hipErrorInvalidValue;
  if (n < 1 || k < 0) return hipErrorInvalidValue;
  k_features<<<n, 64, 0, st>>>(n, k, S, cen, Rm, FT, sid, desc, X);
  return hipGetLastError();
}

// Xb[r][f] = bf16((X[src(r)][f] - mean[f]) * istd[f]); src(r) = idx ? idx[r] : r;
// optionally Tb[r][o] = T[src(r)][o] * tinv.
__global__ void k_gather(int rows, int F, int O, const int* idx, const float* X, const float* mean,
                         const float* istd, uint16_t* Xb, const float* T, float tinv, float* Tb) {
  const int r = blockIdx.y;
  if (r >= rows) return;
  const int src = idx ? idx[r] : r;
  for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < F; f += gridDim.x * blockDim.x)
    Xb[(size_t)r * F + f] = f2bf((X[(size_t)src * F + f] - mean[f]) * istd[f]);
  if (T)
    for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < O; o += gridDim.x * blockDim.x)
      Tb[(size_t)r * O + o] = T[(size_t)src * O + o] * tinv;
}

hipError_t launch_gather(int rows, int F, int O, const int* idx, const float* X, const float* mean,
                         const float* istd, uint16_t* Xb, const float* T, float tinv, float* Tb,
                         hipStream_t st) {
  if (rows < 1) return hipSuccess;
  dim3 grid(2, rows);
  k_gather<<<grid, 256, 0, st>>>(rows, F, O, idx, X, mean, istd, Xb, T, tinv, Tb);
  return hipGetLastError();
}

// Column statistics over `rows` rows: mean[f] and 1/std[f] (0 for constant columns).
__global__ __launch_bounds__(256) void k_colstats(int rows, int F, const float* X, float* mean,
                                                  float* istd) {
  __shared__ double red[4];
  const int f = blockIdx.x;
  double a = 0.0;
  for (int r = threadIdx.x; r < rows; r += 256) a += X[(size_t)r * F + f];
  const double mu = block_sum(a, red) / rows;
  double b = 0.0;
  for (int r = threadIdx.x; r < rows; r += 256) {
    const double d = X[(size_t)r * F + f] - mu;
    b += d * d;
  }
  const double var = block_sum(b, red) / rows;
  if (threadIdx.x == 0) {
    mean[f] = (float)mu;
    istd[f] = var > 1e-20 ? (float)(1.0 / sqrt(var)) : 0.f;
  }
}

hipError_t launch_colstats(int rows, int F, const float* X, float* mean, float* istd,
                           hipStream_t st) {
  k_colstats<<<F, 256, 0, st>>>(rows, F, X, mean, istd);
  return hipGetLastError();
}

// RMS of cnt values into out[0] (as 1/rms in out[1]).
__global__ __launch_bounds__(256) void k_rms(size_t cnt, const float* T, float* out) {
  __shared__ double red[4];
  double a = 0.0;
  for (size_t i = threadIdx.x; i < cnt; i += 256) a += (double)T[i] * T[i];
  const double s = block_sum(a, red);
  if (threadIdx.x == 0) {
    const double rms = sqrt(s / (double)(cnt > 0 ? cnt : 1));
    out[0] = (float)(rms > 0 ? rms : 1.0);
    out[1] = (float)(rms > 0 ? 1.0 / rms : 1.0);
  }
}

hipError_t launch_rms(size_t cnt, const float* T, float* out, hipStream_t st) {
  k_rms<<<1, 256, 0, st>>>(cnt, T, out);
  return hipGetLastError();
}

// mu[:, body i] += scale * R_i Y_B(grid) coef_i  (band synthesis of a body-frame density)
// Four lanes per node, each summing a quarter of the band coefficients with independent
// loads in flight, joined by two butterfly steps; the first lane of the four writes.
__global__ __launch_bounds__(256) void k_band_synth(int n, int M, int p, const float* coef,
                                                    const float* scale, const double* Ytab,
                                                    const double* Rm, double* mu) {
  const size_t N = (size_t)n * M;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t g = t >> 2;
  const int q = (int)(t & 3);
  const bool act = g < N;
  const size_t gc = act ? g : 0;
  const int i = (int)(gc / M), a = (int)(gc % M);
  const int nB = p * p + 2 * p;
  const float* cf = coef + (size_t)i * 3 * nB;
  double v0 = 0, v1 = 0, v2 = 0;
  for (int b = q; b < nB; b += 4) {
    const int full = b < p * p ? b : b + 1;
    const double y = Ytab[(size_t)full * M + a];
    v0 += y * cf[b];
    v1 += y * cf[nB + b];
    v2 += y * cf[2 * nB + b];
  }
  for (int o = 1; o < 4; o <<= 1) {
    v0 += __shfl_xor(v0, o, 64);
    v1 += __shfl_xor(v1, o, 64);
    v2 += __shfl_xor(v2, o, 64);
  }
  if (!act || q != 0) return;
  const double sc = scale ? (double)scale[0] : 1.0;
  const double* R = Rm + 9 * i;
  for (int c = 0; c < 3; ++c)
    mu[c * N + g] += sc * (R[3 * c] * v0 + R[3 * c + 1] * v1 + R[3 * c + 2] * v2);
}

hipError_t launch_band_synth(int n, int M, int p, const float* coef, const float* scale,
                             const double* Ytab, const double* Rm, double* mu, hipStream_t st) {
  const size_t N = (size_t)n * M;
  k_band_synth<<<(unsigned)((4 * N + 255) / 256), 256, 0, st>>>(n, M, p, coef, scale, Ytab, Rm, mu);
  return hipGetLastError();
}

// out[i][c][b] = sum_a F[b][a] (R_i^T dmu)[c][a]  (body-frame band coefficients), fp32 out.
__global__ __launch_bounds__(256) void k_band_analysis(int n, int M, int p, const double* dmu,
                                                       const double* Rm, const double* Ftab,
                                                       float* out) {
  extern __shared__ double bodyv[];  // [3][M]
  const size_t N = (size_t)n * M;
  const int i = blockIdx.x;
  const int nB = p * p + 2 * p;
  const double* R = Rm + 9 * i;
  for (int a = threadIdx.x; a < M; a += 256) {
    const size_t g = (size_t)i * M + a;
    const double v0 = dmu[g], v1 = dmu[N + g], v2 = dmu[2 * N + g];
    bodyv[a] = R[0] * v0 + R[3] * v1 + R[6] * v2;
    bodyv[M + a] = R[1] * v0 + R[4] * v1 + R[7] * v2;
    bodyv[2 * M + a] = R[2] * v0 + R[5] * v1 + R[8] * v2;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nB; b += 256) {
    double s0 = 0, s1 = 0, s2 = 0;
    for (int a = 0; a < M; ++a) {
      const double f = Ftab[(size_t)b * M + a];
      s0 += f * bodyv[a];
      s1 += f * bodyv[M + a];
      s2 += f * bodyv[2 * M + a];
    }
    float* o = out + (size_t)i * 3 * nB;
    o[b] = (float)s0;
    o[nB + b] = (float)s1;
    o[2 * nB + b] = (float)s2;
  }
}

hipError_t launch_band_analysis(int n, int M, int p, const double* dmu, const double* Rm,
                                const double* Ftab, float* out, hipStream_t st) {
  k_band_analysis<<<n, 256, 3 * M * sizeof(double), st>>>(n, M, p, dmu, Rm, Ftab, out);
  return hipGetLastError();
}

}  // namespace rbm
