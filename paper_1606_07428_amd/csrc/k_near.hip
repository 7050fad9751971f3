// Near-singular evaluation by upsampling (§3): for a target close to another body the
// smooth rule over that body is evaluated on a finer grid of order p_u.  The geometry
// is evaluated exactly from the shape's SH coefficients at the fine nodes and the
// density by its band-limited interpolant.  This file holds the setup (fine geometry,
// bounding radii, interpolation matrix), the per-pose near list, the interpolation
// GEMM, the packing of fine sources and the correction sum, which uses the same pair
// arithmetic (pair.h) as the all-pairs sum of k_far.hip.
#include "common.h"
#include "kernels.h"
#include "pair.h"

namespace rbm {

// Fine nodes of every shape: r' = x'(s) - x^c (coarse-grid area centroid, so both grids
// place the body identically) and the smooth weights w' = (pi/p_u) lam'_j J'.  One thread
// per fine node; the shape's coordinate coefficients (degree <= p) sit in LDS.
__global__ __launch_bounds__(256) void k_fine_geometry(int p, int pu, const double* __restrict__ coef_all,
                                                       const double* __restrict__ glu_t,
                                                       const double* __restrict__ glu_w,
                                                       const double* __restrict__ shp_all,
                                                       double* __restrict__ fr_all,
                                                       double* __restrict__ fw_all) {
  extern __shared__ double cf[];  // [3][nc]
  const int nc = (p + 1) * (p + 1), Mu = (pu + 1) * 2 * pu;
  const int s = blockIdx.y;
  for (int i = threadIdx.x; i < 3 * nc; i += blockDim.x) cf[i] = coef_all[(size_t)s * 3 * nc + i];
  __syncthreads();
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= Mu) return;
  const int j = b / (2 * pu), k = b % (2 * pu);
  const double x = glu_t[j], sn = sqrt(fmax(0.0, 1.0 - x * x)), ph = RBM_PI * k / pu;
  double X[3] = {0, 0, 0}, Xt[3] = {0, 0, 0}, Xp[3] = {0, 0, 0};
  int cur_m = -1;
  double cm = 1.0, sm = 0.0;
  const double r2 = 1.41421356237309504880;
  legendre_sweep(p, x, sn, [&](int l, int m, double P, double Q, double D) {
    const int i0 = l * l + l;
    if (m == 0) {
      for (int c = 0; c < 3; ++c) {
        X[c] += cf[c * nc + i0] * P;
        Xt[c] += cf[c * nc + i0] * D;
      }
      return;
    }
    if (m != cur_m) {
      sincos(m * ph, &sm, &cm);
      cur_m = m;
    }
    // Y_{l,m} = sqrt2 P cos(m phi), Y_{l,-m} = sqrt2 P sin(m phi); (dY/dphi)/sin via Q
    for (int c = 0; c < 3; ++c) {
      const double ap = cf[c * nc + i0 + m], am = cf[c * nc + i0 - m];
      X[c] += r2 * P * (ap * cm + am * sm);
      Xt[c] += r2 * D * (ap * cm + am * sm);
      Xp[c] += r2 * m * Q * (am * cm - ap * sm);
    }
  });
  const double cx = Xt[1] * Xp[2] - Xt[2] * Xp[1];
  const double cy = Xt[2] * Xp[0] - Xt[0] * Xp[2];
  const double cz = Xt[0] * Xp[1] - Xt[1] * Xp[0];
  const double J = sqrt(cx * cx + cy * cy + cz * cz);
  const double* xc = shp_all + (size_t)s * 32 + 1;
  double* fr = fr_all + (size_t)s * 3 * Mu;
  for (int c = 0; c < 3; ++c) fr[(size_t)c * Mu + b] = X[c] - xc[c];
  fw_all[(size_t)s * Mu + b] = RBM_PI / pu * glu_w[j] * J;
}

// rb[s] = max_b |r'_b| over the fine nodes (the bounding radius of the near test).
__global__ __launch_bounds__(256) void k_bound_radius(int Mu, const double* __restrict__ fr_all,
                                                      double* __restrict__ rb) {
  __shared__ double red[4];
  const int s = blockIdx.x;
  const double* fr = fr_all + (size_t)s * 3 * Mu;
  double m = 0.0;
  for (int b = threadIdx.x; b < Mu; b += 256) {
    const double x = fr[b], y = fr[Mu + b], z = fr[2 * Mu + b];
    m = fmax(m, x * x + y * y + z * z);
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) rb[s] = sqrt(fmax(fmax(red[0], red[1]), fmax(red[2], red[3])));
}

// Interpolation matrix, column-major [M][Mu]: U[a*Mu + b] = weight of coarse node a in
// the band-limited interpolant at fine node b,
//   U = w_a sum_{(l,m) in B_p} nu_lm Y_lm(s_b) Y_lm(s_a),  w_a = (pi/p) lam_j(a).
// By the addition theorem sum_m Y_lm(s_b) Y_lm(s_a) = (2l+1)/(4pi) P_l(s_a . s_b) for the
// full degree-l space; B_p drops (p,-p) (whose sine vanishes at every coarse node) and
// halves (p,p), so U = w_a [sum_{l<=p} (2l+1)/(4pi) P_l(cos g) - Y_pp(s_b) Y_pp(s_a) / 2],
// with Y_pp = sqrt2 A_p sin^p(theta) cos(p phi), A_p^2 = (2p+1)/(4pi) prod_k (2k-1)/(2k).
__global__ __launch_bounds__(256) void k_interp_matrix(int p, int pu, const double* __restrict__ gl_t,
                                                       const double* __restrict__ gl_w,
                                                       const double* __restrict__ glu_t,
                                                       double* __restrict__ U) {
  const int M = (p + 1) * 2 * p, Mu = (pu + 1) * 2 * pu;
  const int b = blockIdx.x * blockDim.x + threadIdx.x, a = blockIdx.y;
  if (b >= Mu || a >= M) return;
  const int ja = a / (2 * p), ka = a % (2 * p), jb = b / (2 * pu), kb = b % (2 * pu);
  const double ta = gl_t[ja], tb = glu_t[jb];
  const double sa = sqrt(fmax(0.0, 1.0 - ta * ta)), sb = sqrt(fmax(0.0, 1.0 - tb * tb));
  const double dphi = RBM_PI * ka / p - RBM_PI * kb / pu;
  const double cg = ta * tb + sa * sb * cos(dphi);
  double pm1 = 1.0, p0 = cg, sum = 1.0 + 3.0 * cg;  // (2l+1) P_l for l = 0, 1
  for (int l = 2; l <= p; ++l) {
    const double pl = ((2.0 * l - 1.0) * cg * p0 - (l - 1.0) * pm1) / l;
    sum += (2.0 * l + 1.0) * pl;
    pm1 = p0;
    p0 = pl;
  }
  double A2 = (2.0 * p + 1.0) / (4.0 * RBM_PI);
  for (int k = 1; k <= p; ++k) A2 *= (2.0 * k - 1.0) / (2.0 * k);
  // Y_pp(s_b) Y_pp(s_a) / 2 = A_p^2 sin^p(a) sin^p(b) cos(p phi_b) (-1)^ka
  const double cpb = cos(p * (RBM_PI * kb / pu));
  const double nyq = A2 * pow(sa * sb, (double)p) * cpb * ((ka & 1) ? -1.0 : 1.0);
  U[(size_t)a * Mu + b] = RBM_PI / p * gl_w[ja] * (sum / (4.0 * RBM_PI) - nyq);
}

// Near list per body i: the j != i with |c_i - c_j| < rb_i + rb_j + kappa h_j, h_j =
// sqrt(|Gamma_j| / M), in increasing j.  cnt[i] is the true count; at most kmax are
// stored, the caller checks cnt against kmax.
__global__ void k_near_list(int n, int M, int kmax, double kappa, const double* __restrict__ cen,
                            const int* __restrict__ sid, const double* __restrict__ rb,
                            const double* __restrict__ shp_all, int* __restrict__ nbr,
                            int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double cx = cen[3 * i], cy = cen[3 * i + 1], cz = cen[3 * i + 2];
  const double ri = rb[sid[i]];
  int c = 0;
  for (int j = 0; j < n; ++j) {
    if (j == i) continue;
    const int sj = sid[j];
    const double dx = cx - cen[3 * j], dy = cy - cen[3 * j + 1], dz = cz - cen[3 * j + 2];
    const double d = sqrt(dx * dx + dy * dy + dz * dz);
    const double h = sqrt(shp_all[(size_t)sj * 32] / M);
    if (d < ri + rb[sj] + kappa * h) {
      if (c < kmax) nbr[(size_t)i * kmax + c] = j;
      ++c;
    }
  }
  cnt[i] = c;
}

// Fine sources: X' = c_i + R_i r'_{s(i)}, q' = w' (R_i) zt, zt = U z per component
// ([3][n*Mu]); z in body frames when z_is_body.
template <typename T>
__global__ void k_pack_fine(int n, int Mu, const int* __restrict__ sid, const double* __restrict__ cen,
                            const double* __restrict__ Rm, const double* __restrict__ fr_all,
                            const double* __restrict__ fw_all, const double* __restrict__ zt,
                            int z_is_body, Src8<T>* __restrict__ srcf) {
  const size_t Nu = (size_t)n * Mu;
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= Nu) return;
  const int i = (int)(g / Mu), b = (int)(g % Mu), s = sid[i];
  const double* R = Rm + 9 * i;
  const double* fr = fr_all + (size_t)s * 3 * Mu;
  const double r0 = fr[b], r1 = fr[Mu + b], r2 = fr[2 * (size_t)Mu + b];
  double v0 = zt[g], v1 = zt[Nu + g], v2 = zt[2 * Nu + g];
  if (z_is_body) {
    const double a0 = R[0] * v0 + R[1] * v1 + R[2] * v2;
    const double a1 = R[3] * v0 + R[4] * v1 + R[5] * v2;
    const double a2 = R[6] * v0 + R[7] * v1 + R[8] * v2;
    v0 = a0; v1 = a1; v2 = a2;
  }
  const double w = fw_all[(size_t)s * Mu + b];
  Src8<T> o;
  o.v[0] = (T)(cen[3 * i] + R[0] * r0 + R[1] * r1 + R[2] * r2);
  o.v[1] = (T)(cen[3 * i + 1] + R[3] * r0 + R[4] * r1 + R[5] * r2);
  o.v[2] = (T)(cen[3 * i + 2] + R[6] * r0 + R[7] * r1 + R[8] * r2);
  o.v[3] = (T)(w * v0);
  o.v[4] = (T)(w * v1);
  o.v[5] = (T)(w * v2);
  o.v[6] = 0;
  o.v[7] = 0;
  srcf[g] = o;
}

// C (Mr x Nc) = A (Mr x K) B (K x Nc), all column-major with leading dimensions Mr, K,
// Mr, on v_mfma_f64_16x16x4_f64: 64 x 64 tile per workgroup, 2 x 2 MFMA tiles per wave,
// K staged by 16 through LDS.  Lane l holds A[l%16][l/16] and B[l/16][l%16] and
// receives D[(l/16) + 4e][l%16] (the float64 instruction's result layout on gfx950).
typedef double d4v_n __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_gemm_f64(int Mr, int K, int Nc, const double* __restrict__ A,
                                                  const double* __restrict__ B, double* __restrict__ C) {
  __shared__ double As[64][17];
  __shared__ double Bs[16][65];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int bm = blockIdx.y * 64, bn = blockIdx.x * 64;
  const int wr = (wid >> 1) * 32, wc = (wid & 1) * 32;
  d4v_n acc[2][2];
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y)
      for (int e = 0; e < 4; ++e) acc[x][y][e] = 0.0;
  const int lr = lane & 15, lk = lane >> 4;
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = tid; e < 1024; e += 256) {
      const int r = e & 63, kk = e >> 6;
      const int gi = bm + r, gk = k0 + kk;
      As[r][kk] = (gi < Mr && gk < K) ? A[(size_t)gk * Mr + gi] : 0.0;
    }
    for (int e = tid; e < 1024; e += 256) {
      const int kk = e & 15, c = e >> 4;
      const int gk = k0 + kk, gj = bn + c;
      Bs[kk][c] = (gk < K && gj < Nc) ? B[(size_t)gj * K + gk] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
#pragma unroll
      for (int ti = 0; ti < 2; ++ti) {
        const double av = As[wr + ti * 16 + lr][ks + lk];
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Bs[ks + lk][wc + tj * 16 + lr],
                                                             acc[ti][tj], 0, 0, 0);
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
        const int row = bm + wr + ti * 16 + lk + 4 * e, col = bn + wc + tj * 16 + lr;
        if (row < Mr && col < Nc) C[(size_t)col * Mr + row] = acc[ti][tj][e];
      }
}

hipError_t launch_fine_geometry(int ns, int p, int pu, const double* coef, const double* glu_t,
                                const double* glu_w, const double* shp, double* fr, double* fw,
                                double* rb, hipStream_t st) {
  const int Mu = (pu + 1) * 2 * pu, nc = (p + 1) * (p + 1);
  dim3 grid((Mu + 255) / 256, ns);
  k_fine_geometry<<<grid, 256, 3 * nc * sizeof(double), st>>>(p, pu, coef, glu_t, glu_w, shp, fr, fw);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_bound_radius<<<ns, 256, 0, st>>>(Mu, fr, rb);
  return hipGetLastError();
}

hipError_t launch_interp_matrix(int p, int pu, const double* gl_t, const double* gl_w,
                                const double* glu_t, double* U, hipStream_t st) {
  const int M = (p + 1) * 2 * p, Mu = (pu + 1) * 2 * pu;
  dim3 grid((Mu + 255) / 256, M);
  k_interp_matrix<<<grid, 256, 0, st>>>(p, pu, gl_t, gl_w, glu_t, U);
  return hipGetLastError();
}

hipError_t launch_near_list(int n, int M, int kmax, double kappa, const double* cen, const int* sid,
                            const double* rb, const double* shp, int* nbr, int* cnt, hipStream_t st) {
  k_near_list<<<(n + 63) / 64, 64, 0, st>>>(n, M, kmax, kappa, cen, sid, rb, shp, nbr, cnt);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fine_sources(int n, int M, int Mu, const double* U, const double* z, int z_is_body,
                               const int* sid, const double* cen, const double* Rm, const double* fr,
                               const double* fw, double* zt, void* srcf, hipStream_t st) {
  // zt (Mu x 3n) = U (Mu x M) z (M x 3n): columns are (component, body) pairs
  dim3 grid((3 * n + 63) / 64, (Mu + 63) / 64);
  k_gemm_f64<<<grid, 256, 0, st>>>(Mu, M, 3 * n, U, z, zt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t Nu = (size_t)n * Mu;
  k_pack_fine<T><<<(unsigned)((Nu + 255) / 256), 256, 0, st>>>(n, Mu, sid, cen, Rm, fr, fw, zt, z_is_body,
                                                                reinterpret_cast<Src8<T>*>(srcf));
  return hipGetLastError();
}

template hipError_t launch_fine_sources<double>(int, int, int, const double*, const double*, int,
                                                const int*, const double*, const double*,
                                                const double*, const double*, double*, void*,
                                                hipStream_t);
template hipError_t launch_fine_sources<float>(int, int, int, const double*, const double*, int,
                                               const int*, const double*, const double*,
                                               const double*, const double*, double*, void*,
                                               hipStream_t);

hipError_t launch_gemm_f64_cm(int Mr, int K, int Nc, const double* A, const double* B, double* C,
                              hipStream_t st) {
  dim3 grid((Nc + 63) / 64, (Mr + 63) / 64);
  k_gemm_f64<<<grid, 256, 0, st>>>(Mr, K, Nc, A, B, C);
  return hipGetLastError();
}

// Correction of the all-pairs sum for near pairs.  Workgroup (i, s) owns the targets of
// body i (one per thread) and split s of the concatenated source list of i's near
// bodies j: for each, the fine sources of j (added) then the plain sources of j
// (subtracted: the all-pairs sum already counted them).  The list position is uniform
// over the workgroup, so sources are wave-uniform loads as in the all-pairs kernel.
// Slot s of out ([S][3][N]) receives the scaled difference for every target of body i,
// zero when the split is empty, so the slots need no clearing.
template <typename T, int KIND>
__global__ __launch_bounds__(1024) void k_near_corr(int N, int M, int Mu, int kmax,
                                                    const T* __restrict__ tx, const T* __restrict__ tn,
                                                    const Src8<T>* __restrict__ src,
                                                    const Src8<T>* __restrict__ srcf,
                                                    const int* __restrict__ nbr,
                                                    const int* __restrict__ cnt,
                                                    double* __restrict__ out) {
  const int i = blockIdx.x, s = blockIdx.y, S = gridDim.y;
  const int a = threadIdx.x;
  const int g = i * M + min(a, M - 1);
  const T xa = tx[g], ya = tx[N + g], za = tx[2 * (size_t)N + g];
  T nx = 0, ny = 0, nz = 0;
  if (KIND == 0) {
    nx = tn[g];
    ny = tn[N + g];
    nz = tn[2 * (size_t)N + g];
  }
  T px = 0, py = 0, pz = 0, mx = 0, my = 0, mz = 0;
  const int c = min(cnt[i], kmax);
  const long seg = (long)Mu + M, L = (long)c * seg;
  const long lo = L * s / S, hi = L * (s + 1) / S;
  for (int k = (int)(lo / seg); k < c && (long)k * seg < hi; ++k) {
    const int j = nbr[(size_t)i * kmax + k];
    const long base = (long)k * seg;
    // fine sources of j: list positions [base, base + Mu)
    const Src8<T>* f = srcf + (size_t)j * Mu;
    const int f0 = (int)(max(lo, base) - base), f1 = (int)(min(hi, base + Mu) - base);
#pragma unroll 4
    for (int t = f0; t < f1; ++t) Pair<T, KIND>::add(xa, ya, za, nx, ny, nz, f[t], px, py, pz);
    // plain sources of j: list positions [base + Mu, base + Mu + M)
    const Src8<T>* q = src + (size_t)j * M;
    const int c0 = (int)(max(lo, base + Mu) - (base + Mu)), c1 = (int)(min(hi, base + seg) - (base + Mu));
#pragma unroll 4
    for (int t = c0; t < c1; ++t) Pair<T, KIND>::add(xa, ya, za, nx, ny, nz, q[t], mx, my, mz);
  }
  if (a < M) {
    const double scale = KIND == 0 ? -3.0 / (4.0 * RBM_PI) : 1.0 / (8.0 * RBM_PI);
    double* o = out + (size_t)s * 3 * N;
    o[g] = scale * ((double)px - (double)mx);
    o[N + g] = scale * ((double)py - (double)my);
    o[2 * (size_t)N + g] = scale * ((double)pz - (double)mz);
  }
}

template <typename T>
hipError_t launch_near_corr(int kind, int n, int M, int Mu, int kmax, int S, const T* tx,
                            const T* tn, const void* src, const void* srcf, const int* nbr,
                            const int* cnt, double* out, hipStream_t st) {
  const int N = n * M;
  dim3 grid(n, S);
  const int bs = ((M + 63) / 64) * 64;
  const Src8<T>* a = reinterpret_cast<const Src8<T>*>(src);
  const Src8<T>* b = reinterpret_cast<const Src8<T>*>(srcf);
  if (kind == 0)
    k_near_corr<T, 0><<<grid, bs, 0, st>>>(N, M, Mu, kmax, tx, tn, a, b, nbr, cnt, out);
  else
    k_near_corr<T, 1><<<grid, bs, 0, st>>>(N, M, Mu, kmax, tx, tn, a, b, nbr, cnt, out);
  return hipGetLastError();
}

template hipError_t launch_near_corr<double>(int, int, int, int, int, int, const double*,
                                             const double*, const void*, const void*, const int*,
                                             const int*, double*, hipStream_t);
template hipError_t launch_near_corr<float>(int, int, int, int, int, int, const float*,
                                            const float*, const void*, const void*, const int*,
                                            const int*, double*, hipStream_t);

}  // namespace rbm
