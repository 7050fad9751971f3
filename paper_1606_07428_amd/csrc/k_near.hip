// Near-singular evaluation by upsampling (§3): for a target close to another body the
// smooth rule over that body is evaluated on a finer grid of order p_u.  The geometry
// is evaluated exactly from the shape's SH coefficients at the fine nodes and the
// density by its band-limited interpolant.  This file holds the setup (fine geometry,
// bounding radii, interpolation matrix), the per-pose near list, the interpolation of
// fine sources and the correction sum, which uses the same pair arithmetic (pair.h) as
// the all-pairs sum of k_far.hip.
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

// Fine sources of the bodies listed in `need` (the bodies that are near some body):
// density zt_c(b) = sum_a U[a][b] z_c(a) (band-limited interpolant; z in body frames when
// z_is_body, then rotated), X' = c_j + R_j r'_b, q' = w'_b zt, packed like the plain
// sources.  kNB fine nodes per lane (b = 256 x + lane + 64 k) and kIB listed bodies per
// wave: U[a][b] is read coalesced over the lanes and the bodies' densities z_c(a) are
// wave-uniform (scalar loads), so each density value feeds kNB multiply-adds and each U
// value 3 kIB; every sum runs over a in order, in one lane.
constexpr int kIB = 4, kNB = 4;
template <typename T>
__global__ __launch_bounds__(256) void k_interp_pack(int n, int M, int Mu, int nneed,
                                                     const int* __restrict__ need,
                                                     const double* __restrict__ U,
                                                     const double* __restrict__ z, int z_is_body,
                                                     const int* __restrict__ sid,
                                                     const double* __restrict__ cen,
                                                     const double* __restrict__ Rm,
                                                     const double* __restrict__ fr_all,
                                                     const double* __restrict__ fw_all,
                                                     Src8<T>* __restrict__ srcf) {
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int q0 = (blockIdx.y * 4 + wv) * kIB;
  if (q0 >= nneed) return;  // whole waves; the kernel has no barrier
  const int jn = min(kIB, nneed - q0);
  const size_t N = (size_t)n * M;
  int bs[kNB];
#pragma unroll
  for (int k = 0; k < kNB; ++k) bs[k] = min(blockIdx.x * 64 * kNB + lane + 64 * k, Mu - 1);
  size_t zo[kIB];
#pragma unroll
  for (int jj = 0; jj < kIB; ++jj) zo[jj] = (size_t)need[q0 + min(jj, jn - 1)] * M;
  double acc[kIB][3][kNB];
#pragma unroll
  for (int jj = 0; jj < kIB; ++jj)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < kNB; ++k) acc[jj][c][k] = 0.0;
  for (int a = 0; a < M; ++a) {
    double u[kNB];
#pragma unroll
    for (int k = 0; k < kNB; ++k) u[k] = U[(size_t)a * Mu + bs[k]];
#pragma unroll
    for (int jj = 0; jj < kIB; ++jj) {
      const size_t g = zo[jj] + a;
      const double z0 = z[g], z1 = z[N + g], z2 = z[2 * N + g];
#pragma unroll
      for (int k = 0; k < kNB; ++k) {
        acc[jj][0][k] += u[k] * z0;
        acc[jj][1][k] += u[k] * z1;
        acc[jj][2][k] += u[k] * z2;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kNB; ++k) {
    const int b = blockIdx.x * 64 * kNB + lane + 64 * k;
    if (b >= Mu) break;
#pragma unroll
    for (int jj = 0; jj < kIB; ++jj) {
      if (jj >= jn) break;
      double v[3] = {acc[jj][0][k], acc[jj][1][k], acc[jj][2][k]};
      const int j = need[q0 + jj], s = sid[j];
      const double* R = Rm + 9 * j;
      if (z_is_body) {
        const double b0 = R[0] * v[0] + R[1] * v[1] + R[2] * v[2];
        const double b1 = R[3] * v[0] + R[4] * v[1] + R[5] * v[2];
        const double b2 = R[6] * v[0] + R[7] * v[1] + R[8] * v[2];
        v[0] = b0; v[1] = b1; v[2] = b2;
      }
      const double* fr = fr_all + (size_t)s * 3 * Mu;
      const double r0 = fr[b], r1 = fr[Mu + b], r2 = fr[2 * (size_t)Mu + b];
      const double w = fw_all[(size_t)s * Mu + b];
      Src8<T> o;
      o.v[0] = (T)(cen[3 * j] + R[0] * r0 + R[1] * r1 + R[2] * r2);
      o.v[1] = (T)(cen[3 * j + 1] + R[3] * r0 + R[4] * r1 + R[5] * r2);
      o.v[2] = (T)(cen[3 * j + 2] + R[6] * r0 + R[7] * r1 + R[8] * r2);
      o.v[3] = (T)(w * v[0]);
      o.v[4] = (T)(w * v[1]);
      o.v[5] = (T)(w * v[2]);
      o.v[6] = 0;
      o.v[7] = 0;
      srcf[(size_t)j * Mu + b] = o;
    }
  }
}

// Correction of the all-pairs sum for near pairs.  The concatenated source list of body
// i (for each near body j: its M_u fine sources, then its M plain sources, which the
// all-pairs sum already counted and are subtracted here; both sums are linear in q) is
// cut into items of ch positions; item t = (body item_body[t], positions [item_pos[t],
// item_pos[t] + ch) clipped to the list).  The workgroup of item t holds body i's targets
// (one per thread); the item's sources are the same for every thread, so they are read
// with wave-uniform (scalar) loads, four at a time, as in the all-pairs sum.  Fine and
// plain sources go to separate accumulators, subtracted at the end.  The scaled sums of
// the item's targets go to slot t ([items][3][M]).
template <typename T, int KIND>
__global__ __launch_bounds__(1024) void k_near_corr(int N, int M, int Mu, int kmax, int ch,
                                                    const int* __restrict__ item_body,
                                                    const int* __restrict__ item_pos,
                                                    const T* __restrict__ tx, const T* __restrict__ tn,
                                                    const Src8<T>* __restrict__ src,
                                                    const Src8<T>* __restrict__ srcf,
                                                    const int* __restrict__ nbr,
                                                    const int* __restrict__ cnt,
                                                    double* __restrict__ slots) {
  const int t = blockIdx.x, i = item_body[t];
  const int a = threadIdx.x;
  const int g = i * M + min(a, M - 1);
  const T xa = tx[g], ya = tx[N + g], za = tx[2 * (size_t)N + g];
  T nx = 0, ny = 0, nz = 0;
  if (KIND == 0) {
    nx = tn[g];
    ny = tn[N + g];
    nz = tn[2 * (size_t)N + g];
  }
  T fx = 0, fy = 0, fz = 0, px = 0, py = 0, pz = 0;
  auto sweep = [&](const Src8<T>* q, int n, T& ax, T& ay, T& az) {
    int k = 0;
    for (; k + 4 <= n; k += 4) {
      const Src8<T> q0 = q[k], q1 = q[k + 1], q2 = q[k + 2], q3 = q[k + 3];
      Pair<T, KIND>::add(xa, ya, za, nx, ny, nz, q0, ax, ay, az);
      Pair<T, KIND>::add(xa, ya, za, nx, ny, nz, q1, ax, ay, az);
      Pair<T, KIND>::add(xa, ya, za, nx, ny, nz, q2, ax, ay, az);
      Pair<T, KIND>::add(xa, ya, za, nx, ny, nz, q3, ax, ay, az);
    }
    for (; k < n; ++k) Pair<T, KIND>::add(xa, ya, za, nx, ny, nz, q[k], ax, ay, az);
  };
  const int seg = Mu + M, L = min(cnt[i], kmax) * seg;
  const int lo = item_pos[t], hi = min(L, lo + ch);
  for (int u = lo; u < hi;) {
    const int k = u / seg, r = u - k * seg;
    const int j = nbr[(size_t)i * kmax + k];
    if (r < Mu) {
      const int n = min(hi - u, Mu - r);
      sweep(srcf + (size_t)j * Mu + r, n, fx, fy, fz);
      u += n;
    } else {
      const int n = min(hi - u, seg - r);
      sweep(src + (size_t)j * M + (r - Mu), n, px, py, pz);
      u += n;
    }
  }
  const T ax = fx - px, ay = fy - py, az = fz - pz;
  if (a < M) {
    const double scale = (KIND == 0 ? -3.0 / (4.0 * RBM_PI) : 1.0 / (8.0 * RBM_PI)) * Pair<T, KIND>::kPost;
    double* o = slots + (size_t)t * 3 * M;
    o[a] = scale * (double)ax;
    o[M + a] = scale * (double)ay;
    o[2 * M + a] = scale * (double)az;
  }
}

// res[c][i*M + a] = sum over body i's items (item_first[i] .. item_first[i+1]-1, in order)
// of slot[c][a]; 0 for bodies without near bodies.
__global__ __launch_bounds__(256) void k_near_reduce(int N, int M, const int* __restrict__ item_first,
                                                     const double* __restrict__ slots,
                                                     double* __restrict__ res) {
  const int i = blockIdx.x;
  const int e = blockIdx.y * blockDim.x + threadIdx.x;
  if (e >= 3 * M) return;
  const int t0 = item_first[i], t1 = item_first[i + 1];
  double v = 0.0;
  int t = t0;
  for (; t + 4 <= t1; t += 4) {
    const double v0 = slots[(size_t)t * 3 * M + e], v1 = slots[(size_t)(t + 1) * 3 * M + e];
    const double v2 = slots[(size_t)(t + 2) * 3 * M + e], v3 = slots[(size_t)(t + 3) * 3 * M + e];
    v += v0;
    v += v1;
    v += v2;
    v += v3;
  }
  for (; t < t1; ++t) v += slots[(size_t)t * 3 * M + e];
  const int comp = e / M, a = e - comp * M;
  res[(size_t)comp * N + (size_t)i * M + a] = v;
}

template <typename T>
hipError_t launch_near_corr(int kind, int n, int M, int Mu, int kmax, int nneed, const int* need,
                            int nitems, int ch, const int* item_body, const int* item_pos,
                            const int* item_first, const T* tx, const T* tn, const void* src,
                            const double* z, int z_is_body, const double* U, const int* sid,
                            const double* cen, const double* Rm, const double* fr, const double* fw,
                            const int* nbr, const int* cnt, void* srcf, double* slots, double* res,
                            hipStream_t st) {
  const int N = n * M;
  if (nitems > 0 && nneed > 0) {
    dim3 gi((Mu + 64 * kNB - 1) / (64 * kNB), (nneed + 4 * kIB - 1) / (4 * kIB));
    k_interp_pack<T><<<gi, 256, 0, st>>>(n, M, Mu, nneed, need, U, z, z_is_body, sid, cen, Rm, fr, fw,
                                         reinterpret_cast<Src8<T>*>(srcf));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int bs = ((M + 63) / 64) * 64;
    const size_t lds = 0;
    const Src8<T>* ps = reinterpret_cast<const Src8<T>*>(src);
    const Src8<T>* pf = reinterpret_cast<const Src8<T>*>(srcf);
    if (kind == 0)
      k_near_corr<T, 0><<<nitems, bs, lds, st>>>(N, M, Mu, kmax, ch, item_body, item_pos, tx, tn, ps, pf,
                                                 nbr, cnt, slots);
    else
      k_near_corr<T, 1><<<nitems, bs, lds, st>>>(N, M, Mu, kmax, ch, item_body, item_pos, tx, tn, ps, pf,
                                                 nbr, cnt, slots);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  dim3 gr(n, (3 * M + 255) / 256);
  k_near_reduce<<<gr, 256, 0, st>>>(N, M, item_first, slots, res);
  return hipGetLastError();
}

template hipError_t launch_near_corr<double>(int, int, int, int, int, int, const int*, int, int,
                                             const int*, const int*, const int*, const double*,
                                             const double*, const void*, const double*, int,
                                             const double*, const int*, const double*,
                                             const double*, const double*, const double*,
                                             const int*, const int*, void*, double*, double*,
                                             hipStream_t);
template hipError_t launch_near_corr<float>(int, int, int, int, int, int, const int*, int, int,
                                            const int*, const int*, const int*, const float*,
                                            const float*, const void*, const double*, int,
                                            const double*, const int*, const double*,
                                            const double*, const double*, const double*,
                                            const int*, const int*, void*, double*, double*,
                                            hipStream_t);

// Contact search (§3.3 contact force algorithm): for candidate body pairs (a, b), the
// closest pair of nodes, by the smallest (|X_a - X_b|^2, ia * M + ib) so that ties go to
// the smallest node indices; out[k] = (d^2, index, x* = midpoint).  One workgroup per pair.
__global__ __launch_bounds__(256) void k_closest_pair(int N, int M, const int* __restrict__ cand,
                                                      const double* __restrict__ X,
                                                      double* __restrict__ out) {
  __shared__ double sd[256];
  __shared__ long si[256];
  const int k = blockIdx.x;
  const int a = cand[2 * k], b = cand[2 * k + 1];
  double best = 1e300;
  long bi = 0x7fffffffffffffffL;
  const long MM = (long)M * M;
  for (long e = threadIdx.x; e < MM; e += 256) {
    const int ia = (int)(e / M), ib = (int)(e - (long)ia * M);
    const size_t ga = (size_t)a * M + ia, gb = (size_t)b * M + ib;
    const double dx = X[ga] - X[gb], dy = X[N + ga] - X[N + gb], dz = X[2 * (size_t)N + ga] - X[2 * (size_t)N + gb];
    const double d2 = dx * dx + dy * dy + dz * dz;
    if (d2 < best || (d2 == best && e < bi)) {
      best = d2;
      bi = e;
    }
  }
  sd[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      const double d = sd[threadIdx.x + h];
      const long i = si[threadIdx.x + h];
      if (d < sd[threadIdx.x] || (d == sd[threadIdx.x] && i < si[threadIdx.x])) {
        sd[threadIdx.x] = d;
        si[threadIdx.x] = i;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const long e = si[0];
    const int ia = (int)(e / M), ib = (int)(e - (long)ia * M);
    const size_t ga = (size_t)a * M + ia, gb = (size_t)b * M + ib;
    out[5 * k] = sd[0];
    out[5 * k + 1] = (double)e;
    for (int c = 0; c < 3; ++c) out[5 * k + 2 + c] = 0.5 * (X[(size_t)c * N + ga] + X[(size_t)c * N + gb]);
  }
}

// Overlap test of candidate body pairs (a, b): for every node y of one body, the node X_r
// of the other body nearest to y (ties: smaller index) and the signed offset
// s = (y - X_r) . N_r along that node's outward normal.  A node of a smooth body lying
// outside the other body has s >= -(covering radius)^2 x curvature / 2, one inside has
// s < 0 growing with its depth.  out[2k + dir] = min over y of s, dir 0: nodes of b against
// body a, dir 1: nodes of a against body b.  One workgroup per (pair, direction); the
// reference body's nodes and normals are staged in LDS.
__global__ __launch_bounds__(256) void k_overlap_depth(int N, int M, const int* __restrict__ cand,
                                                       const double* __restrict__ X,
                                                       const double* __restrict__ Nn,
                                                       double* __restrict__ out) {
  extern __shared__ double sref[];  // [6][M]: reference nodes then normals
  const int k = blockIdx.x, dir = blockIdx.y;
  const int a = cand[2 * k], b = cand[2 * k + 1];
  const int rb = dir == 0 ? a : b, tb = dir == 0 ? b : a;
  for (int e = threadIdx.x; e < 3 * M; e += 256) {
    const int c = e / M, i = e - c * M;
    sref[e] = X[(size_t)c * N + (size_t)rb * M + i];
    sref[3 * M + e] = Nn[(size_t)c * N + (size_t)rb * M + i];
  }
  __syncthreads();
  double smin = 1e300;
  for (int t = threadIdx.x; t < M; t += 256) {
    const size_t g = (size_t)tb * M + t;
    const double yx = X[g], yy = X[N + g], yz = X[2 * (size_t)N + g];
    double best = 1e300;
    int bi = 0;
    for (int i = 0; i < M; ++i) {
      const double dx = yx - sref[i], dy = yy - sref[M + i], dz = yz - sref[2 * M + i];
      const double d2 = dx * dx + dy * dy + dz * dz;
      if (d2 < best) {
        best = d2;
        bi = i;
      }
    }
    const double s = (yx - sref[bi]) * sref[3 * M + bi] + (yy - sref[M + bi]) * sref[4 * M + bi] +
                     (yz - sref[2 * M + bi]) * sref[5 * M + bi];
    smin = fmin(smin, s);
  }
  __shared__ double red[256];
  red[threadIdx.x] = smin;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[2 * k + dir] = red[0];
}

// Largest nearest-neighbour spacing of a shape's nodes: hs[s] = max_a min_{b != a} |r_a - r_b|
// over r [ns][3][M].  One workgroup per shape.
__global__ __launch_bounds__(256) void k_node_spacing(int M, const double* __restrict__ r,
                                                      double* __restrict__ hs) {
  const double* rs = r + (size_t)blockIdx.x * 3 * M;
  double hmax = 0.0;
  for (int a = threadIdx.x; a < M; a += 256) {
    double best = 1e300;
    for (int b = 0; b < M; ++b) {
      if (b == a) continue;
      const double dx = rs[a] - rs[b], dy = rs[M + a] - rs[M + b], dz = rs[2 * M + a] - rs[2 * M + b];
      best = fmin(best, dx * dx + dy * dy + dz * dz);
    }
    hmax = fmax(hmax, best);
  }
  __shared__ double red[256];
  red[threadIdx.x] = hmax;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) hs[blockIdx.x] = sqrt(red[0]);
}

hipError_t launch_overlap_depth(int ncand, int N, int M, const int* cand, const double* X, const double* Nn,
                                double* out, hipStream_t st) {
  if (ncand < 1) return hipSuccess;
  k_overlap_depth<<<dim3(ncand, 2), 256, 6 * (size_t)M * sizeof(double), st>>>(N, M, cand, X, Nn, out);
  return hipGetLastError();
}

hipError_t launch_node_spacing(int ns, int M, const double* r, double* hs, hipStream_t st) {
  k_node_spacing<<<ns, 256, 0, st>>>(M, r, hs);
  return hipGetLastError();
}

hipError_t launch_closest_pairs(int ncand, int N, int M, const int* cand, const double* X, double* out,
                                hipStream_t st) {
  if (ncand < 1) return hipSuccess;
  k_closest_pair<<<ncand, 256, 0, st>>>(N, M, cand, X, out);
  return hipGetLastError();
}

hipError_t launch_bound_radius(int ns, int M, const double* r, double* rb, hipStream_t st) {
  k_bound_radius<<<ns, 256, 0, st>>>(M, r, rb);
  return hipGetLastError();
}

}  // namespace rbm
