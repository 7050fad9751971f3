// Magnetostatics of permeable bodies (§4, magnetorheological flows): the scalar Laplace
// operators of the second-kind equation (1/2 I + eta K^L) q = eta H0 . n, the exterior
// field H = -grad phi on the surface, phi = -H0 . x + S^L[q], and its Maxwell traction
// mu0 [(H . n) H - |H|^2 n / 2], the incident density of the mobility problem.  Self
// interactions use the singular rule of §3 (rotated grid, band-limited interpolant);
// interactions between bodies use the all-pairs sums of k_far.hip (kinds 2 and 3).
#include "common.h"
#include "kernels.h"
#include "pair.h"

namespace rbm {

// Laplace self operators of every shape, column-major [s][a * M + t] (weight of node a in
// the integral at target t): S^L with kernel 1/(4 pi r) and K^L with -(r . n_t)/(4 pi r^3),
// r = x_t - y.  One workgroup per (target t, shape s); the rotated nodes q of the rule go
// through LDS in chunks of NC: C[k][b] = sum_q W_q J_q kern_k(q) Y_b(s_q), then
// row(t) = C F with F the forward transform (grid -> band B_p).
template <int NC>
__global__ __launch_bounds__(256) void k_singular_laplace(int p, int ps,
                                                          const double* __restrict__ coef_all,
                                                          const double* __restrict__ gx_all,
                                                          const double* __restrict__ gn_all,
                                                          const double* __restrict__ nth,
                                                          const double* __restrict__ nph,
                                                          const double* __restrict__ rnodes,
                                                          const double* __restrict__ rW,
                                                          const double* __restrict__ Ft,
                                                          double* __restrict__ SL,
                                                          double* __restrict__ KL) {
  extern __shared__ double lds[];
  // row stride of the staged harmonics: odd, so that the contraction, whose lanes
  // read one row each at the same column, hits distinct LDS banks (a stride of 64
  // doubles put every lane in one bank)
  constexpr int YS = NC + 1;
  const int M = (p + 1) * 2 * p, nc = (p + 1) * (p + 1), nB = p * p + 2 * p;
  const int Ms = (ps + 1) * 2 * ps;
  const int t = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  double* cf = lds;             // [3][nc]
  double* Ych = cf + 3 * nc;    // [nB][YS]
  double* Kw = Ych + nB * YS;   // [2][NC]
  double* ltab = Kw + 2 * NC;   // Legendre recurrence coefficients
  for (int i = tid; i < 3 * nc; i += 256) cf[i] = coef_all[(size_t)s * 3 * nc + i];
  legendre_table(p, ltab, tid, 256);
  double st, ct, sp, cp;
  sincos(nth[t], &st, &ct);
  sincos(nph[t], &sp, &cp);
  const double Q[9] = {cp * ct, -sp, cp * st, sp * ct, cp, sp * st, -st, 0.0, ct};
  const double* gx = gx_all + (size_t)s * 3 * M;
  const double* gn = gn_all + (size_t)s * 3 * M;
  const double xt0 = gx[t], xt1 = gx[M + t], xt2 = gx[2 * M + t];
  const double nt0 = gn[t], nt1 = gn[M + t], nt2 = gn[2 * M + t];
  const double c4 = 1.0 / (4.0 * RBM_PI);
  double acc0[2] = {0.0, 0.0}, acc1[2] = {0.0, 0.0};
  for (int chunk = 0; chunk < Ms; chunk += NC) {
    __syncthreads();
    if (tid < NC) {
      const int q = chunk + tid;
      if (q < Ms) {
        const double s0 = rnodes[q], s1 = rnodes[Ms + q], s2 = rnodes[2 * Ms + q];
        const double v0 = Q[0] * s0 + Q[1] * s1 + Q[2] * s2;
        const double v1 = Q[3] * s0 + Q[4] * s1 + Q[5] * s2;
        const double v2 = Q[6] * s0 + Q[7] * s1 + Q[8] * s2;
        const double sx = sqrt(v0 * v0 + v1 * v1), cx = v2, ph = atan2(v1, v0);
        double x[3] = {0, 0, 0}, dt[3] = {0, 0, 0}, dp[3] = {0, 0, 0};
        int cur_m = -1;
        double cm = 1.0, sm = 0.0;
        legendre_sweep(p, cx, sx, [&](int l, int m, double P, double Qv, double D) {
          const int i0 = l * l + l;
          if (m == 0) {
            for (int c = 0; c < 3; ++c) {
              x[c] += cf[c * nc + i0] * P;
              dt[c] += cf[c * nc + i0] * D;
            }
            Ych[band_index(l, 0, p) * YS + tid] = P;
            return;
          }
          if (m != cur_m) {
            sincos(m * ph, &sm, &cm);
            cur_m = m;
          }
          const double r2 = 1.41421356237309504880;
          const double yp = r2 * P * cm, ym = r2 * P * sm;
          for (int c = 0; c < 3; ++c) {
            const double ap = cf[c * nc + i0 + m], am = cf[c * nc + i0 - m];
            x[c] += ap * yp + am * ym;
            dt[c] += r2 * D * (ap * cm + am * sm);
            dp[c] += r2 * m * Qv * (am * cm - ap * sm);
          }
          Ych[band_index(l, m, p) * YS + tid] = yp;
          const int bm = band_index(l, -m, p);
          if (bm >= 0) Ych[bm * YS + tid] = ym;
        }, ltab);
        const double c0 = dt[1] * dp[2] - dt[2] * dp[1];
        const double c1 = dt[2] * dp[0] - dt[0] * dp[2];
        const double c2 = dt[0] * dp[1] - dt[1] * dp[0];
        const double w = rW[q] * sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        const double r0 = xt0 - x[0], r1 = xt1 - x[1], r2v = xt2 - x[2];
        const double di = 1.0 / sqrt(r0 * r0 + r1 * r1 + r2v * r2v);
        Kw[tid] = w * c4 * di;
        Kw[NC + tid] = -w * c4 * (r0 * nt0 + r1 * nt1 + r2v * nt2) * di * di * di;
      } else {
        Kw[tid] = Kw[NC + tid] = 0.0;
        for (int b = 0; b < nB; ++b) Ych[b * YS + tid] = 0.0;
      }
    }
    __syncthreads();
    if (tid < nB)
      for (int q = 0; q < NC; ++q) {
        const double y = Ych[tid * YS + q];
        acc0[0] += Kw[q] * y;
        acc0[1] += Kw[NC + q] * y;
      }
    if (tid + 256 < nB)
      for (int q = 0; q < NC; ++q) {
        const double y = Ych[(tid + 256) * YS + q];
        acc1[0] += Kw[q] * y;
        acc1[1] += Kw[NC + q] * y;
      }
  }
  __syncthreads();
  double* Cs = Ych;  // [2][nB]
  if (tid < nB) {
    Cs[tid] = acc0[0];
    Cs[nB + tid] = acc0[1];
  }
  if (tid + 256 < nB) {
    Cs[tid + 256] = acc1[0];
    Cs[nB + tid + 256] = acc1[1];
  }
  __syncthreads();
  for (int a = tid; a < M; a += 256) {
    double vs = 0.0, vk = 0.0;
    const double* f = Ft + (size_t)a * nB;
    for (int b = 0; b < nB; ++b) {
      vs += Cs[b] * f[b];
      vk += Cs[nB + b] * f[b];
    }
    SL[(size_t)s * M * M + (size_t)a * M + t] = vs;
    KL[(size_t)s * M * M + (size_t)a * M + t] = vk;
  }
}

// Spectral derivatives on the grid, column-major [a * M + t]: D_t gives d/dtheta and D_p
// (d/dphi)/sin(theta) of the band-limited interpolant at node t from the values at node a:
// D = Y'_B(node t)^T F.  Ytab-style tables use the full index l*l + l + m, F the band one.
__global__ void k_derivative_matrices(int p, const double* __restrict__ Yttab,
                                      const double* __restrict__ Ypstab,
                                      const double* __restrict__ Ftab, double* __restrict__ Dt,
                                      double* __restrict__ Dp) {
  const int M = (p + 1) * 2 * p;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)M * M) return;
  const int a = (int)(e / M), t = (int)(e % M);
  double vt = 0.0, vp = 0.0;
  for (int l = 0; l <= p; ++l)
    for (int m = -l; m <= l; ++m) {
      const int b = band_index(l, m, p);
      if (b < 0) continue;
      const int k = l * l + l + m;
      const double f = Ftab[(size_t)b * M + a];
      vt += Yttab[(size_t)k * M + t] * f;
      vp += Ypstab[(size_t)k * M + t] * f;
    }
  Dt[e] = vt;
  Dp[e] = vp;
}

// Body-frame tangents of every shape at the grid: x_theta and x_phi/sin(theta), [s][6][M].
__global__ void k_shape_tangents(int p, int ns, const double* __restrict__ coef_all,
                                 const double* __restrict__ Yttab, const double* __restrict__ Ypstab,
                                 double* __restrict__ tang) {
  const int M = (p + 1) * 2 * p, nc = (p + 1) * (p + 1);
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)ns * M) return;
  const int s = (int)(e / M), a = (int)(e % M);
  const double* cf = coef_all + (size_t)s * 3 * nc;
  double xt[3] = {0, 0, 0}, xp[3] = {0, 0, 0};
  for (int i = 0; i < nc; ++i) {
    const double yt = Yttab[(size_t)i * M + a], yp = Ypstab[(size_t)i * M + a];
    for (int c = 0; c < 3; ++c) {
      xt[c] += cf[c * nc + i] * yt;
      xp[c] += cf[c * nc + i] * yp;
    }
  }
  double* o = tang + (size_t)s * 6 * M;
  for (int c = 0; c < 3; ++c) {
    o[(size_t)c * M + a] = xt[c];
    o[(size_t)(3 + c) * M + a] = xp[c];
  }
}

// y[i*M + t] = sum_a A_{s(i)}[a*M + t] x[i*M + a] for every body (column-major blocks).
__global__ __launch_bounds__(256) void k_scalar_self(int n, int M, const int* __restrict__ sid,
                                                     const double* __restrict__ A,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ y) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * M) return;
  const int i = (int)(e / M), t = (int)(e % M);
  const double* Ai = A + (size_t)sid[i] * M * M;
  const double* xi = x + (size_t)i * M;
  double v = 0.0;
  for (int a = 0; a < M; ++a) v += Ai[(size_t)a * M + t] * xi[a];
  y[e] = v;
}

// Packed scalar sources: (x, y, z, w q, 0, 0, 0, 0).
__global__ void k_pack_scalar(int N, const double* __restrict__ X, const double* __restrict__ W,
                              const double* __restrict__ q, Src8<double>* __restrict__ src) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  Src8<double> s;
  s.v[0] = X[g];
  s.v[1] = X[N + g];
  s.v[2] = X[2 * (size_t)N + g];
  s.v[3] = W[g] * q[g];
  s.v[4] = s.v[5] = s.v[6] = s.v[7] = 0.0;
  src[g] = s;
}

// out = cv v + cs self + cp sum_s part[s][0][g] (first component of the split slots).
__global__ void k_scalar_combine(int N, int nsplit, const double* __restrict__ part, double cp,
                                 const double* __restrict__ self, double cs,
                                 const double* __restrict__ v, double cv, double* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  double f = 0.0;
  for (int s = 0; s < nsplit; ++s) f += part[(size_t)s * 3 * N + g];
  double r = cp * f;
  if (self) r += cs * self[g];
  if (v) r += cv * v[g];
  out[g] = r;
}

// Exterior field and Maxwell traction at every node: tangential gradient of phi by the
// derivative matrices and the lab-frame tangents (a = R x_theta, b = R x_phi/sin), normal
// derivative dn (exterior, from the jump relation), H = -(grad_s phi + n dn),
// rho = mu0 [(H . n) H - |H|^2 n / 2] ([3][N]).
__global__ __launch_bounds__(256) void k_magnetic_traction(int n, int M, const int* __restrict__ sid,
                                                           const double* __restrict__ Rm,
                                                           const double* __restrict__ Nn,
                                                           const double* __restrict__ tang,
                                                           const double* __restrict__ Dt,
                                                           const double* __restrict__ Dp,
                                                           const double* __restrict__ phi,
                                                           const double* __restrict__ dn,
                                                           double mu0, double* __restrict__ rho) {
  const size_t N = (size_t)n * M;
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int i = (int)(g / M), t = (int)(g % M);
  const double* ph = phi + (size_t)i * M;
  double ft = 0.0, fp = 0.0;
  for (int a = 0; a < M; ++a) {
    ft += Dt[(size_t)a * M + t] * ph[a];
    fp += Dp[(size_t)a * M + t] * ph[a];
  }
  const double* R = Rm + 9 * i;
  const double* tg = tang + (size_t)sid[i] * 6 * M;
  const double u0 = tg[t], u1 = tg[M + t], u2 = tg[2 * M + t];
  const double w0 = tg[3 * M + t], w1 = tg[4 * M + t], w2 = tg[5 * M + t];
  const double av[3] = {R[0] * u0 + R[1] * u1 + R[2] * u2, R[3] * u0 + R[4] * u1 + R[5] * u2,
                        R[6] * u0 + R[7] * u1 + R[8] * u2};
  const double bv[3] = {R[0] * w0 + R[1] * w1 + R[2] * w2, R[3] * w0 + R[4] * w1 + R[5] * w2,
                        R[6] * w0 + R[7] * w1 + R[8] * w2};
  const double aa = av[0] * av[0] + av[1] * av[1] + av[2] * av[2];
  const double bb = bv[0] * bv[0] + bv[1] * bv[1] + bv[2] * bv[2];
  const double ab = av[0] * bv[0] + av[1] * bv[1] + av[2] * bv[2];
  const double det = aa * bb - ab * ab;
  const double ca = (bb * ft - ab * fp) / det, cb = (aa * fp - ab * ft) / det;
  const double nv[3] = {Nn[g], Nn[N + g], Nn[2 * N + g]};
  double H[3];
  for (int c = 0; c < 3; ++c) H[c] = -(ca * av[c] + cb * bv[c] + dn[g] * nv[c]);
  const double Hn = H[0] * nv[0] + H[1] * nv[1] + H[2] * nv[2];
  const double H2 = H[0] * H[0] + H[1] * H[1] + H[2] * H[2];
  for (int c = 0; c < 3; ++c) rho[(size_t)c * N + g] = mu0 * (Hn * H[c] - 0.5 * H2 * nv[c]);
}

hipError_t launch_singular_laplace(int ns, int p, int ps, const double* coef, const double* gx,
                                   const double* gn, const double* node_th, const double* node_ph,
                                   const double* rnodes, const double* rW, const double* Fttab,
                                   double* SL, double* KL, hipStream_t st) {
  const int M = (p + 1) * 2 * p;
  dim3 grid(M, ns);
  const int nodes = singular_chunk(p, 2);
  const size_t lds = singular_lds_bytes(p, nodes, 2);
  auto run = [&](auto kern) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    kern<<<grid, 256, lds, st>>>(p, ps, coef, gx, gn, node_th, node_ph, rnodes, rW, Fttab, SL, KL);
    return hipSuccess;
  };
  hipError_t e = nodes == 64 ? run(k_singular_laplace<64>) : nodes == 48 ? run(k_singular_laplace<48>)
                             : run(k_singular_laplace<32>);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_magnetic_tables(int p, int ns, const double* coef, const double* Yttab,
                                  const double* Ypstab, const double* Ftab, double* Dt, double* Dp,
                                  double* tang, hipStream_t st) {
  const int M = (p + 1) * 2 * p;
  const size_t mm = (size_t)M * M;
  k_derivative_matrices<<<(unsigned)((mm + 255) / 256), 256, 0, st>>>(p, Yttab, Ypstab, Ftab, Dt, Dp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t nm = (size_t)ns * M;
  k_shape_tangents<<<(unsigned)((nm + 255) / 256), 256, 0, st>>>(p, ns, coef, Yttab, Ypstab, tang);
  return hipGetLastError();
}

hipError_t launch_scalar_self(int n, int M, const int* sid, const double* A, const double* x, double* y,
                              hipStream_t st) {
  const size_t N = (size_t)n * M;
  k_scalar_self<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(n, M, sid, A, x, y);
  return hipGetLastError();
}

hipError_t launch_pack_scalar(int N, const double* X, const double* W, const double* q, void* src,
                              hipStream_t st) {
  k_pack_scalar<<<(N + 255) / 256, 256, 0, st>>>(N, X, W, q, reinterpret_cast<Src8<double>*>(src));
  return hipGetLastError();
}

hipError_t launch_scalar_combine(int N, int nsplit, const double* part, double cp, const double* self,
                                 double cs, const double* v, double cv, double* out, hipStream_t st) {
  k_scalar_combine<<<(N + 255) / 256, 256, 0, st>>>(N, nsplit, part, cp, self, cs, v, cv, out);
  return hipGetLastError();
}

__global__ void k_hdot(int N, const double* __restrict__ V, double h0, double h1, double h2, double scale,
                       int accumulate, double* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const double v = scale * (h0 * V[g] + h1 * V[N + g] + h2 * V[2 * (size_t)N + g]);
  out[g] = accumulate ? out[g] + v : v;
}

hipError_t launch_hdot(int N, const double* V, double h0, double h1, double h2, double scale,
                       int accumulate, double* out, hipStream_t st) {
  k_hdot<<<(N + 255) / 256, 256, 0, st>>>(N, V, h0, h1, h2, scale, accumulate, out);
  return hipGetLastError();
}

hipError_t launch_magnetic_traction(int n, int M, const int* sid, const double* Rm, const double* Nn,
                                    const double* tang, const double* Dt, const double* Dp,
                                    const double* phi, const double* dn, double mu0, double* rho,
                                    hipStream_t st) {
  const size_t N = (size_t)n * M;
  k_magnetic_traction<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(n, M, sid, Rm, Nn, tang, Dt, Dp, phi,
                                                                   dn, mu0, rho);
  return hipGetLastError();
}

}  // namespace rbm
