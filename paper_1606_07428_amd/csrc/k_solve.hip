// Per-solve kernels (float64): body poses, lab-frame nodes, the incident density of
// §2.2, per-body moments (the L operator of §2.3 and the rigid projection of §3.3),
// and the velocity evaluation.
#include "common.h"
#include "kernels.h"

namespace rbm {

// R_i = R(q_i), tau_i^{-1} in the lab frame = R tau0^{-1} R^T, area.
__global__ void k_body_prep(int n, const double* quat, const int* sid, const double* shp,
                            double* Rm, double* tauinv_lab, double* area_b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double R[9];
  quat_to_rot(quat + 4 * i, R);
  const double* sp = shp + (size_t)sid[i] * 32;
  const double* ti = sp + 13;
  double T[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double v = 0.0;
      for (int e = 0; e < 3; ++e)
        for (int f = 0; f < 3; ++f) v += R[3 * r + e] * ti[3 * e + f] * R[3 * c + f];
      T[3 * r + c] = v;
    }
  for (int k = 0; k < 9; ++k) {
    Rm[9 * i + k] = R[k];
    tauinv_lab[9 * i + k] = T[k];
  }
  area_b[i] = sp[0];
}

hipError_t launch_body_prep(int n, const double* quat, const int* sid, const double* shp,
                            double* Rm, double* tauinv_lab, double* area_b, hipStream_t st) {
  k_body_prep<<<(n + 63) / 64, 64, 0, st>>>(n, quat, sid, shp, Rm, tauinv_lab, area_b);
  return hipGetLastError();
}

// X = c_i + R_i r, N = R_i n (rigid kinematics of §3.3), W = w (rotation invariant).
__global__ void k_nodes(int n, int M, const int* sid, const double* cen, const double* Rm,
                        const double* gr, const double* gn, const double* gw, double* X,
                        double* Nn, double* W, float* Xf, float* Nf) {
  const size_t N = (size_t)n * M;
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int i = (int)(g / M), a = (int)(g % M);
  const int s = sid[i];
  const double* R = Rm + 9 * i;
  const double* r = gr + (size_t)s * 3 * M;
  const double* nn = gn + (size_t)s * 3 * M;
  const double r0 = r[a], r1 = r[M + a], r2 = r[2 * M + a];
  const double n0 = nn[a], n1 = nn[M + a], n2 = nn[2 * M + a];
  for (int c = 0; c < 3; ++c) {
    const double x = cen[3 * i + c] + R[3 * c] * r0 + R[3 * c + 1] * r1 + R[3 * c + 2] * r2;
    const double nv = R[3 * c] * n0 + R[3 * c + 1] * n1 + R[3 * c + 2] * n2;
    X[c * N + g] = x;
    Nn[c * N + g] = nv;
    Xf[c * N + g] = (float)x;
    Nf[c * N + g] = (float)nv;
  }
  W[g] = gw[(size_t)s * M + a];
}

hipError_t launch_nodes(int n, int M, const int* sid, const double* cen, const double* Rm,
                        const double* gr, const double* gn, const double* gw, double* X,
                        double* Nn, double* W, float* Xf, float* Nf, hipStream_t st) {
  const size_t N = (size_t)n * M;
  k_nodes<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(n, M, sid, cen, Rm, gr, gn, gw, X, Nn, W,
                                                       Xf, Nf);
  return hipGetLastError();
}

// rho = F_i/|Gamma_i| + (tau_i^{-1} T_i) x (X - c_i)   (incident density, §2.2)
__global__ void k_rho(int n, int M, const double* FT, const double* cen, const double* X,
                      const double* tauinv_lab, const double* area_b, double* rho) {
  const size_t N = (size_t)n * M;
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int i = (int)(g / M);
  const double* ft = FT + 6 * i;
  const double* ti = tauinv_lab + 9 * i;
  const double O0 = ti[0] * ft[3] + ti[1] * ft[4] + ti[2] * ft[5];
  const double O1 = ti[3] * ft[3] + ti[4] * ft[4] + ti[5] * ft[5];
  const double O2 = ti[6] * ft[3] + ti[7] * ft[4] + ti[8] * ft[5];
  const double r0 = X[g] - cen[3 * i], r1 = X[N + g] - cen[3 * i + 1],
               r2 = X[2 * N + g] - cen[3 * i + 2];
  const double ia = 1.0 / area_b[i];
  rho[g] = ft[0] * ia + (O1 * r2 - O2 * r1);
  rho[N + g] = ft[1] * ia + (O2 * r0 - O0 * r2);
  rho[2 * N + g] = ft[2] * ia + (O0 * r1 - O1 * r0);
}

hipError_t launch_rho(int n, int M, const double* FT, const double* cen, const double* X,
                      const double* tauinv_lab, const double* area_b, double* rho, hipStream_t st) {
  const size_t N = (size_t)n * M;
  k_rho<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(n, M, FT, cen, X, tauinv_lab, area_b, rho);
  return hipGetLastError();
}

// mom[i] = (sum_a w u_a, sum_a w (X_a - c_i) x u_a), one workgroup per body.
__global__ __launch_bounds__(256) void k_moments(int n, int M, const double* u, const double* X,
                                                 const double* W, const double* cen,
                                                 double* mom) {
  __shared__ double red[8];
  const size_t N = (size_t)n * M;
  const int i = blockIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int a = threadIdx.x; a < M; a += 256) {
    const size_t g = (size_t)i * M + a;
    const double w = W[g];
    const double u0 = u[g], u1 = u[N + g], u2 = u[2 * N + g];
    const double r0 = X[g] - cen[3 * i], r1 = X[N + g] - cen[3 * i + 1],
                 r2 = X[2 * N + g] - cen[3 * i + 2];
    acc[0] += w * u0;
    acc[1] += w * u1;
    acc[2] += w * u2;
    acc[3] += w * (r1 * u2 - r2 * u1);
    acc[4] += w * (r2 * u0 - r0 * u2);
    acc[5] += w * (r0 * u1 - r1 * u0);
  }
  for (int k = 0; k < 6; ++k) {
    const double v = block_sum(acc[k], red);
    if (threadIdx.x == 0) mom[6 * i + k] = v;
  }
}

hipError_t launch_moments(int n, int M, const double* u, const double* X, const double* W,
                          const double* cen, double* mom, hipStream_t st) {
  k_moments<<<n, 256, 0, st>>>(n, M, u, X, W, cen, mom);
  return hipGetLastError();
}

// out += sign * (F_i + T_i x (X - c_i)) with (F_i, T_i) = mom[i]: the L operator of §2.3.
__global__ void k_add_rigid(int n, int M, const double* mom, const double* X, const double* cen,
                            double sign, double* out) {
  const size_t N = (size_t)n * M;
  const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int i = (int)(g / M);
  const double* m = mom + 6 * i;
  const double r0 = X[g] - cen[3 * i], r1 = X[N + g] - cen[3 * i + 1],
               r2 = X[2 * N + g] - cen[3 * i + 2];
  out[g] += sign * (m[0] + (m[4] * r2 - m[5] * r1));
  out[N + g] += sign * (m[1] + (m[5] * r0 - m[3] * r2));
  out[2 * N + g] += sign * (m[2] + (m[3] * r1 - m[4] * r0));
}

hipError_t launch_add_rigid(int n, int M, const double* mom, const double* X, const double* cen,
                            double sign, double* out, hipStream_t st) {
  const size_t N = (size_t)n * M;
  k_add_rigid<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(n, M, mom, X, cen, sign, out);
  return hipGetLastError();
}

// Self part of (v_i, omega_i): R_i V0_{s(i)} R_i^T sigma_i, one workgroup per body.
__global__ __launch_bounds__(256) void k_velocity_self(int n, int M, const int* sid,
                                                       const double* V0, const double* Rm,
                                                       const double* sig, double* vw) {
  __shared__ double red[8];
  const size_t N = (size_t)n * M;
  const int M3 = 3 * M;
  const int i = blockIdx.x;
  const double* R = Rm + 9 * i;
  const double* V = V0 + (size_t)sid[i] * 6 * M3;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int a = threadIdx.x; a < M; a += 256) {
    const size_t g = (size_t)i * M + a;
    const double v0 = sig[g], v1 = sig[N + g], v2 = sig[2 * N + g];
    const double b0 = R[0] * v0 + R[3] * v1 + R[6] * v2;
    const double b1 = R[1] * v0 + R[4] * v1 + R[7] * v2;
    const double b2 = R[2] * v0 + R[5] * v1 + R[8] * v2;
    for (int k = 0; k < 6; ++k)
      acc[k] += V[(size_t)k * M3 + a] * b0 + V[(size_t)k * M3 + M + a] * b1 +
                V[(size_t)k * M3 + 2 * M + a] * b2;
  }
  double s[6];
  for (int k = 0; k < 6; ++k) s[k] = block_sum(acc[k], red);
  if (threadIdx.x == 0) {
    for (int c = 0; c < 3; ++c) {
      vw[6 * i + c] = R[3 * c] * s[0] + R[3 * c + 1] * s[1] + R[3 * c + 2] * s[2];
      vw[6 * i + 3 + c] = R[3 * c] * s[3] + R[3 * c + 1] * s[4] + R[3 * c + 2] * s[5];
    }
  }
}

hipError_t launch_velocity_self(int n, int M, const int* sid, const double* V0, const double* Rm,
                                const double* sig, double* vw_self, hipStream_t st) {
  k_velocity_self<<<n, 256, 0, st>>>(n, M, sid, V0, Rm, sig, vw_self);
  return hipGetLastError();
}

// VW = (mom_far[0:3]/|Gamma| + self, tau_lab^{-1} mom_far[3:6] + self)   (§3.3)
__global__ void k_velocity_final(int n, const double* mom, const double* vws,
                                 const double* tauinv_lab, const double* area_b, double* VW) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* m = mom + 6 * i;
  const double* ti = tauinv_lab + 9 * i;
  const double ia = 1.0 / area_b[i];
  for (int c = 0; c < 3; ++c) {
    VW[6 * i + c] = m[c] * ia + vws[6 * i + c];
    VW[6 * i + 3 + c] = ti[3 * c] * m[3] + ti[3 * c + 1] * m[4] + ti[3 * c + 2] * m[5] +
                        vws[6 * i + 3 + c];
  }
}

hipError_t launch_velocity_final(int n, const double* mom_far, const double* vw_self,
                                 const double* tauinv_lab, const double* area_b, double* VW,
                                 hipStream_t st) {
  k_velocity_final<<<(n + 63) / 64, 64, 0, st>>>(n, mom_far, vw_self, tauinv_lab, area_b, VW);
  return hipGetLastError();
}

// ---- RK4 on centroids and quaternions (§3.3) ----------------------------------------
// k layout per body: [dc/dt (3), dq/dt (4)].
__device__ inline void qnormalize(double* q) {
  const double s = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) q[k] *= s;
}

__global__ void k_rk_stage(int n, const double* c0, const double* q0, const double* k, double a,
                           double dt, double* cen, double* quat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double q[4];
  const bool first = (a == 0.0);  // the first stage reads no derivative
  for (int c = 0; c < 3; ++c) cen[3 * i + c] = c0[3 * i + c] + (first ? 0.0 : a * dt * k[7 * i + c]);
  for (int c = 0; c < 4; ++c) q[c] = q0[4 * i + c] + (first ? 0.0 : a * dt * k[7 * i + 3 + c]);
  qnormalize(q);
  for (int c = 0; c < 4; ++c) quat[4 * i + c] = q[c];
}

hipError_t launch_rk_stage(int n, const double* c0, const double* q0, const double* k, double a,
                           double dt, double* cen, double* quat, hipStream_t st) {
  k_rk_stage<<<(n + 63) / 64, 64, 0, st>>>(n, c0, q0, k, a, dt, cen, quat);
  return hipGetLastError();
}

// k = (v, 1/2 (0, omega) (x) q); acc = (first ? 0 : acc) + wgt k
__global__ void k_rk_deriv(int n, const double* VW, const double* quat, double* k, double* acc,
                           double wgt, int first) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* v = VW + 6 * i;
  const double* q = quat + 4 * i;
  const double ox = v[3], oy = v[4], oz = v[5];
  double d[7];
  d[0] = v[0];
  d[1] = v[1];
  d[2] = v[2];
  d[3] = 0.5 * (-ox * q[1] - oy * q[2] - oz * q[3]);
  d[4] = 0.5 * (ox * q[0] + oy * q[3] - oz * q[2]);
  d[5] = 0.5 * (-ox * q[3] + oy * q[0] + oz * q[1]);
  d[6] = 0.5 * (ox * q[2] - oy * q[1] + oz * q[0]);
  for (int c = 0; c < 7; ++c) {
    k[7 * i + c] = d[c];
    acc[7 * i + c] = (first ? 0.0 : acc[7 * i + c]) + wgt * d[c];
  }
}

hipError_t launch_rk_deriv(int n, const double* VW, const double* quat, double* k, double* acc,
                           double wgt, int first, hipStream_t st) {
  k_rk_deriv<<<(n + 63) / 64, 64, 0, st>>>(n, VW, quat, k, acc, wgt, first);
  return hipGetLastError();
}

__global__ void k_rk_final(int n, const double* c0, const double* q0, const double* acc, double dt,
                           double* cen, double* quat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double q[4];
  for (int c = 0; c < 3; ++c) cen[3 * i + c] = c0[3 * i + c] + dt / 6.0 * acc[7 * i + c];
  for (int c = 0; c < 4; ++c) q[c] = q0[4 * i + c] + dt / 6.0 * acc[7 * i + 3 + c];
  qnormalize(q);
  for (int c = 0; c < 4; ++c) quat[4 * i + c] = q[c];
}

hipError_t launch_rk_final(int n, const double* c0, const double* q0, const double* acc, double dt,
                           double* cen, double* quat, hipStream_t st) {
  k_rk_final<<<(n + 63) / 64, 64, 0, st>>>(n, c0, q0, acc, dt, cen, quat);
  return hipGetLastError();
}

}  // namespace rbm
