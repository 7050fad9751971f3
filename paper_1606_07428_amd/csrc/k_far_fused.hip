// The float64 traction and Stokeslet sums of one density in one pass over the source pairs:
//
//   y_a = -(3/4pi) sum_{b not on body(a)} d (d.N_a)(d.q_b)/|d|^5          (traction, §2.1)
//   u_a =  (1/8pi) sum_{b not on body(a)} [q_b/|d| + d (d.q_b)/|d|^3]     (Stokeslet, §2.1)
//
// d = X_a - X_b, q_b = w_b sigma_b.  The solve needs both for sigma = rho + mu at its last
// refinement: the traction sum gives the float64 residual b - A mu (§2.3) and the Stokeslet
// sum the velocities (§3.3).  Per pair the two share d, |d|^2, d.q and the hardware
// estimate y of |d|^-1 with e = 1 - |d|^2 y^2: the traction takes y^5 (1 + 5e/2 + 35e^2/8)
// and the Stokeslet the corrected |d|^-1 = y (1 + e/2 + 3e^2/8), 35 float64 operations and
// one v_rsq_f64 instead of 24 + 22 and two.  Same mapping as the all-pairs kernel: one
// target per lane, wave-uniform source loads (scalar loads into SGPRs), the source range
// split over blockIdx.y with long chunks first, same-body pairs masked by index range; two
// partial-sum arrays, combined like the kernel's.
#include "common.h"
#include "kernels.h"
#include "far_plan.h"
#include "pair.h"

namespace rbm {

__device__ __forceinline__ void pair_ts(double xa, double ya, double za, double nx, double ny, double nz,
                                        const Src8<double>& s, double& tx, double& ty, double& tz,
                                        double& ux, double& uy, double& uz) {
  const double dx = xa - s.v[0], dy = ya - s.v[1], dz = za - s.v[2];
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double dq = dx * s.v[3] + dy * s.v[4] + dz * s.v[5];
  const double y = __builtin_amdgcn_rsq(r2);
  const double y2 = y * y;
  const double e = fma(-r2, y2, 1.0);
  // traction: (2/5) (d.N)(d.q) |d|^-5, the 5/2 applied with the final scale
  const double dn = dx * nx + dy * ny + dz * nz;
  const double f = ((dn * dq) * y) * (y2 * y2) * fma(e, fma(e, 1.75, 1.0), 0.4);
  tx = fma(f, dx, tx);
  ty = fma(f, dy, ty);
  tz = fma(f, dz, tz);
  // Stokeslet: (q + u d) / |d| with u = (d.q) / |d|^2
  const double ri = fma(y * e, fma(e, 0.375, 0.5), y);
  const double u = dq * (ri * ri);
  ux = fma(ri, fma(u, dx, s.v[3]), ux);
  uy = fma(ri, fma(u, dy, s.v[4]), uy);
  uz = fma(ri, fma(u, dz, s.v[5]), uz);
}

__global__ __launch_bounds__(256) void k_far_ts(int N, int M, const double* __restrict__ tx,
                                                const double* __restrict__ tn,
                                                const Src8<double>* __restrict__ src,
                                                double* __restrict__ part_t, double* __restrict__ part_u,
                                                int s1, int c1, int c2) {
  const int split = blockIdx.y;
  const int b0 = split < s1 ? split * c1 : s1 * c1 + (split - s1) * c2;
  const int b1 = min(N, b0 + (split < s1 ? c1 : c2));
  const int a0 = blockIdx.x * 256 + (int)threadIdx.x;
  const int a = min(a0, N - 1);
  const double xa = tx[a], ya = tx[N + a], za = tx[2 * N + a];
  const double nx = tn[a], ny = tn[N + a], nz = tn[2 * N + a];
  double t0 = 0, t1 = 0, t2 = 0, u0 = 0, u1 = 0, u2 = 0;
  const int blo_t = (a / M) * M;
  const int base = blockIdx.x * 256;
  const int last = min(N, base + 256) - 1;
  const int blo = (base / M) * M, bhi = (last / M + 1) * M;
  auto fast = [&](int s0, int e) {
    int b = s0;
    for (; b + 4 <= e; b += 4) {
      const Src8<double> q0 = src[b], q1 = src[b + 1], q2 = src[b + 2], q3 = src[b + 3];
      pair_ts(xa, ya, za, nx, ny, nz, q0, t0, t1, t2, u0, u1, u2);
      pair_ts(xa, ya, za, nx, ny, nz, q1, t0, t1, t2, u0, u1, u2);
      pair_ts(xa, ya, za, nx, ny, nz, q2, t0, t1, t2, u0, u1, u2);
      pair_ts(xa, ya, za, nx, ny, nz, q3, t0, t1, t2, u0, u1, u2);
    }
    for (; b < e; ++b) pair_ts(xa, ya, za, nx, ny, nz, src[b], t0, t1, t2, u0, u1, u2);
  };
  fast(b0, min(b1, blo));
  {
    const int s0 = max(b0, blo), e = min(b1, bhi);
    for (int b = s0; b < e; ++b) {
      double p0 = 0, p1 = 0, p2 = 0, q0 = 0, q1 = 0, q2 = 0;
      pair_ts(xa, ya, za, nx, ny, nz, src[b], p0, p1, p2, q0, q1, q2);
      const bool other = (unsigned)(b - blo_t) >= (unsigned)M;
      t0 += other ? p0 : 0.0;
      t1 += other ? p1 : 0.0;
      t2 += other ? p2 : 0.0;
      u0 += other ? q0 : 0.0;
      u1 += other ? q1 : 0.0;
      u2 += other ? q2 : 0.0;
    }
  }
  fast(max(b0, bhi), b1);
  if (a0 < N) {
    const double st = (-3.0 / (4.0 * RBM_PI)) * 2.5, su = 1.0 / (8.0 * RBM_PI);
    double* ot = part_t + (size_t)split * 3 * N;
    double* ou = part_u + (size_t)split * 3 * N;
    ot[a0] = st * t0;
    ot[N + a0] = st * t1;
    ot[2 * (size_t)N + a0] = st * t2;
    ou[a0] = su * u0;
    ou[N + a0] = su * u1;
    ou[2 * (size_t)N + a0] = su * u2;
  }
}

hipError_t launch_far_ts(int N, int M, const double* tx, const double* nrm, const void* src, double* part_t,
                         double* part_u, int nsplit, hipStream_t st) {
  if (N <= 0 || nsplit < 1) return hipErrorInvalidValue;
  const FarChunks fc = far_chunks(N, nsplit);
  dim3 grid((N + 255) / 256, nsplit);
  k_far_ts<<<grid, 256, 0, st>>>(N, M, tx, nrm, reinterpret_cast<const Src8<double>*>(src), part_t, part_u,
                                 fc.s1, fc.c1, fc.c2);
  return hipGetLastError();
}

}  // namespace rbm
