// Device helpers shared by the gfx950 kernels of the mobility library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef RBM_PI
#define RBM_PI 3.14159265358979323846
#endif

namespace rbm {

constexpr int kWave = 64;

// Band index of mode (l, m) in B_p (all (l, m) with l <= p except (p, -p)), or -1.
__host__ __device__ inline int band_index(int l, int m, int p) {
  if (l < p) return l * l + l + m;
  if (m == -p) return -1;
  return p * p + (m + p - 1);
}

// Rotated-node chunk of the singular-quadrature kernels (k_singular, k_singular_laplace):
// the largest of 64, 48 and 32 nodes whose LDS lets two workgroups share a CU's 160 KB,
// else 32 (one workgroup per CU).  With two resident workgroups one's node sweep, which
// runs on a single wave, overlaps the other's contraction.  LDS per workgroup in doubles:
// coefficients 3 (p+1)^2, staged harmonics nB (NC+1) (odd row stride), nkw kernel weights
// per node, the Legendre table.
inline size_t singular_lds_bytes(int p, int nc_nodes, int nkw) {
  const size_t nc = (size_t)(p + 1) * (p + 1), nB = (size_t)p * p + 2 * p;
  return (3 * nc + nB * (nc_nodes + 1) + (size_t)nkw * nc_nodes + 2 * nc + 2 * (p + 1)) * sizeof(double);
}
inline int singular_chunk(int p, int nkw) {
  constexpr size_t kLdsPerCu = 160 * 1024;
  for (int n : {64, 48})
    if (2 * singular_lds_bytes(p, n, nkw) <= kLdsPerCu) return n;
  return 32;
}

// Sweep over the normalized associated Legendre functions N_lm P_l^m(x) (no
// Condon-Shortley phase), 0 <= m <= l <= L, with x = cos(theta), s = sin(theta) >= 0.
// For every (l, m) it calls f(l, m, P, Q, D) with Q = P / sin(theta) (pole regular,
// defined for m >= 1, 0 for m = 0) and D = dP/dtheta.  Recurrences:
//   P_mm = sqrt((2m+1)/(2m)) s P_{m-1,m-1},  P_{m+1,m} = sqrt(2m+3) x P_mm,
//   P_lm = a (x P_{l-1,m} - b P_{l-2,m}), a = sqrt((4l^2-1)/(l^2-m^2)),
//   b = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)); D follows by differentiating them in theta
//   (dx/dtheta = -s), with D_mm = m x Q_mm.
//
// The recurrence coefficients depend only on (l, m).  With `tab` == nullptr they are
// computed inline; otherwise tab holds legendre_table() for this L.
__device__ __forceinline__ int legendre_table_size(int L) { return 2 * (L + 1) * (L + 1) + 2 * (L + 1); }

// tab[2*(l*(L+1)+m)] = a_lm, tab[2*(l*(L+1)+m)+1] = b_lm (l >= m+2);
// tab[2*(L+1)^2 + 2m] = sqrt((2m+1)/(2m)), tab[2*(L+1)^2 + 2m + 1] = sqrt(2m+3).
__device__ inline void legendre_table(int L, double* tab, int tid, int nt) {
  const int n2 = (L + 1) * (L + 1);
  for (int i = tid; i < n2; i += nt) {
    const int l = i / (L + 1), m = i % (L + 1);
    double a = 0.0, b = 0.0;
    if (l >= m + 2) {
      a = sqrt((4.0 * l * l - 1.0) / (double)(l * l - m * m));
      b = sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
    }
    tab[2 * i] = a;
    tab[2 * i + 1] = b;
  }
  for (int m = tid; m <= L; m += nt) {
    tab[2 * n2 + 2 * m] = m > 0 ? sqrt((2.0 * m + 1.0) / (2.0 * m)) : 0.0;
    tab[2 * n2 + 2 * m + 1] = sqrt(2.0 * m + 3.0);
  }
}

template <class F>
__device__ __forceinline__ void legendre_sweep(int L, double x, double s, F&& f,
                                               const double* tab = nullptr) {
  double pmm = 0.28209479177387814347;  // 1/sqrt(4 pi)
  double qmm = 0.0;
  const int n2 = (L + 1) * (L + 1);
  for (int m = 0; m <= L; ++m) {
    if (m > 0) {
      const double c = tab ? tab[2 * n2 + 2 * m] : sqrt((2.0 * m + 1.0) / (2.0 * m));
      qmm = c * pmm;
      pmm = c * s * pmm;
    }
    double p0 = pmm, q0 = qmm, d0 = m * x * qmm;
    f(m, m, p0, q0, d0);
    if (m < L) {
      const double c = tab ? tab[2 * n2 + 2 * m + 1] : sqrt(2.0 * m + 3.0);
      double p1 = c * x * p0, q1 = c * x * q0, d1 = c * (x * d0 - s * p0);
      f(m + 1, m, p1, q1, d1);
      for (int l = m + 2; l <= L; ++l) {
        double a, b;
        if (tab) {
          a = tab[2 * (l * (L + 1) + m)];
          b = tab[2 * (l * (L + 1) + m) + 1];
        } else {
          a = sqrt((4.0 * l * l - 1.0) / (double)(l * l - m * m));
          b = sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
        }
        const double p2 = a * (x * p1 - b * p0);
        const double q2 = a * (x * q1 - b * q0);
        const double d2 = a * (x * d1 - s * p1 - b * d0);
        f(l, m, p2, q2, d2);
        p0 = p1; p1 = p2; q0 = q1; q1 = q2; d0 = d1; d1 = d2;
      }
    }
  }
}

// The columns m = r, 7 - r, 8 + r, 15 - r, ... (r in 0..3) of legendre_sweep, for four
// lanes sharing one point: every lane gets about a quarter of the (l, m) terms, and each
// value is formed by the same operations in the same order as in legendre_sweep (the
// diagonal P_mm, Q_mm are carried through the columns a lane skips).  Needs the table.
template <class F>
__device__ __forceinline__ void legendre_columns4(int L, int r, double x, double s, F&& f,
                                                  const double* tab) {
  double pmm = 0.28209479177387814347;  // 1/sqrt(4 pi)
  double qmm = 0.0;
  const int n2 = (L + 1) * (L + 1);
  int mm = 0;  // pmm, qmm belong to column mm
  for (int k = 0;; ++k) {
    const int m = (k & 1) ? 4 * k + 3 - r : 4 * k + r;
    if (m > L) break;
    for (; mm < m; ++mm) {
      const double c = tab[2 * n2 + 2 * (mm + 1)];
      qmm = c * pmm;
      pmm = c * s * pmm;
    }
    double p0 = pmm, q0 = qmm, d0 = m * x * qmm;
    f(m, m, p0, q0, d0);
    if (m < L) {
      const double c = tab[2 * n2 + 2 * m + 1];
      double p1 = c * x * p0, q1 = c * x * q0, d1 = c * (x * d0 - s * p0);
      f(m + 1, m, p1, q1, d1);
      for (int l = m + 2; l <= L; ++l) {
        const double a = tab[2 * (l * (L + 1) + m)];
        const double b = tab[2 * (l * (L + 1) + m) + 1];
        const double p2 = a * (x * p1 - b * p0);
        const double q2 = a * (x * q1 - b * q0);
        const double d2 = a * (x * d1 - s * p1 - b * d0);
        f(l, m, p2, q2, d2);
        p0 = p1; p1 = p2; q0 = q1; q1 = q2; d0 = d1; d1 = d2;
      }
    }
  }
}

// Rotation matrix (row-major) of a unit quaternion (w, x, y, z), body -> lab.
__host__ __device__ inline void quat_to_rot(const double* q, double* R) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  const double nrm = sqrt(w * w + x * x + y * y + z * z);
  w /= nrm; x /= nrm; y /= nrm; z /= nrm;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

__host__ __device__ inline void inv3(const double* A, double* B) {
  const double c00 = A[4] * A[8] - A[5] * A[7];
  const double c01 = A[5] * A[6] - A[3] * A[8];
  const double c02 = A[3] * A[7] - A[4] * A[6];
  const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  const double id = 1.0 / det;
  B[0] = c00 * id; B[1] = (A[2] * A[7] - A[1] * A[8]) * id; B[2] = (A[1] * A[5] - A[2] * A[4]) * id;
  B[3] = c01 * id; B[4] = (A[0] * A[8] - A[2] * A[6]) * id; B[5] = (A[2] * A[3] - A[0] * A[5]) * id;
  B[6] = c02 * id; B[7] = (A[1] * A[6] - A[0] * A[7]) * id; B[8] = (A[0] * A[4] - A[1] * A[3]) * id;
}

// Deterministic block-wide sum of one double per thread (blockDim.x a multiple of 64,
// <= 1024).  `sh` must hold blockDim.x/64 doubles.  Result valid in every thread.
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) t += sh[i];
  return t;
}

}  // namespace rbm
