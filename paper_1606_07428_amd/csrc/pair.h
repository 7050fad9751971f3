// Pair arithmetic of the smooth-rule sums between bodies (§2.1, §3, §4): the packed
// source record and the contribution of one source to one target for the traction (kind
// 0), Stokeslet (1), Laplace normal-derivative (2) and Laplace single-layer (3) kernels,
// shared by the all-pairs sum (k_far.hip) and the near-singular correction (k_near.hip).
#pragma once
#include "common.h"

namespace rbm {

template <typename T> struct alignas(8 * sizeof(T)) Src8 { T v[8]; };

// 1/sqrt(x) in float64: hardware estimate plus one third-order correction
// y <- y + y e (1/2 + 3/8 e), e = 1 - x y^2 (error cubes each step).  Used by the
// Stokeslet sum, which needs |r|^-1 and |r|^-3.
__device__ __forceinline__ double rsqrt_t(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double t = x * y;
  const double e = fma(-t, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }

// |r|^-5 from r2 = |r|^2.  float64: with the hardware estimate y (relative error
// < 2^-24 on gfx950) and e = 1 - r2 y^2, |r|^-5 = y^5 (1 - e)^(-5/2)
// = y^5 (1 + 5e/2 + 35e^2/8 + O(e^3)), accurate to float64 rounding with the two terms.
__device__ __forceinline__ double rinv5_t(double r2) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double y2 = y * y;
  const double e = fma(-r2, y2, 1.0);
  const double y5 = y2 * y2 * y;
  // 1 + 5e/2 + 35e^2/8 = 1 + (5e/2)(1 + 7e/4): every step has at most one constant that
  // is not an inline operand, so no constant has to be rebuilt in registers per pair
  return y5 * fma(2.5 * e, fma(e, 1.75, 1.0), 1.0);
}
__device__ __forceinline__ float rinv5_t(float r2) {
  const float y = __builtin_amdgcn_rsqf(r2);
  const float y2 = y * y;
  return y2 * y2 * y;
}

// (2/5) w |r|^-5, the traction pair factor over 5/2.  float64: the two-term correction
// of rinv5_t, 1 + 5e/2 + 35e^2/8, taken as (5/2)(2/5 + e (1 + 7e/4)) with w folded into
// y^5 first and the 5/2 left to the caller's final scale (Pair::kPost): every step then
// has at most one constant that is not an inline operand, and the pair costs one
// multiply fewer than w * rinv5_t(r2).  float32 has no correction and no post factor.
__device__ __forceinline__ double w_rinv5_t(double w, double r2) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double y2 = y * y;
  const double e = fma(-r2, y2, 1.0);
  const double wy5 = (w * y) * (y2 * y2);
  return wy5 * fma(e, fma(e, 1.75, 1.0), 0.4);
}
__device__ __forceinline__ float w_rinv5_t(float w, float r2) { return w * rinv5_t(r2); }

// (2/3) w |r|^-3 for the Laplace normal derivative: y^3 (1 - e)^(-3/2) = y^3 (1 + 3e/2 +
// 15e^2/8 + O(e^3)) = (3/2) y^3 (2/3 + e (1 + 5e/4)), the 3/2 left to the caller's final
// scale (Pair::kPost), so that every step has at most one constant that is not an
// inline operand.
__device__ __forceinline__ double w_rinv3_t(double w, double r2) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double y2 = y * y;
  const double e = fma(-r2, y2, 1.0);
  const double wy3 = (w * y) * y2;
  return wy3 * fma(e, fma(e, 1.25, 1.0), 2.0 / 3.0);
}

template <typename T, int KIND>
struct Pair {
  // factor the caller applies to the accumulated sums with the kernel's constant
  static constexpr double kPost = sizeof(T) != 8 ? 1.0 : KIND == 0 ? 2.5 : KIND == 2 ? 1.5 : 1.0;
  __device__ __forceinline__ static void add(T xa, T ya, T za, T nx, T ny, T nz,
                                             const Src8<T>& s, T& ax, T& ay, T& az) {
    const T dx = xa - s.v[0], dy = ya - s.v[1], dz = za - s.v[2];
    const T r2 = dx * dx + dy * dy + dz * dz;
    const T dq = dx * s.v[3] + dy * s.v[4] + dz * s.v[5];
    if (KIND == 0) {
      const T dn = dx * nx + dy * ny + dz * nz;
      const T f = w_rinv5_t(dn * dq, r2);
      ax += f * dx;
      ay += f * dy;
      az += f * dz;
    } else if (KIND == 1) {
      // q/|d| + d (d.q)/|d|^3 = (q + u d)/|d| with u = (d.q)/|d|^2: two fused
      // multiply-adds per component
      const T ri = rsqrt_t(r2);
      const T u = dq * (ri * ri);
      ax += ri * (s.v[3] + u * dx);
      ay += ri * (s.v[4] + u * dy);
      az += ri * (s.v[5] + u * dz);
    } else if (KIND == 2) {
      // Laplace, normal derivative at the target of the single layer: (d.N_a) q_b / |d|^3
      // (float64 only; the sum carries the factor 2/3 that kPost undoes)
      ax += w_rinv3_t((dx * nx + dy * ny + dz * nz) * s.v[3], r2);
    } else {
      // Laplace single layer: q_b / |d|
      ax += s.v[3] * rsqrt_t(r2);
    }
  }
};

}  // namespace rbm
