// All-pairs sums between bodies (the far part of the matvec and of the velocity
// evaluation), replacing the Stokes FMM of §3.1 by a direct tiled sum on one GPU.
//
//   traction  (kind 0): y_a = -(3/4pi) sum_{b not on body(a)} d (d.N_a)(d.q_b)/|d|^5
//   Stokeslet (kind 1): u_a = (1/8pi) sum_{b not on body(a)} [q_b/|d| + d (d.q_b)/|d|^3]
//   d = X_a - X_b, q_b = w_b sigma_b (smooth quadrature of §3); the 1/eta of the
//   Stokeslet is applied by the caller.
//
// Mapping on gfx950: each lane owns TPL targets (position, normal, accumulators in
// VGPRs).  Sources are packed AoS, 8 values per source (x, y, z, qx, qy, qz, 0, 0),
// and every lane of a wave reads the same source, so the loads are wave-uniform
// and the compiler issues them as scalar loads: source data arrive in SGPRs and
// feed the VALU directly, with no LDS traffic and no VGPRs spent on sources.  The
// source range is split over blockIdx.y so that small problems still fill the 256
// CUs; partial sums go to part[split][3][N] and are combined deterministically.
// Workgroups are dispatched split by split, so the last splits are the ones running
// while the grid drains and SIMDs fall below full occupancy: the first half of the
// splits take long chunks (85% of the sources) and the second half share the rest in
// short ones, which shortens that ragged end at the same number of slots.
// Same-body pairs are excluded by index range: only the source segment that
// overlaps the block's body range takes the per-lane masked path.
#include "common.h"
#include "kernels.h"
#include "far_plan.h"
#include "pair.h"

namespace rbm {

// Constant factor of each kernel's sum: traction -3/(4pi), Stokeslet 1/(8pi) (the 1/eta
// is applied by the caller), Laplace normal derivative -1/(4pi), Laplace single layer 1/(4pi).
__host__ __device__ constexpr double kind_scale(int kind) {
  return kind == 0 ? -3.0 / (4.0 * RBM_PI)
                   : kind == 1 ? 1.0 / (8.0 * RBM_PI) : kind == 2 ? -1.0 / (4.0 * RBM_PI) : 1.0 / (4.0 * RBM_PI);
}

template <typename T, int KIND, int TPL>
__global__ __launch_bounds__(256) void k_far(int N, int M, const T* __restrict__ tx,
                                             const T* __restrict__ tn,
                                             const Src8<T>* __restrict__ src,
                                             double* __restrict__ part, int s1, int c1, int c2) {
  // splits below s1 cover c1 sources each, the rest c2; a split past the end is empty
  // (b0 >= b1) and writes zeros to its slot
  const int split = blockIdx.y;
  const int b0 = split < s1 ? split * c1 : s1 * c1 + (split - s1) * c2;
  const int b1 = min(N, b0 + (split < s1 ? c1 : c2));
  const int base = blockIdx.x * (256 * TPL);
  T xa[TPL], ya[TPL], za[TPL], nx[TPL], ny[TPL], nz[TPL], ax[TPL], ay[TPL], az[TPL];
  int blo_t[TPL];
#pragma unroll
  for (int u = 0; u < TPL; ++u) {
    const int a = min(base + u * 256 + (int)threadIdx.x, N - 1);
    xa[u] = tx[a];
    ya[u] = tx[N + a];
    za[u] = tx[2 * N + a];
    if (KIND == 0 || KIND == 2) {
      nx[u] = tn[a];
      ny[u] = tn[N + a];
      nz[u] = tn[2 * N + a];
    } else {
      nx[u] = ny[u] = nz[u] = 0;
    }
    ax[u] = ay[u] = az[u] = 0;
    blo_t[u] = (a / M) * M;
  }
  const int last = min(N, base + 256 * TPL) - 1;
  const int blo = (base / M) * M, bhi = (last / M + 1) * M;
  auto fast = [&](int s0, int e) {
    int b = s0;
    if (sizeof(T) == 4 && b + 4 <= e) {
      // fp32: the next four sources are loaded while the current four are used
      Src8<T> cur[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) cur[k] = src[b + k];
      for (; b + 8 <= e; b += 4) {
        Src8<T> nxt[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) nxt[k] = src[b + 4 + k];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int u = 0; u < TPL; ++u)
            Pair<T, KIND>::add(xa[u], ya[u], za[u], nx[u], ny[u], nz[u], cur[k], ax[u], ay[u], az[u]);
#pragma unroll
        for (int k = 0; k < 4; ++k) cur[k] = nxt[k];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int u = 0; u < TPL; ++u)
          Pair<T, KIND>::add(xa[u], ya[u], za[u], nx[u], ny[u], nz[u], cur[k], ax[u], ay[u], az[u]);
      b += 4;
    }
    for (; b + 4 <= e; b += 4) {
      const Src8<T> q0 = src[b], q1 = src[b + 1], q2 = src[b + 2], q3 = src[b + 3];
#pragma unroll
      for (int u = 0; u < TPL; ++u) {
        Pair<T, KIND>::add(xa[u], ya[u], za[u], nx[u], ny[u], nz[u], q0, ax[u], ay[u], az[u]);
        Pair<T, KIND>::add(xa[u], ya[u], za[u], nx[u], ny[u], nz[u], q1, ax[u], ay[u], az[u]);
        Pair<T, KIND>::add(xa[u], ya[u], za[u], nx[u], ny[u], nz[u], q2, ax[u], ay[u], az[u]);
        Pair<T, KIND>::add(xa[u], ya[u], za[u], nx[u], ny[u], nz[u], q3, ax[u], ay[u], az[u]);
      }
    }
    for (; b < e; ++b) {
      const Src8<T> q0 = src[b];
#pragma unroll
      for (int u = 0; u < TPL; ++u)
        Pair<T, KIND>::add(xa[u], ya[u], za[u], nx[u], ny[u], nz[u], q0, ax[u], ay[u], az[u]);
    }
  };
  // fast segment before the block's bodies
  fast(b0, min(b1, blo));
  // masked segment overlapping the block's bodies
  {
    const int s0 = max(b0, blo), e = min(b1, bhi);
    for (int b = s0; b < e; ++b) {
      const Src8<T> s = src[b];
#pragma unroll
      for (int u = 0; u < TPL; ++u) {
        T px = 0, py = 0, pz = 0;
        Pair<T, KIND>::add(xa[u], ya[u], za[u], nx[u], ny[u], nz[u], s, px, py, pz);
        const bool other = (unsigned)(b - blo_t[u]) >= (unsigned)M;
        ax[u] += other ? px : (T)0;
        ay[u] += other ? py : (T)0;
        az[u] += other ? pz : (T)0;
      }
    }
  }
  // fast segment after the block's bodies
  fast(max(b0, bhi), b1);
  const double scale = kind_scale(KIND) * Pair<T, KIND>::kPost;
#pragma unroll
  for (int u = 0; u < TPL; ++u) {
    const int a = base + u * 256 + (int)threadIdx.x;
    if (a < N) {
      double* o = part + (size_t)split * 3 * N;
      o[a] = scale * (double)ax[u];
      o[N + a] = scale * (double)ay[u];
      o[2 * (size_t)N + a] = scale * (double)az[u];
    }
  }
}

constexpr int kTPL = 1;

template <typename T>
hipError_t launch_far(int kind, int N, int M, const T* tx, const T* nrm, const void* src,
                      double* part, int nsplit, hipStream_t st) {
  if (N <= 0 || nsplit < 1) return hipErrorInvalidValue;
  const FarChunks fc = far_chunks(N, nsplit);
  dim3 grid((N + 256 * kTPL - 1) / (256 * kTPL), nsplit);
  const Src8<T>* s = reinterpret_cast<const Src8<T>*>(src);
  if (kind >= 2) {
    // the scalar Laplace sums of the magnetostatic problem (float64 only)
    if constexpr (sizeof(T) == 8) {
      if (kind == 2)
        k_far<T, 2, kTPL><<<grid, 256, 0, st>>>(N, M, tx, nrm, s, part, fc.s1, fc.c1, fc.c2);
      else
        k_far<T, 3, kTPL><<<grid, 256, 0, st>>>(N, M, tx, nrm, s, part, fc.s1, fc.c1, fc.c2);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  if (kind == 0)
    k_far<T, 0, kTPL><<<grid, 256, 0, st>>>(N, M, tx, nrm, s, part, fc.s1, fc.c1, fc.c2);
  else
    k_far<T, 1, kTPL><<<grid, 256, 0, st>>>(N, M, tx, nrm, s, part, fc.s1, fc.c1, fc.c2);
  return hipGetLastError();
}

template hipError_t launch_far<double>(int, int, int, const double*, const double*, const void*,
                                       double*, int, hipStream_t);
template hipError_t launch_far<float>(int, int, int, const float*, const float*, const void*,
                                      double*, int, hipStream_t);

// q_g = W_g * z_g (z rotated to the lab frame first when given in body frames).
template <typename T>
__global__ void k_pack(int N, int M, const double* __restrict__ X, const double* __restrict__ W,
                       const double* __restrict__ Rm, const double* __restrict__ z, int z_is_body,
                       double* __restrict__ zlab, Src8<T>* __restrict__ src) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  double v0 = z[g], v1 = z[N + g], v2 = z[2 * (size_t)N + g];
  if (z_is_body) {
    const double* R = Rm + 9 * (g / M);
    const double a0 = R[0] * v0 + R[1] * v1 + R[2] * v2;
    const double a1 = R[3] * v0 + R[4] * v1 + R[5] * v2;
    const double a2 = R[6] * v0 + R[7] * v1 + R[8] * v2;
    v0 = a0; v1 = a1; v2 = a2;
  }
  if (zlab) {
    zlab[g] = v0;
    zlab[N + g] = v1;
    zlab[2 * (size_t)N + g] = v2;
  }
  const double w = W ? W[g] : 1.0;
  Src8<T> s;
  s.v[0] = (T)X[g];
  s.v[1] = (T)X[N + g];
  s.v[2] = (T)X[2 * (size_t)N + g];
  s.v[3] = (T)(w * v0);
  s.v[4] = (T)(w * v1);
  s.v[5] = (T)(w * v2);
  s.v[6] = 0;
  s.v[7] = 0;
  src[g] = s;
}

template <typename T>
hipError_t launch_pack_sources(int N, int M, const double* X, const double* W, const double* Rm,
                               const double* z, int z_is_body, double* z_lab_out, void* src,
                               hipStream_t st) {
  k_pack<T><<<(N + 255) / 256, 256, 0, st>>>(N, M, X, W, Rm, z, z_is_body, z_lab_out,
                                             reinterpret_cast<Src8<T>*>(src));
  return hipGetLastError();
}

template hipError_t launch_pack_sources<double>(int, int, const double*, const double*,
                                                const double*, const double*, int, double*, void*,
                                                hipStream_t);
template hipError_t launch_pack_sources<float>(int, int, const double*, const double*,
                                               const double*, const double*, int, double*, void*,
                                               hipStream_t);

// out = ca*a + cb*(R_i b_body) + cp*sum_s part[s]   (fixed summation order); out may be
// a, not b_body.  The slot sum over the split is the memory-bound part.
// 64 outputs per workgroup: wave q of the four sums slots s = q, q + 4, ... of them in
// increasing s (each load a coalesced 512-byte segment), and wave 0 adds the four sums as
// (s0 + s1) + (s2 + s3), so every output is the same as with one thread and four
// round-robin accumulators, with four times the loads in flight.
__global__ __launch_bounds__(256) void k_combine(int N, int M, int nsplit, const double* __restrict__ part,
                                                 double cp, const double* a, double ca,
                                                 const double* __restrict__ bb,
                                                 const double* __restrict__ Rm, double cb, double* out) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int t = blockIdx.x * 64 + lane;
  const bool act = t < 3 * N;
  if (part) {
    double sq = 0.0;
    if (act) {
      const size_t stride = 3 * (size_t)N;
      const double* p = part + t;
      for (int s = q; s < nsplit; s += 4) sq += p[(size_t)s * stride];
    }
    red[q][lane] = sq;
  }
  __syncthreads();
  if (q != 0 || !act) return;
  const int c = t / N, g = t - c * N;
  double v = 0.0;
  if (part) v = cp * ((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]));
  if (bb) {
    const double* R = Rm + 9 * (g / M) + 3 * c;
    v += cb * (R[0] * bb[g] + R[1] * bb[N + g] + R[2] * bb[2 * (size_t)N + g]);
  }
  if (a) v += ca * a[t];
  out[t] = v;
}

hipError_t launch_combine(int N, int M, int nsplit, const double* part, double cp,
                          const double* a, double ca, const double* b_body, const double* Rm,
                          double cb, double* out, hipStream_t st) {
  k_combine<<<(3 * N + 63) / 64, 256, 0, st>>>(N, M, nsplit, part, cp, a, ca, b_body, Rm, cb, out);
  return hipGetLastError();
}

}  // namespace rbm
