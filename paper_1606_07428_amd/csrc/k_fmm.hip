// Fast multipole evaluation of the off-body traction sum, an O(N) equivalent of the FMM
// the paper uses for the far field (§3.1).
//
// Stokes through four harmonic potentials: phi_j = sum q_j / |x - y| (j = 1..3) and
// psi = sum ((y - c).q) / |x - y| with c the centre of the box that carries the
// expansion.  At a target x in a leaf with centre c, s = x - c:
//   traction = (1/4pi) [ (div phi) N + (H(psi) - s_j H(phi_j)) N ]      (H: Hessian),
// which is the traction [-pI + grad u + grad u^T] N of the Stokeslet field (§2.1).
//
// Complex solid harmonics with factorial normalisation (no Condon-Shortley phase):
//   R_n^m = r^n P_n^m e^{i m phi} / (n+m)!,  I_n^m = (n-m)! P_n^m e^{i m phi} / r^{n+1},
//   X_n^{-m} = (-1)^m conj(X_n^m); expansions store m >= 0 only, coefficient n(n+1)/2 + m,
//   the four densities of a coefficient adjacent.
// Multipole about c: M_n^m = sum q conj(R_n^m(y - c)); local about c: phi = sum L conj(R(x - c)).
//   M2M (child c1 -> parent c2): M'_n^m = sum_{k,l} M_k^l conj(R_{n-k}^{m-l}(c1 - c2))
//   M2L (a = c_t - c_s):          L_k^l  = (-1)^k sum_{n,m} M_n^m I_{n+k}^{m+l}(a)
//   L2L (parent c -> child c'):   L'_j^i = sum_{k,l} L_k^l conj(R_{k-j}^{l-i}(c' - c))
//   d/dz of a local expansion shifts L_{k+1}^l, (d/dx + i d/dy) shifts L_{k+1}^{l+1}.
// Moving the psi expansion from centre c to c' adds (c - c') . (phi_1, phi_2, phi_3)
// expansions: before the translation in M2M and L2L, after it (by linearity) in M2L.
//
// Tree: uniform octree over the bounding cube of the points (side D, corner lo), leaf
// level L with leaf width >= the largest body diameter, so the nodes of one body lie in
// the same or adjacent leaves: every same-body pair falls in the direct near field,
// where it is skipped; none goes through an expansion.  Near field: the 27 adjacent
// leaves.  Interaction lists at levels 2..L: boxes not adjacent whose parents are.
#include "common.h"
#include "kernels.h"
#include "pair.h"

namespace rbm {

constexpr int kFmmPMax = kFmmMaxOrder;
constexpr int kFmmKc = (kFmmPMax + 1) * (kFmmPMax + 2) / 2;          // coefficients, m >= 0
constexpr int kFmmLeafMax = kFmmLeafCap;                              // points per leaf
constexpr int kFmmVecs = 343;                                         // displacements in [-3, 3]^3

template <typename T> struct Cx { T re, im; };

template <typename T>
__device__ __forceinline__ void cfma(Cx<T>& acc, Cx<T> a, Cx<T> b) {
  acc.re = fma(a.re, b.re, fma(-a.im, b.im, acc.re));
  acc.im = fma(a.re, b.im, fma(a.im, b.re, acc.im));
}

__host__ __device__ __forceinline__ int tri(int n, int m) { return n * (n + 1) / 2 + m; }

// Entry (n, m) of a half table, any sign of m: X_n^{-m} = (-1)^m conj(X_n^m).
template <typename T>
__device__ __forceinline__ Cx<T> cget(const Cx<T>* a, int n, int m) {
  if (m >= 0) return a[tri(n, m)];
  const Cx<T> v = a[tri(n, -m)];
  return (m & 1) ? Cx<T>{-v.re, v.im} : Cx<T>{v.re, -v.im};
}

// R_n^m(x, y, z) for 0 <= m <= n <= P into out[tri(n, m)] (conjugated if conj):
//   R_m^m = R_{m-1}^{m-1} (x + iy) / (2m),  R_{m+1}^m = z R_m^m,
//   R_n^m = ((2n - 1) z R_{n-1}^m - r^2 R_{n-2}^m) / ((n - m)(n + m)).
template <typename T, typename S>
__device__ void regular_table(int P, S x, S y, S z, Cx<T>* out, bool conj) {
  const S r2 = x * x + y * y + z * z;
  S dre = 1, dim = 0;
  const S sg = conj ? S(-1) : S(1);
  for (int m = 0; m <= P; ++m) {
    if (m > 0) {
      const S inv = S(1) / S(2 * m);
      const S nre = (dre * x - dim * y) * inv, nim = (dre * y + dim * x) * inv;
      dre = nre;
      dim = nim;
    }
    out[tri(m, m)] = Cx<T>{(T)dre, (T)(sg * dim)};
    if (m + 1 > P) continue;
    S are = dre, aim = dim;            // R_{n-2}
    S bre = z * dre, bim = z * dim;    // R_{n-1}
    out[tri(m + 1, m)] = Cx<T>{(T)bre, (T)(sg * bim)};
    for (int n = m + 2; n <= P; ++n) {
      const S c1 = S(2 * n - 1), inv = S(1) / S((n - m) * (n + m));
      const S vre = (c1 * z * bre - r2 * are) * inv, vim = (c1 * z * bim - r2 * aim) * inv;
      are = bre; aim = bim;
      bre = vre; bim = vim;
      out[tri(n, m)] = Cx<T>{(T)vre, (T)(sg * vim)};
    }
  }
}

// I_n^m(x, y, z) for 0 <= m <= n <= Q into out[n^2 + n + m] and, by I_n^{-m} =
// (-1)^m conj(I_n^m), out[n^2 + n - m] (all m, (Q + 1)^2 entries):
//   I_0^0 = 1/r,  I_m^m = I_{m-1}^{m-1} (2m - 1)(x + iy) / r^2,  I_{m+1}^m = (2m + 1) z I_m^m / r^2,
//   I_n^m = ((2n - 1) z I_{n-1}^m - (n + m - 1)(n - m - 1) I_{n-2}^m) / r^2.
template <typename T>
__device__ void irregular_table(int Q, double x, double y, double z, Cx<T>* out) {
  const double r2 = x * x + y * y + z * z, ir2 = 1.0 / r2;
  double dre = 1.0 / sqrt(r2), dim = 0.0;
  auto put = [&](int n, int m, double re, double im) {
    out[n * n + n + m] = Cx<T>{(T)re, (T)im};
    if (m > 0) out[n * n + n - m] = (m & 1) ? Cx<T>{(T)-re, (T)im} : Cx<T>{(T)re, (T)-im};
  };
  for (int m = 0; m <= Q; ++m) {
    if (m > 0) {
      const double c = (2 * m - 1) * ir2;
      const double nre = (dre * x - dim * y) * c, nim = (dre * y + dim * x) * c;
      dre = nre;
      dim = nim;
    }
    put(m, m, dre, dim);
    if (m + 1 > Q) continue;
    double are = dre, aim = dim;
    double bre = (2 * m + 1) * z * ir2 * dre, bim = (2 * m + 1) * z * ir2 * dim;
    put(m + 1, m, bre, bim);
    for (int n = m + 2; n <= Q; ++n) {
      const double c1 = (2.0 * n - 1.0) * z, c2 = (double)(n + m - 1) * (double)(n - m - 1);
      const double vre = (c1 * bre - c2 * are) * ir2, vim = (c1 * bim - c2 * aim) * ir2;
      are = bre; aim = bim;
      bre = vre; bim = vim;
      put(n, m, vre, vim);
    }
  }
}

// ---------------------------------------------------------------------------------
// Tree construction (float64 coordinates)

// Componentwise min and max of X ([3][N]) into out[6] (one workgroup).
__global__ void __launch_bounds__(1024) k_fmm_bounds(int N, const double* __restrict__ X, double* out) {
  __shared__ double red[6][1024];
  double v[6] = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300};
  for (int i = threadIdx.x; i < N; i += blockDim.x)
    for (int d = 0; d < 3; ++d) {
      const double x = X[(size_t)d * N + i];
      v[d] = fmin(v[d], x);
      v[3 + d] = fmax(v[3 + d], x);
    }
  for (int d = 0; d < 6; ++d) red[d][threadIdx.x] = v[d];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int d = 0; d < 6; ++d)
        red[d][threadIdx.x] = d < 3 ? fmin(red[d][threadIdx.x], red[d][threadIdx.x + s])
                                    : fmax(red[d][threadIdx.x], red[d][threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x < 6) out[threadIdx.x] = red[threadIdx.x][0];
}

__device__ __forceinline__ int leaf_coord(double x, double lo, double w, int nb) {
  const int i = (int)floor((x - lo) / w);
  return i < 0 ? 0 : (i >= nb ? nb - 1 : i);
}

__global__ void k_fmm_count(int N, const double* __restrict__ X, double lox, double loy, double loz,
                            double w, int nb, int* __restrict__ leaf, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int a = leaf_coord(X[i], lox, w, nb);
  const int b = leaf_coord(X[(size_t)N + i], loy, w, nb);
  const int c = leaf_coord(X[2 * (size_t)N + i], loz, w, nb);
  const int id = (c * nb + b) * nb + a;
  leaf[i] = id;
  atomicAdd(cnt + id, 1);
}

// Exclusive scan of cnt[0, nbox) into start[0, nbox]; largest count to *maxcnt.
__global__ void __launch_bounds__(1024) k_fmm_scan(int nbox, const int* __restrict__ cnt,
                                                   int* __restrict__ start, int* __restrict__ maxcnt) {
  __shared__ int part[1024], pmax[1024];
  const int t = threadIdx.x, nt = blockDim.x;
  const int chunk = (nbox + nt - 1) / nt;
  const int b0 = min(nbox, t * chunk), b1 = min(nbox, b0 + chunk);
  int s = 0, mx = 0;
  for (int b = b0; b < b1; ++b) {
    s += cnt[b];
    mx = max(mx, cnt[b]);
  }
  part[t] = s;
  pmax[t] = mx;
  __syncthreads();
  if (t == 0) {
    int run = 0, m = 0;
    for (int i = 0; i < nt; ++i) {
      const int v = part[i];
      part[i] = run;
      run += v;
      m = max(m, pmax[i]);
    }
    start[nbox] = run;
    *maxcnt = m;
  }
  __syncthreads();
  int run = part[t];
  for (int b = b0; b < b1; ++b) {
    start[b] = run;
    run += cnt[b];
  }
}

__global__ void k_fmm_scatter(int N, const int* __restrict__ leaf, const int* __restrict__ start,
                              int* __restrict__ fill, int* __restrict__ perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int b = leaf[i];
  perm[start[b] + atomicAdd(fill + b, 1)] = i;
}

// Order every leaf's segment of perm by point index (the atomic scatter leaves it in
// arbitrary order): rank of each entry = number of smaller entries in the segment.
__global__ void __launch_bounds__(256) k_fmm_sort(const int* __restrict__ start, int* __restrict__ perm) {
  __shared__ int v[kFmmLeafMax];
  const int b = blockIdx.x;
  const int s0 = start[b], n = start[b + 1] - s0;
  if (n <= 1 || n > kFmmLeafMax) return;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v[i] = perm[s0 + i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int x = v[i];
    int r = 0;
    for (int k = 0; k < n; ++k) r += v[k] < x;
    perm[s0 + r] = x;
  }
}

// Sorted geometry: Xs[p] = (x, y, z, body), Ns[p] = (nx, ny, nz, 0) of point perm[p].
__global__ void k_fmm_gather(int N, int M, const int* __restrict__ perm, const double* __restrict__ X,
                             const double* __restrict__ Nn, double4* __restrict__ Xs,
                             double4* __restrict__ Ns) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int i = perm[p];
  Xs[p] = make_double4(X[i], X[(size_t)N + i], X[2 * (size_t)N + i], (double)(i / M));
  Ns[p] = make_double4(Nn[i], Nn[(size_t)N + i], Nn[2 * (size_t)N + i], 0.0);
}

// Points per box one level up: cp[parent] = sum of its eight children's counts.
__global__ void k_fmm_level_count(int np, const int* __restrict__ cc, int* __restrict__ cp) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= np * np * np) return;
  const int i = b % np, j = (b / np) % np, k = b / (np * np);
  const int nc = 2 * np;
  int s = 0;
  for (int o = 0; o < 8; ++o) {
    const int ci = 2 * i + (o & 1), cj = 2 * j + ((o >> 1) & 1), ck = 2 * k + (o >> 2);
    s += cc[(ck * nc + cj) * nc + ci];
  }
  cp[b] = s;
}

// Translation tables of levels 2..L (child width w = D / 2^lev):
//   tabR[lev][o] = conj(R(t_o)), t_o = ((o_x - 1/2) w, (o_y - 1/2) w, (o_z - 1/2) w) (child
//   centre minus parent centre, used by M2M into level lev - 1 and by L2L into level lev);
//   tabI[lev][v] = I(v w) for v in [-3, 3]^3 with max |v_i| >= 2 (M2L), degree 2P, all m
//   ((2P + 1)^2 entries, n^2 + n + m).
template <typename T>
__global__ void k_fmm_tables(int P, int L, double D, Cx<T>* __restrict__ tabR, Cx<T>* __restrict__ tabI) {
  const int lev = 2 + blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (lev > L || e >= 8 + kFmmVecs) return;
  const int Kc = tri(P + 1, 0), F2 = (2 * P + 1) * (2 * P + 1);
  const double w = ldexp(D, -lev);
  if (e < 8) {
    const double tx = ((e & 1) - 0.5) * w, ty = (((e >> 1) & 1) - 0.5) * w, tz = ((e >> 2) - 0.5) * w;
    regular_table<T, double>(P, tx, ty, tz, tabR + ((size_t)(lev - 2) * 8 + e) * Kc, true);
  } else {
    const int v = e - 8;
    const int vx = v % 7 - 3, vy = (v / 7) % 7 - 3, vz = v / 49 - 3;
    if (abs(vx) <= 1 && abs(vy) <= 1 && abs(vz) <= 1) return;
    irregular_table<T>(2 * P, vx * w, vy * w, vz * w, tabI + ((size_t)(lev - 2) * kFmmVecs + v) * F2);
  }
}

// ---------------------------------------------------------------------------------
// Expansions: [box][Kc][density 0..3] complex (the four densities of one coefficient are
// adjacent, so a wave-uniform reader takes them in one scalar load), density 3 = psi.

// Entry (n, m), any sign of m, of density d of an interleaved expansion.
template <typename T>
__device__ __forceinline__ Cx<T> cget4(const Cx<T>* a, int n, int m, int d) {
  if (m >= 0) return a[tri(n, m) * 4 + d];
  const Cx<T> v = a[tri(n, -m) * 4 + d];
  return (m & 1) ? Cx<T>{-v.re, v.im} : Cx<T>{v.re, -v.im};
}

__device__ __forceinline__ void tri_inv(int c, int& n, int& m) {
  n = (int)((sqrtf(8.0f * c + 1.0f) - 1.0f) * 0.5f);
  while (tri(n + 1, 0) <= c) ++n;
  while (tri(n, 0) > c) --n;
  m = c - tri(n, 0);
}

// Column m (n = m..P) of conj(R_n^m(x, y, z)) into out[tri(n, m)]: the recurrences of
// regular_table for one m, in the same order, so the entries are the same.
template <typename T>
__device__ void regular_column(int P, int m, T x, T y, T z, Cx<T>* out) {
  const T r2 = x * x + y * y + z * z;
  T dre = 1, dim = 0;
  for (int k = 1; k <= m; ++k) {
    const T inv = T(1) / T(2 * k);
    const T nre = (dre * x - dim * y) * inv, nim = (dre * y + dim * x) * inv;
    dre = nre;
    dim = nim;
  }
  out[tri(m, m)] = Cx<T>{dre, -dim};
  if (m + 1 > P) return;
  T are = dre, aim = dim;
  T bre = z * dre, bim = z * dim;
  out[tri(m + 1, m)] = Cx<T>{bre, -bim};
  for (int n = m + 2; n <= P; ++n) {
    const T c1 = T(2 * n - 1), inv = T(1) / T((n - m) * (n + m));
    const T vre = (c1 * z * bre - r2 * are) * inv, vim = (c1 * z * bim - r2 * aim) * inv;
    are = bre; aim = bim;
    bre = vre; bim = vim;
    out[tri(n, m)] = Cx<T>{vre, -vim};
  }
}

// points per P2M chunk (the chunk's tables fill 39 KB of LDS in either precision)
template <typename T> struct P2mChunk { static constexpr int v = sizeof(T) == 8 ? 16 : 32; };

// Leaf multipoles: M_d[c] = sum_p charge_d(p) conj(R_c(y_p - centre)), charges
// (q_x, q_y, q_z, (y - centre).q), sources in leaf order.  One workgroup per leaf, 4 Kc
// threads (one output each, density fastest).  The regular tables of a chunk of points
// are built one (point, m) column per thread, then every output sums over the chunk in
// point order.
template <typename T>
__global__ void __launch_bounds__(1024) k_fmm_p2m(int P, int nb, double lox, double loy, double loz, double w,
                                                  const int* __restrict__ start, const int* __restrict__ perm,
                                                  const double4* __restrict__ Xs, const Src8<T>* __restrict__ src,
                                                  Cx<T>* __restrict__ Mout) {
  constexpr int CH = P2mChunk<T>::v;
  __shared__ Cx<T> Rt[CH][kFmmKc];
  __shared__ T ch[CH][4];
  __shared__ T sp[CH][3];
  const int b = blockIdx.x;
  const int Kc = tri(P + 1, 0);
  const int i = b % nb, j = (b / nb) % nb, k = b / (nb * nb);
  const double cx = lox + (i + 0.5) * w, cy = loy + (j + 0.5) * w, cz = loz + (k + 0.5) * w;
  const int s0 = start[b], n = start[b + 1] - s0;
  const int o = threadIdx.x;
  const int d = o & 3, c = min(o >> 2, Kc - 1);
  const bool live = o < 4 * Kc;
  Cx<T> acc{0, 0};
  for (int base = 0; base < n; base += CH) {
    const int cnt = min(CH, n - base);
    if (o < cnt) {
      const int p = s0 + base + o;
      const double4 x = Xs[p];
      const Src8<T> s = src[p];
      const T sx = (T)(x.x - cx), sy = (T)(x.y - cy), sz = (T)(x.z - cz);
      ch[o][0] = s.v[3];
      ch[o][1] = s.v[4];
      ch[o][2] = s.v[5];
      ch[o][3] = sx * s.v[3] + sy * s.v[4] + sz * s.v[5];
      sp[o][0] = sx;
      sp[o][1] = sy;
      sp[o][2] = sz;
    }
    __syncthreads();
    for (int t = o; t < cnt * (P + 1); t += blockDim.x) {
      const int q = t / (P + 1), m = t - q * (P + 1);
      regular_column<T>(P, m, sp[q][0], sp[q][1], sp[q][2], Rt[q]);
    }
    __syncthreads();
    if (live)
      for (int q = 0; q < cnt; ++q) {
        acc.re = fma(ch[q][d], Rt[q][c].re, acc.re);
        acc.im = fma(ch[q][d], Rt[q][c].im, acc.im);
      }
    __syncthreads();
  }
  if (live) Mout[((size_t)b * Kc + c) * 4 + d] = acc;
}

// Multipoles of level lev - 1 from their eight children at level lev (side nc).
template <typename T>
__global__ void __launch_bounds__(1024) k_fmm_m2m(int P, int nc, double wc, const int* __restrict__ cntc,
                                                  const Cx<T>* __restrict__ tabR, const Cx<T>* __restrict__ Mc,
                                                  Cx<T>* __restrict__ Mp) {
  __shared__ Cx<T> Mch[4][kFmmKc];
  __shared__ Cx<T> Rt[kFmmKc];
  const int np = nc / 2, b = blockIdx.x;
  const int Kc = tri(P + 1, 0);
  const int i = b % np, j = (b / np) % np, k = b / (np * np);
  const int o = threadIdx.x, d = o & 3, c = min(o >> 2, Kc - 1);
  const bool live = o < 4 * Kc;
  int n = 0, m = 0;
  tri_inv(c, n, m);
  Cx<T> acc{0, 0};
  for (int e = 0; e < 8; ++e) {
    const int ci = 2 * i + (e & 1), cj = 2 * j + ((e >> 1) & 1), ck = 2 * k + (e >> 2);
    const int cb = (ck * nc + cj) * nc + ci;
    if (cntc[cb] == 0) continue;
    const T tx = (T)(((e & 1) - 0.5) * wc), ty = (T)((((e >> 1) & 1) - 0.5) * wc), tz = (T)(((e >> 2) - 0.5) * wc);
    const Cx<T>* src = Mc + (size_t)cb * 4 * Kc;
    for (int q = threadIdx.x; q < Kc; q += blockDim.x) {
      const Cx<T> a = src[4 * q], bb = src[4 * q + 1], cc = src[4 * q + 2], dd = src[4 * q + 3];
      Mch[0][q] = a;
      Mch[1][q] = bb;
      Mch[2][q] = cc;
      // psi moves from the child centre to the parent's: + (c1 - c2) . phi
      Mch[3][q] = Cx<T>{dd.re + tx * a.re + ty * bb.re + tz * cc.re, dd.im + tx * a.im + ty * bb.im + tz * cc.im};
      Rt[q] = tabR[(size_t)e * Kc + q];
    }
    __syncthreads();
    if (live)
      for (int kk = 0; kk <= n; ++kk)
        for (int l = max(-kk, m - (n - kk)); l <= min(kk, m + (n - kk)); ++l)
          cfma(acc, cget(Mch[d], kk, l), cget(Rt, n - kk, m - l));
    __syncthreads();
  }
  if (live) Mp[((size_t)b * Kc + c) * 4 + d] = acc;
}

// Locals from the interaction lists (M2L), every level 2..L in one launch: workgroup g
// takes box g - first[lev] of level lev (side nl = 2^lev, width w = D / 2^lev), boxes
// without points are skipped.  One thread per local coefficient (k, l), l >= 0, for all four
// densities, so every table entry a thread reads serves four products.  The source
// multipoles are the same for the whole workgroup: they are read in their stored half
// (m >= 0) with wave-uniform (scalar) loads, the four densities of a coefficient in one, and
// the m < 0 half enters through X_n^{-m} = (-1)^m conj(X_n^m), which pairs the terms of +m
// and -m:  M I_a + (-1)^m conj(M) I_b = M.re (I_a.re + s I_b.re) + ..., four real FMAs per
// density and stored coefficient instead of eight.  The irregular table of the
// displacement (all m) is staged in LDS.  The psi shift from the source centre to the
// target's (- a . phi) is applied after the translation, by linearity:
// T(psi - a.phi) = T(psi) - a . T(phi).  The parents' locals are added afterwards (L2L).
// Per level: points per box, first box in the expansion arrays, first workgroup of the
// level in the fused M2L launch (levels 2..L, ascending).
struct FmmLevels {
  const int* cnt[8];
  size_t off[8];
  int first[9];
};

template <typename T>
__global__ void __launch_bounds__(256) k_fmm_m2l(int P, int L, double D, FmmLevels lv,
                                                 const Cx<T>* __restrict__ tabI, const Cx<T>* __restrict__ Mexp,
                                                 Cx<T>* __restrict__ Lexp) {
  constexpr int kFull2 = (2 * kFmmPMax + 1) * (2 * kFmmPMax + 1);
  __shared__ Cx<T> It[kFull2];
  int lev = 2;
  while (lev < L && (int)blockIdx.x >= lv.first[lev + 1]) ++lev;
  const int b = (int)blockIdx.x - lv.first[lev];
  const int* cnt = lv.cnt[lev];
  if (cnt[b] == 0) return;
  const int nl = 1 << lev;
  const double w = ldexp(D, -lev);
  const int Kc = tri(P + 1, 0), F2 = (2 * P + 1) * (2 * P + 1);
  const Cx<T>* Mlev = Mexp + lv.off[lev] * 4 * Kc;
  const Cx<T>* tabl = tabI + (size_t)(lev - 2) * kFmmVecs * F2;
  const int i = b % nl, j = (b / nl) % nl, k = b / (nl * nl);
  const int c = threadIdx.x;
  const bool act = c < Kc;
  int kk = 0, ll = 0;
  if (act) tri_inv(c, kk, ll);
  Cx<T> acc[4];
  for (int d = 0; d < 4; ++d) acc[d] = Cx<T>{0, 0};
  const T sk_sign = (kk & 1) ? T(-1) : T(1);
  const int pi = i / 2, pj = j / 2, pk = k / 2;
  for (int sk = max(0, 2 * pk - 2); sk <= min(nl - 1, 2 * pk + 3); ++sk)
    for (int sj = max(0, 2 * pj - 2); sj <= min(nl - 1, 2 * pj + 3); ++sj)
      for (int si = max(0, 2 * pi - 2); si <= min(nl - 1, 2 * pi + 3); ++si) {
        const int vx = i - si, vy = j - sj, vz = k - sk;
        if (abs(vx) <= 1 && abs(vy) <= 1 && abs(vz) <= 1) continue;
        const int sb = (sk * nl + sj) * nl + si;
        if (cnt[sb] == 0) continue;
        const Cx<T>* tv = tabl + (size_t)(((vz + 3) * 7 + (vy + 3)) * 7 + (vx + 3)) * F2;
        __syncthreads();  // the previous source's table has been read
        for (int q = threadIdx.x; q < F2; q += blockDim.x) It[q] = tv[q];
        __syncthreads();
        if (act) {
          Cx<T> pt[4];
          for (int d = 0; d < 4; ++d) pt[d] = Cx<T>{0, 0};
          // M I_a + sg conj(M) I_b for the stored coefficient M (four densities at v)
          auto pair = [&](const Cx<T>* v, int ia, int ib, T sg) {
            const Cx<T> ip = It[ia], im = It[ib];
            const T s1 = fma(sg, im.re, ip.re), s2 = fma(sg, im.im, -ip.im);
            const T s3 = fma(sg, im.im, ip.im), s4 = fma(-sg, im.re, ip.re);
            for (int d = 0; d < 4; ++d) {
              const Cx<T> a = v[d];
              pt[d].re = fma(a.re, s1, fma(a.im, s2, pt[d].re));
              pt[d].im = fma(a.re, s3, fma(a.im, s4, pt[d].im));
            }
          };
          // the source's coefficients in stored order: (n, 0), (n, 1), ..., (n, n), (n + 1, 0), ...
          const Cx<T>* v = Mlev + (size_t)sb * 4 * Kc;
          for (int n = 0; n <= P; ++n) {
            const int nk = n + kk;
            const int bi = nk * nk + nk + ll;
            {
              const Cx<T> ip = It[bi];
              for (int d = 0; d < 4; ++d) cfma(pt[d], v[d], ip);
              v += 4;
            }
            int m = 1;
            for (; m + 1 <= n; m += 2, v += 8) {
              pair(v, bi + m, bi - m, T(-1));
              pair(v + 4, bi + m + 1, bi - m - 1, T(1));
            }
            if (m <= n) {
              pair(v, bi + m, bi - m, T(-1));
              v += 4;
            }
          }
          // psi about the target centre: T(psi) - a . T(phi), a = c_t - c_s
          const T ax = (T)(vx * w), ay = (T)(vy * w), az = (T)(vz * w);
          pt[3].re -= ax * pt[0].re + ay * pt[1].re + az * pt[2].re;
          pt[3].im -= ax * pt[0].im + ay * pt[1].im + az * pt[2].im;
          for (int d = 0; d < 4; ++d) {
            acc[d].re = fma(sk_sign, pt[d].re, acc[d].re);
            acc[d].im = fma(sk_sign, pt[d].im, acc[d].im);
          }
        }
      }
  if (act) {
    Cx<T>* out = Lexp + (lv.off[lev] + (size_t)b) * 4 * Kc + (size_t)c * 4;
    for (int d = 0; d < 4; ++d) out[d] = acc[d];
  }
}

// Locals of level lev (side nl, width w) += the parent's locals translated to the box
// centre (L2L); the psi expansion moves from the parent centre to the child's by
// - (c' - c) . phi.  One workgroup per box, one thread per coefficient, four densities.
template <typename T>
__global__ void __launch_bounds__(256) k_fmm_l2l(int P, int nl, double w, const int* __restrict__ cnt,
                                                 const Cx<T>* __restrict__ tabR, const Cx<T>* __restrict__ Lpar,
                                                 Cx<T>* __restrict__ Llev) {
  __shared__ Cx<T> Ps[4][kFmmKc];
  __shared__ Cx<T> Rt[kFmmKc];
  const int b = blockIdx.x;
  if (cnt[b] == 0) return;
  const int Kc = tri(P + 1, 0);
  const int i = b % nl, j = (b / nl) % nl, k = b / (nl * nl);
  const int c = threadIdx.x;
  const bool act = c < Kc;
  int kk = 0, ll = 0;
  if (act) tri_inv(c, kk, ll);
  const int np = nl / 2;
  const int e = (i & 1) | ((j & 1) << 1) | ((k & 1) << 2);
  const T tx = (T)(((e & 1) - 0.5) * w), ty = (T)((((e >> 1) & 1) - 0.5) * w), tz = (T)(((e >> 2) - 0.5) * w);
  const Cx<T>* src = Lpar + (size_t)(((k / 2) * np + j / 2) * np + i / 2) * 4 * Kc;
  for (int q = threadIdx.x; q < Kc; q += blockDim.x) {
    const Cx<T> a = src[4 * q], bb = src[4 * q + 1], cc = src[4 * q + 2], dd = src[4 * q + 3];
    Ps[0][q] = a;
    Ps[1][q] = bb;
    Ps[2][q] = cc;
    Ps[3][q] = Cx<T>{dd.re - tx * a.re - ty * bb.re - tz * cc.re, dd.im - tx * a.im - ty * bb.im - tz * cc.im};
    Rt[q] = tabR[(size_t)e * Kc + q];
  }
  __syncthreads();
  if (!act) return;
  Cx<T>* out = Llev + ((size_t)b * Kc + c) * 4;
  Cx<T> acc[4];
  for (int d = 0; d < 4; ++d) acc[d] = out[d];
  for (int n = kk; n <= P; ++n)
    for (int l = max(-n, ll - (n - kk)); l <= min(n, ll + (n - kk)); ++l) {
      const Cx<T> r = cget(Rt, n - kk, l - ll);
      for (int d = 0; d < 4; ++d) cfma(acc[d], cget(Ps[d], n, l), r);
    }
  for (int d = 0; d < 4; ++d) out[d] = acc[d];
}

// Work items of the leaf kernel: (leaf, first target) for every 64 targets of a leaf.
__global__ void k_fmm_task_count(int nbox, const int* __restrict__ cnt, int* __restrict__ tcnt) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nbox) tcnt[b] = (cnt[b] + 63) / 64;
}

__global__ void k_fmm_task_fill(int nbox, const int* __restrict__ tcnt, const int* __restrict__ toff,
                                int2* __restrict__ task) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbox) return;
  for (int j = 0; j < tcnt[b]; ++j) task[toff[b] + j] = make_int2(b, 64 * j);
}

// Sources in leaf order: srt[p] = src[perm[p]] with the body index in v[6].
template <typename T>
__global__ void k_fmm_pack_sorted(int N, const int* __restrict__ perm, const double4* __restrict__ Xs,
                                  const Src8<T>* __restrict__ src, Src8<T>* __restrict__ srt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  Src8<T> s = src[perm[p]];
  s.v[6] = (T)Xs[p].w;
  s.v[7] = 0;
  srt[p] = s;
}

// Leaf evaluation, one wave per work item (64 targets of one leaf, one per lane): far field
// from the leaf's local expansions, plus the direct traction sum over the points of the 27
// adjacent leaves that belong to other bodies.  The leaf is wave-uniform, so its expansion
// coefficients and the sources (9 contiguous ranges of the leaf-ordered points) are read
// with scalar loads.  Writes -(3/4pi)-scaled sums to out[3][N] at the original indices.
template <typename T>
__global__ void __launch_bounds__(256) k_fmm_leaf(int P, int nb, double lox, double loy, double loz, double w,
                                                  int N, int ntask, const int2* __restrict__ task,
                                                  const int* __restrict__ start, const int* __restrict__ perm,
                                                  const double4* __restrict__ Xs, const double4* __restrict__ Ns,
                                                  const Src8<T>* __restrict__ srt, const Cx<T>* __restrict__ Lleaf,
                                                  int far_on, double* __restrict__ out) {
  const int wv = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (wv >= ntask) return;
  const int lane = threadIdx.x & 63;
  const int2 tk = task[wv];
  const int b = __builtin_amdgcn_readfirstlane(tk.x), t0 = __builtin_amdgcn_readfirstlane(tk.y);
  const int s0 = start[b], nt = start[b + 1] - s0;
  const int t = t0 + lane;
  const bool live = t < nt;
  const int Kc = tri(P + 1, 0);
  const int i = b % nb, j = (b / nb) % nb, k = b / (nb * nb);
  const double cx = lox + (i + 0.5) * w, cy = loy + (j + 0.5) * w, cz = loz + (k + 0.5) * w;
  const double4 xt = Xs[s0 + (live ? t : 0)], nn = Ns[s0 + (live ? t : 0)];
  const T xa = (T)xt.x, ya = (T)xt.y, za = (T)xt.z, nx = (T)nn.x, ny = (T)nn.y, nz = (T)nn.z;
  const T bt = (T)xt.w;
  T fx = 0, fy = 0, fz = 0;
  if (far_on) {
    const Cx<T>* Lb = Lleaf + (size_t)b * 4 * Kc;
    const T ssx = (T)(xt.x - cx), ssy = (T)(xt.y - cy), ssz = (T)(xt.z - cz);
    const T r2 = ssx * ssx + ssy * ssy + ssz * ssz;
    // gradient sums (d/dx + i d/dy) phi_0, phi_1 and d/dz phi_2; for all four densities
    // A = (d/dx + i d/dy)^2, B = d/dz (d/dx + i d/dy), C = d^2/dz^2
    Cx<T> g0{0, 0}, g1{0, 0}, g2{0, 0}, A[4], B[4], C[4];
    for (int dd = 0; dd < 4; ++dd) A[dd] = B[dd] = C[dd] = Cx<T>{0, 0};
    auto term = [&](int kk, int l, Cx<T> v) {
      if (kk <= P - 1) {
        cfma(g0, cget4(Lb, kk + 1, l + 1, 0), v);
        cfma(g1, cget4(Lb, kk + 1, l + 1, 1), v);
        cfma(g2, cget4(Lb, kk + 1, l, 2), v);
      }
      if (kk <= P - 2)
        for (int dd = 0; dd < 4; ++dd) {
          cfma(A[dd], cget4(Lb, kk + 2, l + 2, dd), v);
          cfma(B[dd], cget4(Lb, kk + 2, l + 1, dd), v);
          cfma(C[dd], cget4(Lb, kk + 2, l, dd), v);
        }
    };
    // R_kk^l(s) column by column (l >= 0): conj(R^l) for +l and (-1)^l R^l for -l
    T dre = 1, dim = 0;
    for (int l = 0; l <= P - 1; ++l) {
      if (l > 0) {
        const T inv = T(1) / T(2 * l);
        const T nre = (dre * ssx - dim * ssy) * inv, nim = (dre * ssy + dim * ssx) * inv;
        dre = nre;
        dim = nim;
      }
      T are = 0, aim = 0, bre = dre, bim = dim;
      for (int kk = l; kk <= P - 1; ++kk) {
        if (kk > l) {
          const T c1 = T(2 * kk - 1), inv = T(1) / T((kk - l) * (kk + l));
          const T vre = (c1 * ssz * bre - r2 * are) * inv, vim = (c1 * ssz * bim - r2 * aim) * inv;
          are = bre; aim = bim;
          bre = vre; bim = vim;
        }
        term(kk, l, Cx<T>{bre, -bim});
        if (l > 0) term(kk, -l, (l & 1) ? Cx<T>{-bre, -bim} : Cx<T>{bre, bim});
      }
    }
    const T div = g0.re + g1.im + g2.re;
    T H[4][6];  // xx, yy, zz, xy, xz, yz
    for (int dd = 0; dd < 4; ++dd) {
      H[dd][0] = T(0.5) * (A[dd].re - C[dd].re);
      H[dd][1] = T(0.5) * (-A[dd].re - C[dd].re);
      H[dd][2] = C[dd].re;
      H[dd][3] = T(0.5) * A[dd].im;
      H[dd][4] = B[dd].re;
      H[dd][5] = B[dd].im;
    }
    T Hs[6];
    for (int e = 0; e < 6; ++e) Hs[e] = H[3][e] - ssx * H[0][e] - ssy * H[1][e] - ssz * H[2][e];
    // the direct sum is kept in units of -(3/4pi): scale the far part by -(1/3)
    const T sc = T(-1.0 / 3.0);
    fx = sc * (div * nx + Hs[0] * nx + Hs[3] * ny + Hs[4] * nz);
    fy = sc * (div * ny + Hs[3] * nx + Hs[1] * ny + Hs[5] * nz);
    fz = sc * (div * nz + Hs[4] * nx + Hs[5] * ny + Hs[2] * nz);
  }
  // near field: traction of the other bodies' points in the 27 adjacent leaves
  // (same-body pairs: weight 0, and |d|^2 + 1 keeps the point's own pair finite; the
  // arithmetic mask keeps the loop free of branches)
  auto near = [&](const Src8<T>& s) {
    const T dx = xa - s.v[0], dy = ya - s.v[1], dz = za - s.v[2];
    const T other = s.v[6] == bt ? T(0) : T(1);
    const T r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, T(1) - other)));
    const T dn = dx * nx + dy * ny + dz * nz;
    const T dq = dx * s.v[3] + dy * s.v[4] + dz * s.v[5];
    const T f = ((dn * dq) * other) * rinv5_t(r2);
    fx += f * dx;
    fy += f * dy;
    fz += f * dz;
  };
  // for each (nk, nj) the leaves ni - 1 .. ni + 1 are consecutive in leaf order
  const int i0 = max(0, i - 1), i1 = min(nb - 1, i + 1);
  for (int nk = max(0, k - 1); nk <= min(nb - 1, k + 1); ++nk)
    for (int nj = max(0, j - 1); nj <= min(nb - 1, j + 1); ++nj) {
      const int row = (nk * nb + nj) * nb;
      const int a0 = __builtin_amdgcn_readfirstlane(start[row + i0]);
      const int a1 = __builtin_amdgcn_readfirstlane(start[row + i1 + 1]);
      // four sources per step: their scalar loads are issued together
      int q = a0;
      for (; q + 4 <= a1; q += 4) {
        const Src8<T> s0 = srt[q], s1 = srt[q + 1], s2 = srt[q + 2], s3 = srt[q + 3];
        near(s0);
        near(s1);
        near(s2);
        near(s3);
      }
      for (; q < a1; ++q) near(srt[q]);
    }
  if (live) {
    const int g = perm[s0 + t];
    const double sc = -3.0 / (4.0 * RBM_PI);
    out[g] = sc * (double)fx;
    out[(size_t)N + g] = sc * (double)fy;
    out[2 * (size_t)N + g] = sc * (double)fz;
  }
}

// ---------------------------------------------------------------------------------
// Launchers

hipError_t launch_fmm_bounds(int N, const double* X, double* out6, hipStream_t st) {
  k_fmm_bounds<<<1, 1024, 0, st>>>(N, X, out6);
  return hipGetLastError();
}

hipError_t launch_fmm_sort_points(int N, int M, const double* X, const double* Nn, const double* lo, double w,
                                  int nb, int* leaf, int* cnt, int* start, int* fill, int* perm, int* maxcnt,
                                  double4* Xs, double4* Ns, hipStream_t st) {
  const int nbox = nb * nb * nb;
  hipError_t e;
  if ((e = hipMemsetAsync(cnt, 0, (size_t)nbox * sizeof(int), st)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(fill, 0, (size_t)nbox * sizeof(int), st)) != hipSuccess) return e;
  k_fmm_count<<<(N + 255) / 256, 256, 0, st>>>(N, X, lo[0], lo[1], lo[2], w, nb, leaf, cnt);
  k_fmm_scan<<<1, 1024, 0, st>>>(nbox, cnt, start, maxcnt);
  k_fmm_scatter<<<(N + 255) / 256, 256, 0, st>>>(N, leaf, start, fill, perm);
  return hipGetLastError();
}

hipError_t launch_fmm_finish_tree(int N, int M, int L, const double* X, const double* Nn, const int* start,
                                  int* perm, double4* Xs, double4* Ns, int* const* cnt_lev, int* tcnt, int* toff,
                                  int2* task, int* scratch, hipStream_t st) {
  const int nb = 1 << L, nbox = nb * nb * nb;
  k_fmm_sort<<<nbox, 256, 0, st>>>(start, perm);
  k_fmm_gather<<<(N + 255) / 256, 256, 0, st>>>(N, M, perm, X, Nn, Xs, Ns);
  for (int lev = L - 1; lev >= 2; --lev) {
    const int np = 1 << lev;
    k_fmm_level_count<<<(np * np * np + 255) / 256, 256, 0, st>>>(np, cnt_lev[lev + 1], cnt_lev[lev]);
  }
  k_fmm_task_count<<<(nbox + 255) / 256, 256, 0, st>>>(nbox, cnt_lev[L], tcnt);
  k_fmm_scan<<<1, 1024, 0, st>>>(nbox, tcnt, toff, scratch);
  k_fmm_task_fill<<<(nbox + 255) / 256, 256, 0, st>>>(nbox, tcnt, toff, task);
  return hipGetLastError();
}

static int fmm_threads(int P) {
  const int o = 4 * tri(P + 1, 0);
  return (o + 63) / 64 * 64;
}

template <typename T>
hipError_t launch_fmm_tables(int P, int L, double D, void* tabR, void* tabI, hipStream_t st) {
  if (P < 2 || P > kFmmPMax || L < 2) return hipErrorInvalidValue;
  dim3 grid((8 + kFmmVecs + 63) / 64, L - 1);
  k_fmm_tables<T><<<grid, 64, 0, st>>>(P, L, D, static_cast<Cx<T>*>(tabR), static_cast<Cx<T>*>(tabI));
  return hipGetLastError();
}

// One evaluation of the traction sums for the sources src (packed, original order):
// multipoles up, locals down, leaf evaluation into out[3][N].  Mexp/Lexp hold levels
// 2..L at box offsets lev_off[lev]; cnt_lev[lev] the points per box.
template <typename T>
hipError_t launch_fmm_apply(int P, int L, const double* lo, double D, int N, const int* start, const int* perm,
                            const double4* Xs, const double4* Ns, int* const* cnt_lev, const size_t* lev_off,
                            int ntask, const int2* task, const void* tabR, const void* tabI, const void* src,
                            void* srt, void* Mexp, void* Lexp, double* out, hipStream_t st) {
  if (P < 2 || P > kFmmPMax || L < 0) return hipErrorInvalidValue;
  const int nb = 1 << L, Kc = tri(P + 1, 0);
  const double w = ldexp(D, -L);
  Src8<T>* so = static_cast<Src8<T>*>(srt);
  Cx<T>* Mx = static_cast<Cx<T>*>(Mexp);
  Cx<T>* Lx = static_cast<Cx<T>*>(Lexp);
  const Cx<T>* tR = static_cast<const Cx<T>*>(tabR);
  const Cx<T>* tI = static_cast<const Cx<T>*>(tabI);
  const int th = fmm_threads(P);
  const bool far_on = L >= 2;
  k_fmm_pack_sorted<T><<<(N + 255) / 256, 256, 0, st>>>(N, perm, Xs, static_cast<const Src8<T>*>(src), so);
  if (far_on) {
    k_fmm_p2m<T><<<nb * nb * nb, th, 0, st>>>(P, nb, lo[0], lo[1], lo[2], w, start, perm, Xs, so,
                                              Mx + lev_off[L] * 4 * Kc);
    for (int lev = L; lev > 2; --lev) {
      const int nc = 1 << lev, np = nc / 2;
      k_fmm_m2m<T><<<np * np * np, th, 0, st>>>(P, nc, ldexp(D, -lev), cnt_lev[lev],
                                                tR + (size_t)(lev - 2) * 8 * Kc, Mx + lev_off[lev] * 4 * Kc,
                                                Mx + lev_off[lev - 1] * 4 * Kc);
    }
    if (L > 6) return hipErrorInvalidValue;
    FmmLevels lv{};
    int nwg = 0;
    for (int lev = 2; lev <= L; ++lev) {
      lv.cnt[lev] = cnt_lev[lev];
      lv.off[lev] = lev_off[lev];
      lv.first[lev] = nwg;
      nwg += 1 << (3 * lev);
    }
    lv.first[L + 1] = nwg;
    const int thl = (Kc + 63) / 64 * 64;
    k_fmm_m2l<T><<<nwg, thl, 0, st>>>(P, L, D, lv, tI, Mx, Lx);
    for (int lev = 3; lev <= L; ++lev) {
      const int nl = 1 << lev;
      k_fmm_l2l<T><<<nl * nl * nl, thl, 0, st>>>(P, nl, ldexp(D, -lev), cnt_lev[lev], tR + (size_t)(lev - 2) * 8 * Kc,
                                                Lx + lev_off[lev - 1] * 4 * Kc, Lx + lev_off[lev] * 4 * Kc);
    }
  }
  if (ntask > 0)
    k_fmm_leaf<T><<<(ntask + 3) / 4, 256, 0, st>>>(P, nb, lo[0], lo[1], lo[2], w, N, ntask, task, start, perm, Xs,
                                                   Ns, so, far_on ? Lx + lev_off[L] * 4 * Kc : nullptr,
                                                   far_on ? 1 : 0, out);
  return hipGetLastError();
}

template hipError_t launch_fmm_tables<double>(int, int, double, void*, void*, hipStream_t);
template hipError_t launch_fmm_tables<float>(int, int, double, void*, void*, hipStream_t);
template hipError_t launch_fmm_apply<double>(int, int, const double*, double, int, const int*, const int*,
                                             const double4*, const double4*, int* const*, const size_t*, int,
                                             const int2*, const void*, const void*, const void*, void*, void*,
                                             void*, double*, hipStream_t);
template hipError_t launch_fmm_apply<float>(int, int, const double*, double, int, const int*, const int*,
                                            const double4*, const double4*, int* const*, const size_t*, int,
                                            const int2*, const void*, const void*, const void*, void*, void*,
                                            void*, double*, hipStream_t);

}  // namespace rbm
