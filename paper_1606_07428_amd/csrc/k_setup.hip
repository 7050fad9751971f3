// Setup kernels (float64): grid tables, shape geometry, singular self operators,
// block inverse and velocity functional.  §2.2, §2.3, §3, §3.1, §3.2 of the paper.
#include "common.h"
#include "kernels.h"

namespace rbm {

// n-point Gauss-Legendre nodes (ascending) and weights by Newton's method on P_n.
__global__ void k_gauss_legendre(int n, double* t, double* w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = -cos(RBM_PI * (i + 0.75) / (n + 0.5));
  double pn = 0.0, pn1 = 0.0;
  for (int it = 0; it < 100; ++it) {
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    pn = p1;
    pn1 = p0;
    const double dp = n * (x * pn - pn1) / (x * x - 1.0);
    const double dx = pn / dp;
    x -= dx;
    if (fabs(dx) < 1e-16) break;
  }
  double p0 = 1.0, p1 = x;
  for (int k = 2; k <= n; ++k) {
    const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  const double dp = n * (x * p1 - p0) / (x * x - 1.0);
  t[i] = x;
  w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
}

hipError_t launch_gauss_legendre(int n, double* t, double* w, hipStream_t st) {
  k_gauss_legendre<<<(n + 63) / 64, 64, 0, st>>>(n, t, w);
  return hipGetLastError();
}

// Per grid node a: real SH tables and the forward transform (§3 grid, band B_p).
__global__ void k_grid_tables(int p, const double* glt, const double* glw, double* Y, double* Yt,
                              double* Yps, double* F, double* Ft, double* nth, double* nph,
                              double* nlam) {
  const int M = (p + 1) * 2 * p;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= M) return;
  const int nB = p * p + 2 * p;
  const int j = a / (2 * p), k = a % (2 * p);
  const double x = glt[j];
  const double s = sqrt(fmax(0.0, 1.0 - x * x));
  const double ph = RBM_PI * k / p;
  const double lam = glw[j];
  nth[a] = acos(x);
  nph[a] = ph;
  nlam[a] = lam;
  const double wq = RBM_PI / p * lam;
  int cur_m = -1;
  double cm = 1.0, sm = 0.0;
  legendre_sweep(p, x, s, [&](int l, int m, double P, double Q, double D) {
    const int i0 = l * l + l;
    if (m == 0) {
      Y[(size_t)i0 * M + a] = P;
      Yt[(size_t)i0 * M + a] = D;
      Yps[(size_t)i0 * M + a] = 0.0;
      const int b = band_index(l, 0, p);
      F[(size_t)b * M + a] = wq * P;
      Ft[(size_t)a * nB + b] = wq * P;
      return;
    }
    if (m != cur_m) {
      sincos(m * ph, &sm, &cm);
      cur_m = m;
    }
    const double r2 = 1.41421356237309504880;
    const double yp = r2 * P * cm, ym = r2 * P * sm;
    Y[(size_t)(i0 + m) * M + a] = yp;
    Y[(size_t)(i0 - m) * M + a] = ym;
    Yt[(size_t)(i0 + m) * M + a] = r2 * D * cm;
    Yt[(size_t)(i0 - m) * M + a] = r2 * D * sm;
    Yps[(size_t)(i0 + m) * M + a] = -r2 * m * Q * sm;
    Yps[(size_t)(i0 - m) * M + a] = r2 * m * Q * cm;
    const int bp = band_index(l, m, p);
    const double nu = (l == p && m == p) ? 0.5 : 1.0;
    F[(size_t)bp * M + a] = wq * nu * yp;
    Ft[(size_t)a * nB + bp] = wq * nu * yp;
    const int bm = band_index(l, -m, p);
    if (bm >= 0) {
      F[(size_t)bm * M + a] = wq * ym;
      Ft[(size_t)a * nB + bm] = wq * ym;
    }
  });
}

hipError_t launch_grid_tables(int p, const double* gl_t, const double* gl_w, double* Ytab,
                              double* Yttab, double* Ypstab, double* Ftab, double* Fttab,
                              double* node_th, double* node_ph, double* node_lam, hipStream_t st) {
  const int M = (p + 1) * 2 * p;
  k_grid_tables<<<(M + 63) / 64, 64, 0, st>>>(p, gl_t, gl_w, Ytab, Yttab, Ypstab, Ftab, Fttab,
                                              node_th, node_ph, node_lam);
  return hipGetLastError();
}

// Rotated GL(ps+1) x trapezoid(2ps) grid and the singular weights
// W_jk = (pi/ps) lam'_j [sum_{nu<=ps} P_nu(t'_j)] sqrt(2(1-t'_j)): since
// 1/|e_z - s'| = sum_nu P_nu(t'), this integrates circle averages of degree <= ps
// in t' exactly against the 1/r singularity at the rotated pole.
__global__ void k_rotated_rule(int ps, const double* glt, const double* glw, double* nodes,
                               double* W) {
  const int Ms = (ps + 1) * 2 * ps;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Ms) return;
  const int j = q / (2 * ps), k = q % (2 * ps);
  const double t = glt[j];
  double pm1 = 0.0, p0 = 1.0, S = 1.0;
  for (int nu = 1; nu <= ps; ++nu) {
    const double pn = ((2.0 * nu - 1.0) * t * p0 - (nu - 1.0) * pm1) / nu;
    pm1 = p0;
    p0 = pn;
    S += pn;
  }
  const double ph = RBM_PI * k / ps;
  const double st = sqrt(fmax(0.0, 1.0 - t * t));
  double sp, cp;
  sincos(ph, &sp, &cp);
  nodes[q] = st * cp;
  nodes[Ms + q] = st * sp;
  nodes[2 * Ms + q] = t;
  W[q] = RBM_PI / ps * glw[j] * S * sqrt(2.0 * (1.0 - t));
}

hipError_t launch_rotated_rule(int ps, const double* glt, const double* glw, double* nodes,
                               double* W, hipStream_t st) {
  const int Ms = (ps + 1) * 2 * ps;
  k_rotated_rule<<<(Ms + 63) / 64, 64, 0, st>>>(ps, glt, glw, nodes, W);
  return hipGetLastError();
}

// Radial shape r(s) = sum rc Y -> coordinate coefficients of x = r(s) s by the
// exact forward transform of the grid values (degree of x below p).
__global__ __launch_bounds__(256) void k_radial_to_coef(int p, int nrc, const double* rc_all,
                                                        const double* Ytab, const double* Ftab,
                                                        const double* nth, const double* nph,
                                                        double* coef_all) {
  extern __shared__ double xg[];  // [3][M]
  const int M = (p + 1) * 2 * p, nc = (p + 1) * (p + 1), nB = p * p + 2 * p;
  const int s = blockIdx.x;
  const double* rc = rc_all + (size_t)s * nrc;
  for (int a = threadIdx.x; a < M; a += blockDim.x) {
    double r = 0.0;
    for (int i = 0; i < nrc; ++i) r += rc[i] * Ytab[(size_t)i * M + a];
    double st, ct, sp, cp;
    sincos(nth[a], &st, &ct);
    sincos(nph[a], &sp, &cp);
    xg[a] = r * st * cp;
    xg[M + a] = r * st * sp;
    xg[2 * M + a] = r * ct;
  }
  __syncthreads();
  double* coef = coef_all + (size_t)s * 3 * nc;
  for (int b = threadIdx.x; b < nB; b += blockDim.x) {
    const int full = b < p * p ? b : b + 1;
    for (int c = 0; c < 3; ++c) {
      double v = 0.0;
      for (int a = 0; a < M; ++a) v += Ftab[(size_t)b * M + a] * xg[c * M + a];
      coef[c * nc + full] = v;
    }
  }
  if (threadIdx.x < 3) coef[threadIdx.x * nc + p * p] = 0.0;  // the dropped (p, -p) mode
}

hipError_t launch_radial_to_coef(int ns, int p, int nrc, const double* rc, const double* Ytab,
                                 const double* Ftab, const double* node_th, const double* node_ph,
                                 double* coef, hipStream_t st) {
  const int M = (p + 1) * 2 * p;
  k_radial_to_coef<<<ns, 256, 3 * M * sizeof(double), st>>>(p, nrc, rc, Ytab, Ftab, node_th,
                                                            node_ph, coef);
  return hipGetLastError();
}

// Per shape: x, outward normal, J = |x_theta x x_phi/sin|, weights w = (pi/p) lam J (§3),
// area, area centroid, tau (§2.2) and tau^{-1}; r = x - x^c.
// shp layout per shape (32 doubles): [0] area, [1..3] xc, [4..12] tau, [13..21] tau^{-1}.
__global__ __launch_bounds__(256) void k_shape_geometry(int p, const double* coef_all,
                                                        const double* Ytab, const double* Yttab,
                                                        const double* Ypstab, const double* nlam,
                                                        double* gx_all, double* gn_all,
                                                        double* gw_all, double* gr_all,
                                                        double* shp_all) {
  __shared__ double red[16];
  const int M = (p + 1) * 2 * p, nc = (p + 1) * (p + 1);
  const int s = blockIdx.x;
  const double* coef = coef_all + (size_t)s * 3 * nc;
  double* gx = gx_all + (size_t)s * 3 * M;
  double* gn = gn_all + (size_t)s * 3 * M;
  double* gw = gw_all + (size_t)s * M;
  double* gr = gr_all + (size_t)s * 3 * M;
  double a_area = 0.0, a_x[3] = {0.0, 0.0, 0.0};
  for (int a = threadIdx.x; a < M; a += blockDim.x) {
    double x[3] = {0, 0, 0}, xt[3] = {0, 0, 0}, xp[3] = {0, 0, 0};
    for (int i = 0; i < nc; ++i) {
      const double y = Ytab[(size_t)i * M + a], yt = Yttab[(size_t)i * M + a],
                   yp = Ypstab[(size_t)i * M + a];
      for (int c = 0; c < 3; ++c) {
        const double cf = coef[c * nc + i];
        x[c] += cf * y;
        xt[c] += cf * yt;
        xp[c] += cf * yp;
      }
    }
    const double cx = xt[1] * xp[2] - xt[2] * xp[1];
    const double cy = xt[2] * xp[0] - xt[0] * xp[2];
    const double cz = xt[0] * xp[1] - xt[1] * xp[0];
    const double J = sqrt(cx * cx + cy * cy + cz * cz);
    const double w = RBM_PI / p * nlam[a] * J;
    for (int c = 0; c < 3; ++c) gx[c * M + a] = x[c];
    gn[a] = cx / J;
    gn[M + a] = cy / J;
    gn[2 * M + a] = cz / J;
    gw[a] = w;
    a_area += w;
    for (int c = 0; c < 3; ++c) a_x[c] += w * x[c];
  }
  const double area = block_sum(a_area, red);
  double xc[3];
  for (int c = 0; c < 3; ++c) xc[c] = block_sum(a_x[c], red) / area;
  __syncthreads();
  double t6[6] = {0, 0, 0, 0, 0, 0};  // xx, yy, zz (of r r^T), xy, xz, yz; and |r|^2 via sum
  for (int a = threadIdx.x; a < M; a += blockDim.x) {
    double r[3];
    for (int c = 0; c < 3; ++c) {
      r[c] = gx[c * M + a] - xc[c];
      gr[c * M + a] = r[c];
    }
    const double w = gw[a];
    t6[0] += w * r[0] * r[0];
    t6[1] += w * r[1] * r[1];
    t6[2] += w * r[2] * r[2];
    t6[3] += w * r[0] * r[1];
    t6[4] += w * r[0] * r[2];
    t6[5] += w * r[1] * r[2];
  }
  double T[6];
  for (int k = 0; k < 6; ++k) T[k] = block_sum(t6[k], red);
  if (threadIdx.x == 0) {
    double* sp = shp_all + (size_t)s * 32;
    const double tr = T[0] + T[1] + T[2];
    double tau[9] = {tr - T[0], -T[3], -T[4], -T[3], tr - T[1], -T[5], -T[4], -T[5], tr - T[2]};
    sp[0] = area;
    sp[1] = xc[0];
    sp[2] = xc[1];
    sp[3] = xc[2];
    for (int k = 0; k < 9; ++k) sp[4 + k] = tau[k];
    inv3(tau, sp + 13);
  }
}

hipError_t launch_shape_geometry(int ns, int p, const double* coef, const double* Ytab,
                                 const double* Yttab, const double* Ypstab, const double* node_lam,
                                 double* gx, double* gn, double* gw, double* gr, double* shp,
                                 hipStream_t st) {
  k_shape_geometry<<<ns, 256, 0, st>>>(p, coef, Ytab, Yttab, Ypstab, node_lam, gx, gn, gw, gr, shp);
  return hipGetLastError();
}

// Singular self operators by grid rotation (§3 and the rule of Gimbutas-Veerapaneni
// cited there).  For the rotated nodes s_q = Q_t s'_q, Q_t = R_z(phi_t) R_y(theta_t):
//   C[k][b] = sum_q W_q J(s_q) kern_k(x_t, x(s_q)) Y_b(s_q)         (b in B_p)
//   row(t)  = C F                                                     (F: grid -> B_p)
// kern = Stokeslet/eta (S) and n_t . T (K); both 3x3 symmetric (6 entries each).
// Outputs are column-major body-frame (3M x 3M) operators: entry (row=c*M+t,
// col=c'*M+a) at [col*3M + row].
//
// One workgroup per (target node t, group of G consecutive shapes).  The rotated nodes
// and their harmonics Y_b(s_q) depend on t alone, so the shapes of a group share them.
// Per chunk of NC rotated nodes, LPN adjacent lanes per (node, shape g) run the Legendre
// recurrence at the node for shape g's surface there (with LPN = 4 each lane takes a
// quarter of the columns m and the lanes add their partial position and tangents by
// shuffles), then form the kernel weights; the lanes of shape 0 also stage the harmonics
// in LDS, and thread b contracts them with the weights of every shape of the group.
// Finally C of each shape goes to LDS and the threads form row(t) of its operators.
template <int NC, int G, int LPN>
__global__ __launch_bounds__(256, 2) void k_singular(int ns, int p, int ps, double eta,
                                                  const double* __restrict__ coef_all,
                                                  const double* __restrict__ gx_all,
                                                  const double* __restrict__ gn_all,
                                                  const double* __restrict__ nth,
                                                  const double* __restrict__ nph,
                                                  const double* __restrict__ rnodes,
                                                  const double* __restrict__ rW,
                                                  const double* __restrict__ Ft,
                                                  double* __restrict__ Sop,
                                                  double* __restrict__ Kop) {
  static_assert(LPN == 1 || LPN == 4, "one or four lanes per (node, shape)");
  static_assert(NC * G * LPN <= 256, "LPN lanes per (node, shape)");
  extern __shared__ double lds[];
  // row stride of the staged harmonics: odd, so that the contraction, whose lanes
  // read one row each at the same column, hits distinct LDS banks (a stride of 64
  // doubles put every lane in one bank)
  constexpr int YS = NC + 1;
  const int M = (p + 1) * 2 * p, M3 = 3 * M, nc = (p + 1) * (p + 1), nB = p * p + 2 * p;
  const int Ms = (ps + 1) * 2 * ps;
  const int t = blockIdx.x, s0 = blockIdx.y * G, tid = threadIdx.x;
  const int ng = min(G, ns - s0);  // shapes in this group
  double* cf = lds;                  // [G][3][nc]
  double* Ych = cf + G * 3 * nc;     // [nB][YS]
  double* Kw = Ych + nB * YS;        // [G][12][NC]
  double* ltab = Kw + G * 12 * NC;   // Legendre recurrence coefficients
  for (int i = tid; i < G * 3 * nc; i += 256)
    cf[i] = i < ng * 3 * nc ? coef_all[(size_t)s0 * 3 * nc + i] : 0.0;
  legendre_table(p, ltab, tid, 256);
  double st, ct, sp, cp;
  sincos(nth[t], &st, &ct);
  sincos(nph[t], &sp, &cp);
  const double Q[9] = {cp * ct, -sp, cp * st, sp * ct, cp, sp * st, -st, 0.0, ct};
  // lanes (node, g, r) of the sweep, r < LPN splitting the Legendre columns: the shape's
  // target point and normal
  const int pair = tid / LPN, r = tid % LPN;
  const int node = pair % NC, g = pair / NC;
  const bool sweeper = pair < NC * G;
  const bool live = sweeper && g < ng;
  double xt0 = 0, xt1 = 0, xt2 = 0, nt0 = 0, nt1 = 0, nt2 = 0;
  if (live) {
    const double* gx = gx_all + (size_t)(s0 + g) * 3 * M;
    const double* gn = gn_all + (size_t)(s0 + g) * 3 * M;
    xt0 = gx[t], xt1 = gx[M + t], xt2 = gx[2 * M + t];
    nt0 = gn[t], nt1 = gn[M + t], nt2 = gn[2 * M + t];
  }
  const double* cfg = cf + (sweeper ? g : 0) * 3 * nc;
  double* Kwg = Kw + (sweeper ? g : 0) * 12 * NC;
  const double cS = 1.0 / (8.0 * RBM_PI * eta);
  const double cK = -3.0 / (4.0 * RBM_PI);
  double acc0[G][12], acc1[12];
#pragma unroll
  for (int gg = 0; gg < G; ++gg)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc0[gg][k] = 0.0;
  for (int k = 0; k < 12; ++k) acc1[k] = 0.0;
  for (int chunk = 0; chunk < Ms; chunk += NC) {
    __syncthreads();
    if (sweeper) {
      const int q = chunk + node;
      if (q < Ms) {
        const double s0n = rnodes[q], s1n = rnodes[Ms + q], s2n = rnodes[2 * Ms + q];
        const double v0 = Q[0] * s0n + Q[1] * s1n + Q[2] * s2n;
        const double v1 = Q[3] * s0n + Q[4] * s1n + Q[5] * s2n;
        const double v2 = Q[6] * s0n + Q[7] * s1n + Q[8] * s2n;
        const double sx = sqrt(v0 * v0 + v1 * v1);   // sin(theta) of the rotated node
        const double cx = v2;                        // cos(theta)
        const double ph = atan2(v1, v0);
        double x[3] = {0, 0, 0}, dt[3] = {0, 0, 0}, dp[3] = {0, 0, 0};
        int cur_m = -1;
        double cm = 1.0, sm = 0.0;
        const bool stage = g == 0;
        auto term = [&](int l, int m, double P, double Qv, double D) {
          const int i0 = l * l + l;
          if (m == 0) {
            for (int c = 0; c < 3; ++c) {
              const double a = cfg[c * nc + i0];
              x[c] += a * P;
              dt[c] += a * D;
            }
            if (stage) Ych[band_index(l, 0, p) * YS + node] = P;
            return;
          }
          if (m != cur_m) {
            sincos(m * ph, &sm, &cm);
            cur_m = m;
          }
          const double r2 = 1.41421356237309504880;
          const double yp = r2 * P * cm, ym = r2 * P * sm;
          const double tp = r2 * D * cm, tm = r2 * D * sm;
          const double pp = -r2 * m * Qv * sm, pm = r2 * m * Qv * cm;
          for (int c = 0; c < 3; ++c) {
            const double ap = cfg[c * nc + i0 + m], am = cfg[c * nc + i0 - m];
            x[c] += ap * yp + am * ym;
            dt[c] += ap * tp + am * tm;
            dp[c] += ap * pp + am * pm;
          }
          if (stage) {
            Ych[band_index(l, m, p) * YS + node] = yp;
            const int bm = band_index(l, -m, p);
            if (bm >= 0) Ych[bm * YS + node] = ym;
          }
        };
        if (LPN == 1) {
          legendre_sweep(p, cx, sx, term, ltab);
        } else {
          legendre_columns4(p, r, cx, sx, term, ltab);
          // the four lanes of the point are adjacent: sum their columns' contributions
#pragma unroll
          for (int o = 1; o < LPN; o <<= 1)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              x[c] += __shfl_xor(x[c], o, 64);
              dt[c] += __shfl_xor(dt[c], o, 64);
              dp[c] += __shfl_xor(dp[c], o, 64);
            }
        }
        if (live && r == 0) {
          const double c0 = dt[1] * dp[2] - dt[2] * dp[1];
          const double c1 = dt[2] * dp[0] - dt[0] * dp[2];
          const double c2 = dt[0] * dp[1] - dt[1] * dp[0];
          const double J = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
          const double w = rW[q] * J;
          const double r0 = xt0 - x[0], r1 = xt1 - x[1], r2v = xt2 - x[2];
          const double d2 = r0 * r0 + r1 * r1 + r2v * r2v;
          const double di = 1.0 / sqrt(d2);
          const double di3 = di * di * di;
          const double ws = w * cS;
          Kwg[0 * NC + node] = ws * (di + r0 * r0 * di3);
          Kwg[1 * NC + node] = ws * (di + r1 * r1 * di3);
          Kwg[2 * NC + node] = ws * (di + r2v * r2v * di3);
          Kwg[3 * NC + node] = ws * r0 * r1 * di3;
          Kwg[4 * NC + node] = ws * r0 * r2v * di3;
          Kwg[5 * NC + node] = ws * r1 * r2v * di3;
          const double rn = r0 * nt0 + r1 * nt1 + r2v * nt2;
          const double wk = w * cK * rn * di3 * di * di;
          Kwg[6 * NC + node] = wk * r0 * r0;
          Kwg[7 * NC + node] = wk * r1 * r1;
          Kwg[8 * NC + node] = wk * r2v * r2v;
          Kwg[9 * NC + node] = wk * r0 * r1;
          Kwg[10 * NC + node] = wk * r0 * r2v;
          Kwg[11 * NC + node] = wk * r1 * r2v;
        } else if (r == 0) {
          for (int k = 0; k < 12; ++k) Kwg[k * NC + node] = 0.0;
        }
      } else {
        if (r == 0)
          for (int k = 0; k < 12; ++k) Kwg[k * NC + node] = 0.0;
        if (g == 0)
          for (int b = r; b < nB; b += LPN) Ych[b * YS + node] = 0.0;
      }
    }
    __syncthreads();
    if (tid < nB) {
      for (int q = 0; q < NC; ++q) {
        const double y = Ych[tid * YS + q];
#pragma unroll
        for (int gg = 0; gg < G; ++gg)
#pragma unroll
          for (int k = 0; k < 12; ++k) acc0[gg][k] += Kw[(gg * 12 + k) * NC + q] * y;
      }
    }
    if (G == 1 && tid + 256 < nB) {
      for (int q = 0; q < NC; ++q) {
        const double y = Ych[(tid + 256) * YS + q];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc1[k] += Kw[k * NC + q] * y;
      }
    }
  }
  __syncthreads();
  // C of every shape of the group, [G][12][nB], over the coefficient, harmonic and weight
  // buffers (the launcher checks that it fits there)
  double* Cs = lds;
  if (tid < nB)
#pragma unroll
    for (int gg = 0; gg < G; ++gg)
#pragma unroll
      for (int k = 0; k < 12; ++k) Cs[(gg * 12 + k) * nB + tid] = acc0[gg][k];
  if (G == 1 && tid + 256 < nB)
    for (int k = 0; k < 12; ++k) Cs[k * nB + tid + 256] = acc1[k];
  __syncthreads();
  const int ci[6] = {0, 1, 2, 0, 0, 1}, cj[6] = {0, 1, 2, 1, 2, 2};
  for (int gg = 0; gg < ng; ++gg) {
    const double* C = Cs + gg * 12 * nB;
    double* S = Sop + (size_t)(s0 + gg) * M3 * M3;
    double* K = Kop + (size_t)(s0 + gg) * M3 * M3;
    for (int a = tid; a < M; a += 256) {
      double v[12];
      for (int k = 0; k < 12; ++k) v[k] = 0.0;
      const double* f = Ft + (size_t)a * nB;
      for (int b = 0; b < nB; ++b) {
        const double fb = f[b];
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] += C[k * nB + b] * fb;
      }
      for (int k = 0; k < 6; ++k) {
        const int c = ci[k], cc = cj[k];
        const size_t rowA = (size_t)c * M + t, colA = (size_t)cc * M + a;
        S[colA * M3 + rowA] = v[k];
        K[colA * M3 + rowA] = v[6 + k];
        if (c != cc) {
          const size_t rowB = (size_t)cc * M + t, colB = (size_t)c * M + a;
          S[colB * M3 + rowB] = v[k];
          K[colB * M3 + rowB] = v[6 + k];
        }
      }
    }
  }
}

// LDS of k_singular<NC, G> in bytes; 0 if the per-shape results C ([G][12][nB]) would not
// fit over its coefficient, harmonic and weight buffers.
static size_t singular_group_lds(int p, int nc_nodes, int g) {
  const size_t nc = (size_t)(p + 1) * (p + 1), nB = (size_t)p * p + 2 * p;
  const size_t front = g * 3 * nc + nB * (nc_nodes + 1) + (size_t)g * 12 * nc_nodes;
  if ((size_t)g * 12 * nB > front) return 0;
  return (front + 2 * nc + 2 * (p + 1)) * sizeof(double);
}

hipError_t launch_singular_assemble(int ns, int p, int ps, double eta, const double* coef,
                                    const double* gx, const double* gn, const double* node_th,
                                    const double* node_ph, const double* rnodes, const double* rW,
                                    const double* Fttab, double* Sop, double* Kop, hipStream_t st) {
  // Two shapes per workgroup, 32 rotated nodes per chunk and four lanes per (node, shape),
  // each sweeping a quarter of the Legendre columns, when the two shapes' accumulators fit
  // one pass over B_p (nB <= 256) and two workgroups fit a CU's LDS; else one shape and
  // one lane per node with the largest chunk that lets two workgroups share a CU
  // (singular_chunk).  (Four shapes per workgroup need 48 accumulators per thread and
  // spill at two waves per SIMD.)
  constexpr size_t kLdsPerCu = 160 * 1024;
  const int M = (p + 1) * 2 * p, nB = p * p + 2 * p;
  int nodes = 0, group = 1;
  if (nB <= 256) {
    const size_t b = singular_group_lds(p, 32, 2);
    if (b && 2 * b <= kLdsPerCu) {
      nodes = 32;
      group = 2;
    }
  }
  if (!nodes) nodes = singular_chunk(p, 12);
  const size_t lds = singular_group_lds(p, nodes, group);
  if (!lds) return hipErrorInvalidValue;
  dim3 grid(M, (ns + group - 1) / group);
  auto run = [&](auto kern) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    kern<<<grid, 256, lds, st>>>(ns, p, ps, eta, coef, gx, gn, node_th, node_ph, rnodes, rW, Fttab, Sop, Kop);
    return hipSuccess;
  };
  hipError_t e;
  if (group == 2)
    e = run(k_singular<32, 2, 4>);
  else
    e = nodes == 64 ? run(k_singular<64, 1, 1>) : nodes == 48 ? run(k_singular<48, 1, 1>) : run(k_singular<32, 1, 1>);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// A0 += 1/2 I + L0 with L0[(c,a),(c',b)] = w_b [(1 + r_a.r_b) d_cc' - r_b[c] r_a[c']]
// (the augmentation L of §2.3 on the grid: int mu + (int r x mu) x r_a).
__global__ void k_finish_A0(int M, const double* gr_all, const double* gw_all, double* A0_all) {
  const int M3 = 3 * M;
  const int s = blockIdx.y;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)M3 * M3) return;
  const int col = (int)(e / M3), row = (int)(e % M3);
  const int c = row / M, a = row % M, cc = col / M, b = col % M;
  const double* r = gr_all + (size_t)s * 3 * M;
  const double wb = gw_all[(size_t)s * M + b];
  const double ra[3] = {r[a], r[M + a], r[2 * M + a]};
  const double rb[3] = {r[b], r[M + b], r[2 * M + b]};
  const double dot = ra[0] * rb[0] + ra[1] * rb[1] + ra[2] * rb[2];
  double v = wb * ((c == cc ? 1.0 + dot : 0.0) - rb[c] * ra[cc]);
  if (row == col) v += 0.5;
  A0_all[(size_t)s * M3 * M3 + e] += v;
}

hipError_t launch_finish_A0(int ns, int M, const double* gr, const double* gw, double* A0,
                            hipStream_t st) {
  const size_t tot = (size_t)9 * M * M;
  dim3 grid((unsigned)((tot + 255) / 256), ns);
  k_finish_A0<<<grid, 256, 0, st>>>(M, gr, gw, A0);
  return hipGetLastError();
}

// Velocity functional V0 = G' S0 (6 x 3M per shape): rows 0..2 average the self
// velocity over the surface, rows 3..5 give tau^{-1} int r x u (§3.3).
__global__ __launch_bounds__(64) void k_velocity_functional(int M, const double* Sop,
                                                            const double* gr_all,
                                                            const double* gw_all,
                                                            const double* shp_all, double* V0) {
  const int M3 = 3 * M;
  const int col = blockIdx.x, s = blockIdx.y, lane = threadIdx.x;
  const double* S = Sop + (size_t)s * M3 * M3 + (size_t)col * M3;
  const double* r = gr_all + (size_t)s * 3 * M;
  const double* w = gw_all + (size_t)s * M;
  const double* sp = shp_all + (size_t)s * 32;
  const double inva = 1.0 / sp[0];
  const double* ti = sp + 13;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int a = lane; a < M; a += 64) {
    const double u0 = S[a], u1 = S[M + a], u2 = S[2 * M + a];
    const double wa = w[a];
    const double r0 = r[a], r1 = r[M + a], r2 = r[2 * M + a];
    acc[0] += wa * u0 * inva;
    acc[1] += wa * u1 * inva;
    acc[2] += wa * u2 * inva;
    const double x0 = r1 * u2 - r2 * u1, x1 = r2 * u0 - r0 * u2, x2 = r0 * u1 - r1 * u0;
    acc[3] += wa * (ti[0] * x0 + ti[1] * x1 + ti[2] * x2);
    acc[4] += wa * (ti[3] * x0 + ti[4] * x1 + ti[5] * x2);
    acc[5] += wa * (ti[6] * x0 + ti[7] * x1 + ti[8] * x2);
  }
  for (int k = 0; k < 6; ++k) {
    const double v = wave_sum(acc[k]);
    if (lane == 0) V0[((size_t)s * 6 + k) * M3 + col] = v;
  }
}

hipError_t launch_velocity_functional(int ns, int M, const double* Sop, const double* gr,
                                      const double* gw, const double* shp, double* V0,
                                      hipStream_t st) {
  dim3 grid(3 * M, ns);
  k_velocity_functional<<<grid, 64, 0, st>>>(M, Sop, gr, gw, shp, V0);
  return hipGetLastError();
}

// In-place Gauss-Jordan inversion with partial pivoting, one workgroup per matrix,
// column-major A[j*n + i] = a_ij, blocked by panels of nb pivots.  Each unblocked step on
// pivot k: search column k, swap rows k and p across all n columns, scale the pivot row,
// eliminate column k from every other row, and store the step's transformation column
// in column k.  Within a panel P = [k0, k0 + nb) the scaling and elimination touch only
// the panel's columns; the panel columns then hold the panel's transformation T
// restricted to P (T differs from I only in those columns), so every other column is
// brought up to date at once by the rank-nb update A(:, J) += (T(:, P) - I_P) A_old(P, J),
// with the panel rows A_old(P, J) staged in LDS.  This reads and writes the matrix once
// per panel instead of once per pivot.  Finally the row interchanges are undone as
// column interchanges in reverse order.
template <int NB>
__global__ __launch_bounds__(1024) void k_gauss_jordan(int n, double* A_all, int* piv_all) {
  constexpr int nb = NB;
  extern __shared__ double sh[];
  double* rows = sh;                 // [nb][n] panel rows before the rank-nb update
  double* rowk = rows + (size_t)nb * n;  // [nb] scaled pivot row within the panel
  double* rv = rowk + nb;            // [16]
  int* ri = (int*)(rv + 16);         // [16]
  __shared__ int pivot_row;
  __shared__ double pivinv_s;
  const int s = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  double* A = A_all + (size_t)s * n * n;
  int* piv = piv_all + (size_t)s * n;
  for (int k0 = 0; k0 < n; k0 += nb) {
    const int kb = min(nb, n - k0);
    for (int k = k0; k < k0 + kb; ++k) {
      // pivot: max |a_ik|, i >= k (ties -> smallest i)
      double best = -1.0;
      int bi = n;
      for (int i = k + tid; i < n; i += nt) {
        const double v = fabs(A[(size_t)k * n + i]);
        if (v > best) { best = v; bi = i; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
      }
      if ((tid & 63) == 0) { rv[tid >> 6] = best; ri[tid >> 6] = bi; }
      __syncthreads();
      if (tid == 0) {
        double b = rv[0];
        int i0 = ri[0];
        for (int w = 1; w < nt / 64; ++w)
          if (rv[w] > b || (rv[w] == b && ri[w] < i0)) { b = rv[w]; i0 = ri[w]; }
        pivot_row = i0;
        piv[k] = i0;
      }
      __syncthreads();
      const int pr = pivot_row;
      if (pr != k) {
        for (int j = tid; j < n; j += nt) {
          const double t1 = A[(size_t)j * n + k];
          A[(size_t)j * n + k] = A[(size_t)j * n + pr];
          A[(size_t)j * n + pr] = t1;
        }
      }
      __syncthreads();
      if (tid == 0) pivinv_s = 1.0 / A[(size_t)k * n + k];
      __syncthreads();
      const double pivinv = pivinv_s;
      for (int j = k0 + tid; j < k0 + kb; j += nt) {
        const double v = (j == k ? 1.0 : A[(size_t)j * n + k]) * pivinv;
        rowk[j - k0] = v;
        A[(size_t)j * n + k] = v;
      }
      __syncthreads();
      for (int i = tid; i < n; i += nt) {
        if (i == k) continue;
        const double f = A[(size_t)k * n + i];
        for (int j = k0; j < k0 + kb; ++j) {
          const double old = (j == k) ? 0.0 : A[(size_t)j * n + i];
          A[(size_t)j * n + i] = old - f * rowk[j - k0];
        }
      }
      __syncthreads();
    }
    // rank-kb update of the columns outside the panel (rows and multipliers of a partial
    // last panel are zero past kb)
    for (int e = tid; e < nb * n; e += nt) {
      const int q = e / n, j = e - q * n;
      rows[(size_t)q * n + j] = q < kb ? A[(size_t)j * n + k0 + q] : 0.0;
    }
    __syncthreads();
    for (int i = tid; i < n; i += nt) {
      double w[nb];
#pragma unroll
      for (int q = 0; q < nb; ++q) {
        const int col = min(k0 + q, n - 1);
        const double a = A[(size_t)col * n + i] - (i == col ? 1.0 : 0.0);
        w[q] = q < kb ? a : 0.0;
      }
      // the columns before and after the panel, four at a time: four independent loads
      // in flight per wave, and the staged rows read as pairs of doubles (aligned: n = 3M
      // is even and both ranges start at a multiple of 4)
      auto update = [&](int j, int j1) {
        for (; j + 4 <= j1; j += 4) {
          double v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = A[(size_t)(j + u) * n + i];
#pragma unroll
          for (int q = 0; q < nb; ++q) {
            const double2 r01 = *reinterpret_cast<const double2*>(rows + (size_t)q * n + j);
            const double2 r23 = *reinterpret_cast<const double2*>(rows + (size_t)q * n + j + 2);
            v[0] = fma(w[q], r01.x, v[0]);
            v[1] = fma(w[q], r01.y, v[1]);
            v[2] = fma(w[q], r23.x, v[2]);
            v[3] = fma(w[q], r23.y, v[3]);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) A[(size_t)(j + u) * n + i] = v[u];
        }
        for (; j < j1; ++j) {
          double v = A[(size_t)j * n + i];
#pragma unroll
          for (int q = 0; q < nb; ++q) v = fma(w[q], rows[(size_t)q * n + j], v);
          A[(size_t)j * n + i] = v;
        }
      };
      update(0, k0);
      update(k0 + kb, n);
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const int pr = piv[k];
    if (pr != k) {
      for (int i = tid; i < n; i += nt) {
        const double t1 = A[(size_t)k * n + i];
        A[(size_t)k * n + i] = A[(size_t)pr * n + i];
        A[(size_t)pr * n + i] = t1;
      }
    }
    __syncthreads();
  }
}

template <int NB>
static hipError_t gj_launch(int ns, int n, double* A, int* piv, hipStream_t st) {
  const size_t lds = ((size_t)NB * n + NB + 16) * sizeof(double) + 16 * sizeof(int);
  hipError_t e = hipFuncSetAttribute((const void*)k_gauss_jordan<NB>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  k_gauss_jordan<NB><<<ns, 1024, lds, st>>>(n, A, piv);
  return hipGetLastError();
}

// Panel width: the largest power of two (at most 16: the multipliers live in registers,
// and 1024 threads leave 128 VGPRs) whose staged panel rows fit 128 KiB of LDS.
hipError_t launch_gauss_jordan(int ns, int n, double* A, int* piv, hipStream_t st) {
  const size_t fit = (128 * 1024) / (8 * (size_t)n);
  if (fit >= 16) return gj_launch<16>(ns, n, A, piv, st);
  if (fit >= 8) return gj_launch<8>(ns, n, A, piv, st);
  if (fit >= 4) return gj_launch<4>(ns, n, A, piv, st);
  if (fit >= 2) return gj_launch<2>(ns, n, A, piv, st);
  return gj_launch<1>(ns, n, A, piv, st);
}

__global__ void k_cast_f32(size_t n, const double* x, float* y) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

__global__ void k_cast_bf16(size_t n, const double* x, uint16_t* y) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float f = (float)x[i];
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
  y[i] = (uint16_t)(u >> 16);
}

hipError_t launch_cast_f32(size_t n, const double* x, float* y, hipStream_t st) {
  k_cast_f32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, x, y);
  return hipGetLastError();
}

hipError_t launch_cast_bf16(size_t n, const double* x, uint16_t* y, hipStream_t st) {
  k_cast_bf16<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, x, y);
  return hipGetLastError();
}

}  // namespace rbm
