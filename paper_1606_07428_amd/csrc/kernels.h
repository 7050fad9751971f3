// Launchers of the gfx950 kernels (host side).  Every launcher enqueues on `st`
// and returns the hipError_t of the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rbm {

hipError_t launch_gemm_bf16(int m, int n, int k, const uint16_t* A, long sa0, long sa1,
                            const uint16_t* B, long sb0, long sb1, float* C, int ldc,
                            const float* bias, float alpha, float beta, hipStream_t st);

// ---- setup (k_setup.hip) ------------------------------------------------------
hipError_t launch_gauss_legendre(int n, double* t, double* w, hipStream_t st);
// grid tables: Y, dY/dtheta, (dY/dphi)/sin(theta) [(p+1)^2][M]; forward matrix F [nB][M];
// transposed forward matrix Ft [M][nB]; node theta/phi/lambda [M].
hipError_t launch_grid_tables(int p, const double* gl_t, const double* gl_w, double* Ytab,
                              double* Yttab, double* Ypstab, double* Ftab, double* Fttab,
                              double* node_th, double* node_ph, double* node_lam, hipStream_t st);
// rotated grid of order ps: nodes [3][Ms] and singular weights [Ms]
hipError_t launch_rotated_rule(int ps, const double* glt, const double* glw, double* nodes,
                               double* W, hipStream_t st);
hipError_t launch_radial_to_coef(int ns, int p, int nrc, const double* rc, const double* Ytab,
                                 const double* Ftab, const double* node_th, const double* node_ph,
                                 double* coef, hipStream_t st);
hipError_t launch_shape_geometry(int ns, int p, const double* coef, const double* Ytab,
                                 const double* Yttab, const double* Ypstab, const double* node_lam,
                                 double* gx, double* gn, double* gw, double* gr, double* shp,
                                 hipStream_t st);
hipError_t launch_singular_assemble(int ns, int p, int ps, double eta, const double* coef,
                                    const double* gx, const double* gn, const double* node_th,
                                    const double* node_ph, const double* rnodes, const double* rW,
                                    const double* Fttab, double* Sop, double* Kop, hipStream_t st);
hipError_t launch_finish_A0(int ns, int M, const double* gr, const double* gw, double* A0,
                            hipStream_t st);
hipError_t launch_velocity_functional(int ns, int M, const double* Sop, const double* gr,
                                      const double* gw, const double* shp, double* V0,
                                      hipStream_t st);
hipError_t launch_gauss_jordan(int ns, int n, double* A, int* piv, hipStream_t st);
hipError_t launch_cast_f32(size_t n, const double* x, float* y, hipStream_t st);
// bf16 stored as raw uint16 (upper half of the fp32 pattern, round to nearest even)
hipError_t launch_cast_bf16(size_t n, const double* x, uint16_t* y, hipStream_t st);

// ---- per-solve geometry and densities (k_solve.hip) ------------------------------
hipError_t launch_body_prep(int n, const double* quat, const int* sid, const double* shp,
                            double* Rm, double* tauinv_lab, double* area_b, hipStream_t st);
hipError_t launch_nodes(int n, int M, const int* sid, const double* cen, const double* Rm,
                        const double* gr, const double* gn, const double* gw, double* X,
                        double* Nn, double* W, float* Xf, float* Nf, hipStream_t st);
hipError_t launch_rho(int n, int M, const double* FT, const double* cen, const double* X,
                      const double* tauinv_lab, const double* area_b, double* rho, hipStream_t st);
// per-body moments of a lab field u[3][N]: out[i] = (sum w u, sum w (X-c) x u)
hipError_t launch_moments(int n, int M, const double* u, const double* X, const double* W,
                          const double* cen, double* mom, hipStream_t st);
// out = a*x + b*y + L-like term: out_g += sign * (F_i + T_i x (X_g - c_i)) from mom
hipError_t launch_add_rigid(int n, int M, const double* mom, const double* X, const double* cen,
                            double sign, double* out, hipStream_t st);
hipError_t launch_velocity_self(int n, int M, const int* sid, const double* V0, const double* Rm,
                                const double* sig, double* vw_self, hipStream_t st);
hipError_t launch_velocity_final(int n, const double* mom_far, const double* vw_self,
                                 const double* tauinv_lab, const double* area_b, double* VW,
                                 hipStream_t st);

// RK4 on (c, q): stage pose y0 + a dt k; derivative and weighted accumulation; final update.
hipError_t launch_rk_stage(int n, const double* c0, const double* q0, const double* k, double a,
                           double dt, double* cen, double* quat, hipStream_t st);
hipError_t launch_rk_deriv(int n, const double* VW, const double* quat, double* k, double* acc,
                           double wgt, int first, hipStream_t st);
hipError_t launch_rk_final(int n, const double* c0, const double* q0, const double* acc, double dt,
                           double* cen, double* quat, hipStream_t st);

// ---- per-body operator apply (k_self.hip) ----------------------------------------
// y_body[3][N] = A_{s(i)} (R_i^T x_lab) per body; A column-major [ns][3M][3M].
template <typename TM>
hipError_t launch_self_apply(int n, int M, const int* sid, const TM* A, const double* Rm,
                             const double* x_lab, double* y_body, hipStream_t st);

// One shape shared by every body: Z = A [R_i^T x_i] as an MFMA GEMM (float64, float32) or
// the bf16 MFMA GEMM; scratchB holds 3N operand values, scratchZ 3N floats (bf16 only).
template <typename TM>
hipError_t launch_self_apply_shared(int n, int M, const TM* A, const double* Rm,
                                    const double* x_lab, void* scratchB, void* scratchZ,
                                    double* y_body, hipStream_t st);

// ---- far field (k_far.hip) -------------------------------------------------------
// Pack sources: (X_g, q_g) with q_g = W_g * (R_i z_body or z_lab)[g] into AoS of T.
// If z_lab_out != nullptr the rotated z is also written (lab frame, float64).
template <typename T>
hipError_t launch_pack_sources(int N, int M, const double* X, const double* W, const double* Rm,
                               const double* z, int z_is_body, double* z_lab_out, void* src,
                               hipStream_t st);
// kind 0 = traction (targets need normals), 1 = Stokeslet.  Writes nsplit partial sums
// part[nsplit][3][N] (float64).  Returns the split used through *nsplit_out.
template <typename T>
hipError_t launch_far(int kind, int N, int M, const T* tx, const T* nrm, const void* src,
                      double* part, int nsplit, hipStream_t st);
// float64 traction (into part_t, as kind 0) and Stokeslet (into part_u, as kind 1) sums of the
// same packed sources in one pass, nsplit partial sums each
hipError_t launch_far_ts(int N, int M, const double* tx, const double* nrm, const void* src, double* part_t,
                         double* part_u, int nsplit, hipStream_t st);
// out[3][N] = ca * a[3][N] (optional) + cb * R_i b_body (optional) + cp * sum_s part[s];
// out may be the same array as a, never as b_body
hipError_t launch_combine(int N, int M, int nsplit, const double* part, double cp,
                          const double* a, double ca, const double* b_body, const double* Rm,
                          double cb, double* out, hipStream_t st);

// ---- Krylov (k_krylov.hip) --------------------------------------------------------
hipError_t launch_dots(int kk, size_t len, const double* V, size_t ldv, const double* w,
                       double* partial, int nblk, hipStream_t st);
// w -= sum_j V[j] h[j]  (or w = sum_j V[j] h[j] if overwrite)
hipError_t launch_vupdate(int kk, size_t len, const double* V, size_t ldv, const double* h,
                          double* w, int overwrite, hipStream_t st);
hipError_t launch_axpby(size_t len, double a, const double* x, double b, const double* y,
                        double* out, hipStream_t st);
hipError_t launch_backsolve(int m, int ldh, const double* H, const double* g, double* y,
                            hipStream_t st);
hipError_t launch_dots_final_sqrt(int nblk, const double* partial, double* h, hipStream_t st);
// GMRES cycle start: V0 = r / rnorm (0 if rnorm = 0), g[0] = rnorm and g[1..ng) = 0,
// H[0..nh) = 0.
hipError_t launch_gmres_init(size_t len, const double* r, double rnorm, double* V0, int ng, double* g,
                             size_t nh, double* H, hipStream_t st);
// One Arnoldi step after w = V[k+1] has been formed: CGS2 against V[0..k] (column k of H),
// w normalised and ||w|| into H, the Givens rotations of column k, g updated and
// |g_{k+1}| written to resid (which may be mapped host memory).  partial holds three
// regions pstride doubles apart, each at least (k + 1) * nblk.
hipError_t launch_arnoldi(int k, size_t len, double* V, size_t ldv, double* partial, size_t pstride,
                          int nblk, int ldh, double* H, double* cs, double* sn, double* g,
                          double* resid, hipStream_t st);

// ---- learned warm start (k_mlp.hip) --------------------------------------------------
hipError_t launch_gemm_bf16(int m, int n, int k, const uint16_t* A, long sa0, long sa1,
                            const uint16_t* B, long sb0, long sb1, float* C, int ldc,
                            const float* bias, float alpha, float beta, hipStream_t st);
hipError_t launch_silu_fwd(size_t cnt, const float* Z, float* H, uint16_t* Hb, hipStream_t st);
hipError_t launch_silu_bwd(size_t cnt, const float* dH, const float* Z, float* dZ, uint16_t* dZb,
                           hipStream_t st);
hipError_t launch_mse(size_t cnt, float inv, const float* Y, const float* T, float* dY,
                      uint16_t* dYb, double* part, hipStream_t st);
hipError_t launch_sum_parts(int nparts, const double* part, double scale, double* out, int accumulate,
                            hipStream_t st);
hipError_t launch_colsum(int rows, int cols, const float* dZ, float* db, hipStream_t st);
hipError_t launch_adam(size_t cnt, float* P, const float* G, float* m, float* v, float lr, float b1,
                       float b2, float eps, int t, uint16_t* Pb, hipStream_t st);
hipError_t launch_to_bf16(size_t cnt, const float* x, uint16_t* y, hipStream_t st);
hipError_t launch_features(int n, int k, int S, const double* cen, const double* Rm,
                           const double* FT, const int* sid, const double* desc, float* X,
                           hipStream_t st);
hipError_t launch_gather(int rows, int F, int O, const int* idx, const float* X, const float* mean,
                         const float* istd, uint16_t* Xb, const float* T, float tinv, float* Tb,
                         hipStream_t st);
hipError_t launch_colstats(int rows, int F, const float* X, float* mean, float* istd,
                           hipStream_t st);
hipError_t launch_rms(size_t cnt, const float* T, float* out, hipStream_t st);
hipError_t launch_band_synth(int n, int M, int p, const float* coef, const float* scale,
                             const double* Ytab, const double* Rm, double* mu, hipStream_t st);
hipError_t launch_band_analysis(int n, int M, int p, const double* dmu, const double* Rm,
                                const double* Ftab, float* out, hipStream_t st);

// ---- near-singular correction by upsampling (k_near.hip) --------------------------
// fine nodes r' [ns][3][Mu], weights w' [ns][Mu], bounding radii rb [ns] at order pu
hipError_t launch_fine_geometry(int ns, int p, int pu, const double* coef, const double* glu_t,
                                const double* glu_w, const double* shp, double* fr, double* fw,
                                double* rb, hipStream_t st);
// band-limited interpolation coarse -> fine, column-major [M][Mu]
hipError_t launch_interp_matrix(int p, int pu, const double* gl_t, const double* gl_w,
                                const double* glu_t, double* U, hipStream_t st);
// near list per body (increasing j, at most kmax stored) and true counts
hipError_t launch_near_list(int n, int M, int kmax, double kappa, const double* cen, const int* sid,
                            const double* rb, const double* shp, int* nbr, int* cnt, hipStream_t st);
// fine-minus-plain sums for near pairs (kind 0 traction, 1 Stokeslet) of the density z ([3][N],
// body frames when z_is_body) whose plain sources are packed in src: fine sources of the nneed
// bodies listed in need (into srcf, n*Mu packed sources), nitems work items of ch list positions
// (item_body, item_pos) into slots [nitems][3][M], then per body the ordered sum of its items
// (item_first[i] .. item_first[i+1]-1) into res [3][N] (zero for bodies without near bodies)
template <typename T>
hipError_t launch_near_corr(int kind, int n, int M, int Mu, int kmax, int nneed, const int* need,
                            int nitems, int ch, const int* item_body, const int* item_pos,
                            const int* item_first, const T* tx, const T* tn, const void* src,
                            const double* z, int z_is_body, const double* U, const int* sid,
                            const double* cen, const double* Rm, const double* fr, const double* fw,
                            const int* nbr, const int* cnt, void* srcf, double* slots, double* res,
                            hipStream_t st);

// contact search: closest node pair of each candidate body pair (cand [k][2]): out [k][5] =
// (distance^2, node-pair index ia*M + ib, midpoint x*)
hipError_t launch_closest_pairs(int ncand, int N, int M, const int* cand, const double* X, double* out,
                                hipStream_t st);
// overlap test: out [k][2] = min over the nodes y of one body of (y - X_r) . N_r, X_r the
// other body's node nearest to y (dir 0: nodes of b against a, dir 1: nodes of a against b)
hipError_t launch_overlap_depth(int ncand, int N, int M, const int* cand, const double* X, const double* Nn,
                                double* out, hipStream_t st);
// hs[s] = largest nearest-neighbour spacing of the M points r [ns][3][M]
hipError_t launch_node_spacing(int ns, int M, const double* r, double* hs, hipStream_t st);
// rb[s] = max_a |r_a| over the M points r [ns][3][M]
hipError_t launch_bound_radius(int ns, int M, const double* r, double* rb, hipStream_t st);

// Fast multipole far field (k_fmm.hip).  Expansion orders up to kFmmMaxOrder; a tree is
// usable when no leaf holds more than kFmmLeafCap points.
constexpr int kFmmMaxOrder = 16;
constexpr int kFmmLeafCap = 4096;
hipError_t launch_fmm_bounds(int N, const double* X, double* out6, hipStream_t st);
hipError_t launch_fmm_sort_points(int N, int M, const double* X, const double* Nn, const double* lo, double w,
                                  int nb, int* leaf, int* cnt, int* start, int* fill, int* perm, int* maxcnt,
                                  double4* Xs, double4* Ns, hipStream_t st);
hipError_t launch_fmm_finish_tree(int N, int M, int L, const double* X, const double* Nn, const int* start,
                                  int* perm, double4* Xs, double4* Ns, int* const* cnt_lev, int* tcnt, int* toff,
                                  int2* task, int* scratch, hipStream_t st);
template <typename T>
hipError_t launch_fmm_tables(int P, int L, double D, void* tabR, void* tabI, hipStream_t st);
template <typename T>
hipError_t launch_fmm_apply(int P, int L, const double* lo, double D, int N, const int* start, const int* perm,
                            const double4* Xs, const double4* Ns, int* const* cnt_lev, const size_t* lev_off,
                            int ntask, const int2* task, const void* tabR, const void* tabI, const void* src,
                            void* srt, void* Mexp, void* Lexp, double* out, hipStream_t st);

// ---- magnetostatics (k_magnetic.hip) -------------------------------------------------
// Laplace self operators S^L, K^L per shape, column-major [ns][M][M] (singular rule)
hipError_t launch_singular_laplace(int ns, int p, int ps, const double* coef, const double* gx,
                                   const double* gn, const double* node_th, const double* node_ph,
                                   const double* rnodes, const double* rW, const double* Fttab,
                                   double* SL, double* KL, hipStream_t st);
// spectral derivative matrices Dt, Dp (column-major M x M) and shape tangents [ns][6][M]
hipError_t launch_magnetic_tables(int p, int ns, const double* coef, const double* Yttab,
                                  const double* Ypstab, const double* Ftab, double* Dt, double* Dp,
                                  double* tang, hipStream_t st);
// y = A_{s(i)} x per body, scalar node vectors
hipError_t launch_scalar_self(int n, int M, const int* sid, const double* A, const double* x, double* y,
                              hipStream_t st);
hipError_t launch_pack_scalar(int N, const double* X, const double* W, const double* q, void* src,
                              hipStream_t st);
// out = cv v + cs self + cp sum of the split slots' first component (v, self may be NULL)
hipError_t launch_scalar_combine(int N, int nsplit, const double* part, double cp, const double* self,
                                 double cs, const double* v, double cv, double* out, hipStream_t st);
// out = (accumulate ? out : 0) + scale (h . V_g), V [3][N]
hipError_t launch_hdot(int N, const double* V, double h0, double h1, double h2, double scale,
                       int accumulate, double* out, hipStream_t st);
// exterior field and Maxwell traction rho [3][N] from phi and the exterior normal derivative dn
hipError_t launch_magnetic_traction(int n, int M, const int* sid, const double* Rm, const double* Nn,
                                    const double* tang, const double* Dt, const double* Dp,
                                    const double* phi, const double* dn, double mu0, double* rho,
                                    hipStream_t st);

}  // namespace rbm
