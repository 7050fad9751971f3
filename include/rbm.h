/*
 * rbm.h - C ABI of the MI355X (gfx950) rigid-body Stokes mobility library.
 *
 * The library solves the mobility problem of Corona, Greengard, Rachh and
 * Veerapaneni, "An integral equation formulation for rigid bodies in Stokes flow
 * in three dimensions" (arXiv 1606.07428): given body shapes, centroids,
 * orientations, forces F_i and torques T_i (§1, mobility relation V = M F), it
 * returns the translational and rotational velocities (v_i, omega_i), using the
 * single-layer second-kind formulation of §2.3 (augmented operator 1/2 I + K + L)
 * discretized with spherical harmonics (§3), the rotated-grid singular self
 * quadrature (§3, §3.1) and right block-diagonal preconditioned GMRES (§3.2).
 * Interactions between bodies are a direct all-pairs sum on the GPU.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All real arrays are float64 and C-contiguous.  Host arrays are owned by the
 *    caller; the library copies what it needs and writes outputs only into
 *    caller buffers.
 *  - The library allocates no device memory.  The caller queries the size with
 *    rbm_workspace_size() and binds one device buffer (e.g. a PyTorch tensor) with
 *    rbm_bind_workspace(); all device state lives there.  Work is issued on the
 *    stream given in rbm_options (NULL = the default stream).
 *  - Spherical harmonics: real orthonormal basis, index l*l + l + m,
 *      Y_l0 = N_l0 P_l(cos t), Y_lm = sqrt2 N_lm P_l^m(cos t) cos(m f) (m > 0),
 *      Y_l,-m = sqrt2 N_lm P_l^m(cos t) sin(m f), no Condon-Shortley phase
 *    (the paper's Y_n^m with P_n^|m| of §3, made real).
 *  - Grid (§3): p+1 Gauss-Legendre nodes in cos(theta) (ascending) times 2p
 *    azimuths phi_k = pi k / p; node a = j*2p + k, M = 2p(p+1) nodes per body.
 *    Density arrays are component-major [3][N], N = n*M, body i's node a at
 *    column i*M + a, in the lab frame.
 *  - Poses: the body frame is the shape's frame recentred at its area centroid;
 *    quat = (w, x, y, z) rotates body to lab; centre = lab position of the area
 *    centroid.  Torques are about that centroid.  F_i is the force the body exerts
 *    on the fluid (traction integrates to -F_i), so an isolated sphere of radius a
 *    moves with v = F/(6 pi eta a), omega = T/(8 pi eta a^3).
 *  - Tracing: with the environment variable RBM_VERBOSE set when a context is created, its
 *    solves print each refinement's residual kind and size and each GMRES cycle's iterations
 *    to stderr.
 *  - Errors: every call returns an rbm_status; rbm_last_error() gives a
 *    thread-local message.  No call throws across the ABI.  Calls on one context
 *    are not thread safe; different contexts are independent.
 *  - Overlap: the formulation of §2 assumes disjoint bodies.  Whenever poses change
 *    (the first solve after rbm_set_bodies, every RK4 stage) bodies whose bounding
 *    spheres (largest centroid-to-node distance) intersect are compared node by node:
 *    for each node y of one body, X the nearest node of the other and N its outward
 *    normal, (y - X).N < -h^2 (h the other shape's largest nearest-neighbour node
 *    spacing) marks y as inside, and the call returns RBM_E_OVERLAP without solving.
 *    Separated bodies never trip the test however close they are; penetrations shallower
 *    than about h^2 may pass it.
 */
#ifndef RBM_H
#define RBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rbm_ctx rbm_ctx;

typedef enum {
  RBM_OK = 0,
  RBM_E_INVAL = -1,   /* bad argument (sizes, NaN/Inf input, unknown shape id, ...) */
  RBM_E_NOMEM = -2,   /* no workspace bound, or the bound one is too small */
  RBM_E_DEVICE = -3,  /* a HIP runtime call failed */
  RBM_E_NOCONV = -4,  /* GMRES hit max_iter before tol; outputs are still written */
  RBM_E_OVERLAP = -5, /* two bodies overlap at the poses of a solve or RK4 stage (see below) */
  RBM_E_STATE = -6    /* call out of order (e.g. solve before setup) */
} rbm_status;

typedef enum {
  RBM_FP64 = 0,        /* everything in float64 */
  RBM_MIXED_FP32 = 1,  /* GMRES-IR: fp32 far sum + fp32 preconditioner, fp64 residuals after the
                          first refinement (which starts from the fp32 / FMM residual) */
  RBM_MIXED_BF16 = 2   /* GMRES-IR: fp32 far sum + bf16 preconditioner (fp32 accumulate) */
} rbm_precision;

typedef enum {
  RBM_GUESS_ZERO = 0,       /* mu_0 = 0 */
  RBM_GUESS_BLOCKDIAG = 1,  /* mu_0 = P^{-1} b, P = block-diagonal self operator (§3.2) */
  RBM_GUESS_USER = 2,       /* mu_0 taken from rbm_set_guess_dev() */
  RBM_GUESS_LEARNED = 3     /* mu_0 = mu_BD + network correction, falling back to mu_BD when its
                               residual is worse than the block-diagonal guess's (see learned API) */
} rbm_guess;

typedef struct {
  int p;            /* SH order, 2 <= p <= 20; M = 2p(p+1) nodes per body */
  int p_sing;       /* order of the rotated grid of the singular rule; 0 -> 2p; >= p+1 */
  double eta;       /* viscosity (> 0) */
  double tol;       /* stop when ||b - A mu||_2 <= tol ||b||_2 */
  int max_iter;     /* Krylov dimension (iterations per GMRES cycle), 1..400 */
  int max_restart;  /* extra GMRES cycles allowed after the first (>= 0) */
  int precision;    /* rbm_precision */
  int guess;        /* rbm_guess */
  double inner_tol; /* GMRES-IR inner relative tolerance (0 -> 1e-4) */
  void* stream;     /* hipStream_t or NULL */
  int p_up;           /* near-singular upsampling (§3): 0 = off (every off-body pair uses the
                         smooth rule of order p); else the order p_u of the finer grid, in
                         [p+1, 48], used for every pair of bodies that are near */
  double near_factor; /* kappa of the near test |c_i - c_j| < R_i + R_j + kappa h_j (R: largest
                         centroid-to-node distance on the fine grid, h_j = sqrt(|Gamma_j|/M));
                         0 -> 5 */
  double contact_delta; /* rbm_step_rk4 only: > 0 switches on the contact forces of §3.3 at every
                           stage (bodies whose closest nodes are within contact_delta, see
                           rbm_find_contacts / rbm_solve_contacts); 0 = off */
  int magnetic;         /* 1: set up the Laplace operators of the magnetostatic problem (§4) for
                           rbm_magnetic_traction_dev and rbm_step_rk4_magnetic (two M x M
                           operators per shape); 0 = off */
  int fmm_order;        /* > 0: order P in [2, 16] of the fast multipole far field (the O(N)
                           equivalent of the FMM of §3.1) used by the inner GMRES of the
                           precision form (precision FP32/BF16) in place of the direct float32
                           sum; outer residuals stay direct float64, so the solve still meets
                           tol.  0 = off (direct sums everywhere) */
  int fmm_max_level;    /* deepest octree level the FMM may use, in [2, 6] (workspace grows as
                           8^level); 0 -> 5 */
  int gmres_lookahead;  /* queueing of GMRES iterations (§3.2): 1 (default) queues iteration
                           k+1 before iteration k's residual estimate is read while the
                           estimates fall steadily and the next is predicted above 8 times the
                           tolerance; 0 never, 2 always (then a converged cycle may run one
                           iteration whose result is discarded).  The iterates and the
                           solution are the same in every mode. */
  double ir_stall;      /* precision form: a refinement whose float64 residual is not below
                           ir_stall times the previous one counts as stalled, and the remaining
                           refinements run their GMRES cycles with float64 operators (exact far
                           sums, float64 preconditioner) to the tolerance; 0 -> 0.5 */
  int velocity_fusion;  /* 1 (default): when a float64 residual is predicted to meet tol, its
                           traction sum and the velocities' Stokeslet sum of the same density
                           rho + mu come from one fused pass; 0: always a separate Stokeslet sum */
} rbm_options;

typedef struct {
  int iters;          /* total inner GMRES iterations */
  int matvecs;        /* applications of the full operator (all precisions) */
  int refinements;    /* GMRES-IR outer steps (0 for RBM_FP64) */
  int cycles;         /* GMRES cycles (restarts + 1) */
  double rel_residual;/* final ||b - A mu|| / ||b|| in float64 */
  double bnorm;       /* ||b|| */
  double ms_total;    /* wall time of the solve on the stream (ms) */
  double ms_far;      /* time in the all-pairs sums (ms, event-timed) */
  double ms_self;     /* time in the per-body operator applies (ms) */
  double far_pairs;   /* off-body pair interactions evaluated (all sums) */
  int n_traction;     /* launches of the float64 traction sum kernel */
  int n_stokeslet;    /* launches of the Stokeslet sum kernel */
  double ms_traction; /* summed duration of the float64 traction kernel launches (ms) */
  double ms_stokeslet;/* summed duration of the Stokeslet kernel launches (ms) */
  double pairs_per_launch; /* off-body pairs of one launch: N^2 - n M^2 */
  int guess_used;     /* rbm_guess actually used for mu_0 */
  int fallback_used;  /* 1 if the learned guess was rejected for the block-diagonal one */
  double init_rel_residual; /* ||b - A mu_0|| / ||b|| (precision form: with the far sum of its inner
                               operators, the residual its first refinement starts from) */
  int near_pairs;     /* ordered near body pairs of the upsampled rule (0 when off) */
  double ms_near;     /* device time of the near-singular corrections (interpolation, sums) */
  int fmm_level;      /* leaf level of the fast multipole tree of this solve (-1: not used) */
  int fmm_applies;    /* far sums evaluated by the fast multipole method */
  int n_traction32;   /* float32 traction sums (direct kernel or fast multipole method) */
  double ms_traction32; /* their summed duration (ms) */
  int fp64_cycles;    /* precision form: GMRES cycles run with float64 operators after a stalled
                         refinement (see rbm_options.ir_stall) */
  int n_fused;        /* float64 residuals evaluated by the fused traction + Stokeslet pass (when
                         the residual was predicted to meet tol) */
  int fused_used;     /* 1 if the velocities took the Stokeslet sum of such a pass */
  double ms_fused;    /* summed duration of the fused pass launches (ms) */
} rbm_solve_info;

/* Default options: p = 8, p_sing = 0, eta = 1, tol = 1e-12, max_iter = 100,
 * max_restart = 4, RBM_FP64, RBM_GUESS_BLOCKDIAG, inner_tol = 1e-4, stream NULL,
 * ir_stall = 0.5, velocity_fusion = 1. */
void rbm_default_options(rbm_options* opt);

/* Create a context.  Validates opt; no device work. */
rbm_status rbm_create(const rbm_options* opt, rbm_ctx** out);
void rbm_destroy(rbm_ctx* ctx);

/* Shapes as coordinate-function coefficients (§3, truncated SH expansion of x):
 * coef[n_shapes][3][(lmax+1)^2] in the body frame, lmax <= p-1. */
rbm_status rbm_set_shapes(rbm_ctx* ctx, int n_shapes, int lmax, const double* coef);

/* Shapes as radial functions r(s) = sum rc_lm Y_lm(s), x = r(s) s:
 * rc[n_shapes][(lmax+1)^2], lmax <= p-2 (x then has degree lmax+1 <= p-1 and is
 * converted exactly to coordinate coefficients on the device). */
rbm_status rbm_set_shapes_radial(rbm_ctx* ctx, int n_shapes, int lmax, const double* rc);

/* Bodies: shape_id[n] in [0, n_shapes), centre[n][3] (lab area centroids),
 * quat[n][4] (w,x,y,z; renormalised if | |q| - 1 | < 1e-6, else RBM_E_INVAL).
 * n may change between calls as long as it stays <= the n the workspace was
 * sized for. */
rbm_status rbm_set_bodies(rbm_ctx* ctx, int n, const int* shape_id,
                          const double* centre, const double* quat);

/* Device bytes needed for n_bodies_max bodies and the shapes already set. */
rbm_status rbm_workspace_size(rbm_ctx* ctx, int n_bodies_max, size_t* bytes);

/* Bind a caller-owned device buffer of at least rbm_workspace_size() bytes
 * (256-byte aligned).  Must precede rbm_setup(). */
rbm_status rbm_bind_workspace(rbm_ctx* ctx, void* dptr, size_t bytes);

/* Setup (Algorithm 1, first line; §3, §3.1): on the device, in float64, build per
 * shape the grid geometry, area, centroid, tau (§2.2), the singular self
 * operators, A0 = 1/2 I + K0 + L0, its inverse (the block preconditioner of §3.2)
 * and the velocity functional.  Call once per shape set. */
rbm_status rbm_setup(rbm_ctx* ctx);

/* Solve the mobility problem for loads FT[n][6] = (F_i, T_i) (lab frame) and
 * write VW[n][6] = (v_i, omega_i).  Host pointers.  info may be NULL. */
rbm_status rbm_solve(rbm_ctx* ctx, const double* FT, double* VW, rbm_solve_info* info);

/* Same with device pointers d_FT[n][6], d_VW[n][6] (no host copies of data; one
 * scalar is read back per GMRES iteration for the stopping test). */
rbm_status rbm_solve_dev(rbm_ctx* ctx, const double* d_FT, double* d_VW, rbm_solve_info* info);

/* Mobility matrix of §1 (V = M F, M symmetric positive definite by the reciprocal theorem
 * and the uniqueness argument of §2) at the current poses: Mmat[6n][6n] (host, row-major),
 * column k = the velocities (v_i, omega_i) for the unit load e_k (forces then torques per
 * body, lab frame), by 6n mobility solves with the context's precision and tolerance.  The
 * solves use the block-diagonal guess (also in the learned or user guess modes, which are
 * restored afterwards) and are not captured as training data.  info (may be NULL): summed
 * iterations, matvecs and times, largest relative residual.  RBM_E_NOCONV if a solve missed
 * tol (all columns are still written). */
rbm_status rbm_mobility_matrix(rbm_ctx* ctx, double* Mmat, rbm_solve_info* info);

/* Run state of Algorithm 1's time loop, to resume it later in this or another context with
 * the same options, shapes and learned configuration: body shape ids, centroids and
 * quaternions, the last solve's densities mu and rho (when there is one), the guess mode,
 * the running block-diagonal residual ratio of the learned fallback test and, when a
 * learned workspace is bound, the network parameters, Adam moments and step count, the
 * training epoch counter, the feature/target scalings and the captured samples.
 * rbm_get_state: buf == NULL writes the record size to *bytes; otherwise *bytes must be at
 * least that size and receives it.  Host memory, owned by the caller.  rbm_set_state
 * restores a record (RBM_E_INVAL for a record of other shapes, order, sizes or learned
 * configuration; RBM_E_STATE if the record holds a learned part and no learned workspace is
 * bound; RBM_E_NOMEM if it has more bodies than the workspace).  A run resumed from a record
 * repeats the uninterrupted run bit for bit. */
rbm_status rbm_get_state(rbm_ctx* ctx, void* buf, size_t* bytes);
rbm_status rbm_set_state(rbm_ctx* ctx, const void* buf, size_t bytes);

/* One classical RK4 step of the rigid-body evolution (§3.3; Algorithm 1, evolve
 * line): four mobility solves with the loads d_FT[n][6] (device pointer, held
 * fixed over the step), dc/dt = v, dq/dt = 1/2 (0, omega) (x) q with omega in the
 * lab frame; stage quaternions are normalised before they define a pose, and so is
 * the final one.  Poses are updated on the device (and mirrored to the host copy
 * read by rbm_get_bodies).  stage_info[4] may be NULL.  Returns RBM_E_NOCONV if a
 * stage solve missed its tolerance (the step is still taken), and RBM_E_OVERLAP if the
 * poses of a stage or of the step's end overlap (the step is not taken: the context keeps
 * the poses it started from). */
rbm_status rbm_step_rk4(rbm_ctx* ctx, double dt, const double* d_FT, rbm_solve_info* stage_info);

/* Current poses: centre[n][3], quat[n][4] (host arrays). */
rbm_status rbm_get_bodies(rbm_ctx* ctx, double* centre, double* quat);

/* Change the initial-guess mode (rbm_guess) of an existing context. */
rbm_status rbm_set_guess(rbm_ctx* ctx, int guess);

/* Initial density for RBM_GUESS_USER: d_mu0[3][N] device array, copied. */
rbm_status rbm_set_guess_dev(rbm_ctx* ctx, const double* d_mu0);

/* ---- Learned GMRES warm start (not in the paper; the block-diagonal guess of §3.2 is
 * its fallback) ---------------------------------------------------------------------
 * A per-body MLP maps body-frame features (own load, shape's radial coefficients,
 * k nearest neighbours' relative position d/|d|^2, relative orientation (two
 * columns of R_i^T R_j) and loads) to the body-frame band coefficients (§3
 * forward transform) of mu* - mu_BD, mu_BD = P^{-1} b.  Layers: F -> hidden x
 * n_hidden -> 3 (p^2 + 2p), SiLU, bf16 MFMA with fp32 accumulation and fp32 Adam
 * master weights.  Training data are captured from the context's own solves. */
typedef struct {
  int k_nbr;                 /* neighbours (1..16), default 8 */
  int hidden;                /* hidden width, default 256 */
  int n_hidden;              /* hidden layers (1..6), default 3 */
  int capacity;              /* captured body states the buffer holds, default 65536; once full,
                                new captures overwrite the oldest rows (a ring), so training
                                can be repeated along a run on its most recent states */
  int batch_max;             /* largest training batch, default 1024 */
  unsigned long long seed;   /* weight initialisation and epoch shuffles */
} rbm_learned_config;

void rbm_learned_default_config(rbm_learned_config* cfg);
/* Device bytes of the learned workspace (weights, Adam state, sample buffer, batch
 * activations).  Needs shapes and a bound solver workspace. */
rbm_status rbm_learned_workspace_size(rbm_ctx* ctx, const rbm_learned_config* cfg, size_t* bytes);
/* Bind it (caller-owned device memory) and initialise the weights. */
rbm_status rbm_learned_bind(rbm_ctx* ctx, const rbm_learned_config* cfg, void* dptr, size_t bytes);
/* Append (features, band coefficients of mu - mu_BD) of every body of the last solve,
 * whose loads were d_FT[n][6] (device).  Silently stops when the buffer is full. */
rbm_status rbm_learned_capture(rbm_ctx* ctx, const double* d_FT);
/* on != 0: capture after every solve (including the four RK4 stages). */
rbm_status rbm_learned_set_capture(rbm_ctx* ctx, int on);
/* `epochs` passes of Adam (learning rate lr) over the buffer in shuffled batches;
 * feature/target scalings are fixed from the buffer on the first call.  *loss gets
 * the last epoch's mean squared error in scaled units. */
rbm_status rbm_learned_train(rbm_ctx* ctx, int epochs, int batch, double lr, double* loss);
/* Sizes: captured samples, features F, outputs O, parameter count (weights then
 * biases per layer, row-major W[in][out]). */
rbm_status rbm_learned_info(rbm_ctx* ctx, int* samples, int* n_features, int* n_outputs,
                            int* n_params);
/* Parameters + scalings: [params (n_params), mean (F), inv_std (F), target scale, 1/scale]. */
rbm_status rbm_learned_get_params(rbm_ctx* ctx, float* host, size_t count);
rbm_status rbm_learned_set_params(rbm_ctx* ctx, const float* host, size_t count);
/* Network on given raw features d_X[rows][F] (device, fp32) -> d_Y[rows][O] (unscaled by
 * the target scale), rows <= max(batch_max, bodies). */
rbm_status rbm_learned_forward_dev(rbm_ctx* ctx, const float* d_X, int rows, float* d_Y);
/* Loss (MSE against d_T[rows][O] times 1/target scale) and the parameter gradient
 * d_grad[n_params] for one batch; no update. */
rbm_status rbm_learned_loss_grad_dev(rbm_ctx* ctx, const float* d_X, const float* d_T, int rows,
                                     float* d_grad, double* loss);
/* Features of the current bodies for loads d_FT: d_X[n][F] (device, fp32). */
rbm_status rbm_learned_features_dev(rbm_ctx* ctx, const double* d_FT, float* d_X);
/* The learned initial density mu_BD + network correction for loads d_FT (device), into
 * d_mu0[3][N] (device); float64 block-diagonal part.  Overwrites the last solve's state. */
rbm_status rbm_learned_guess_dev(rbm_ctx* ctx, const double* d_FT, double* d_mu0);

/* Copy out the last solve's densities ([3][N] host arrays; either may be NULL). */
rbm_status rbm_get_density(rbm_ctx* ctx, double* mu, double* rho);

/* y = A mu on the device ([3][N] lab frame, float64): the augmented operator of §2.3,
 * 1/2 I + K + L, with K the singular self blocks plus the off-body sum (upsampled for
 * near pairs when p_up > 0), at the current poses.  d_mu and d_y must not alias.
 * Synchronous on the context stream. */
rbm_status rbm_apply_dev(rbm_ctx* ctx, const double* d_mu, double* d_y);

/* Contact search (§3.3, contact force algorithm): body pairs a < b whose closest pair of
 * nodes is less than delta apart, at the current poses; the contact point is the
 * midpoint of that node pair (ties: smallest node indices).  Writes the first
 * min(found, max_contacts) pairs ([k][2], increasing a then b) and points ([k][3]) to
 * host arrays and the number found to *n_found.  Fails with RBM_E_INVAL when more than
 * 32 n candidate pairs have bounding spheres within delta. */
rbm_status rbm_find_contacts(rbm_ctx* ctx, double delta, int max_contacts, int* n_found,
                             int* pairs, double* points);

/* Mobility solve with contact forces (§3.3): for each contact k (bodies a, b touching at
 * x_k) a force F_k on a and -F_k on b, both at x_k, chosen so that the rigid motions agree
 * at x_k: (D M C) F_c = -D V_0 with V_0 the velocities for the loads FT, one mobility
 * solve per unit contact-force component (3 n_contacts solves), the small system solved
 * on the host by LU with partial pivoting; V = V_0 + M C F_c.  FT, VW: host [n][6];
 * pairs [n_contacts][2], points [n_contacts][3], Fc [n_contacts][3] (force on body a).
 * info: the V_0 solve's record with iterations, matvecs and times summed over all
 * solves.  RBM_E_INVAL for a singular contact system. */
rbm_status rbm_solve_contacts(rbm_ctx* ctx, const double* FT, int n_contacts, const int* pairs,
                              const double* points, double* VW, double* Fc, rbm_solve_info* info);

/* Magnetostatics of permeable bodies (§4, magnetorheological flows), float64, current poses:
 * bodies of permeability mu_ratio * mu0 in a fluid of permeability mu0 and the uniform field
 * H0 (host [3]).  Solves (1/2 I + eta K^L) q = eta H0 . n, eta = (mu_ratio - 1)/(mu_ratio + 1),
 * by unpreconditioned GMRES to ||residual|| <= tol ||rhs|| (iterations to *iters, may be NULL),
 * with phi = -H0 . x + S^L[q]; writes the Maxwell traction of the fluid side
 * mu0 [(H . n) H - |H|^2 n / 2], H = -grad phi (exterior limit), to d_rho ([3][N], device) and,
 * if d_FT is not NULL, the net force and torque (about the centroid) per body ([n][6],
 * device).  Needs options.magnetic = 1.  RBM_E_NOCONV if GMRES stops short of tol. */
rbm_status rbm_magnetic_traction_dev(rbm_ctx* ctx, const double* H0, double mu_ratio, double mu0,
                                     double tol, double* d_rho, double* d_FT, int* iters);

/* Mobility solve with a given incident density rho ([3][N], device; e.g. the Maxwell
 * traction above) in place of F/|Gamma| + tau^{-1} T x (x - x^c) (§2.2, §4); velocities
 * to d_VW ([n][6], device).  The learned guess is not used here (block-diagonal instead). */
rbm_status rbm_solve_density_dev(rbm_ctx* ctx, const double* d_rho, double* d_VW, rbm_solve_info* info);

/* One RK4 step of a magnetorheological suspension (§4): at each of the four stages the
 * magnetostatic problem of rbm_magnetic_traction_dev is solved at the stage poses (H0 host
 * [3], mu_ratio, mu0, GMRES tolerance tol_mag) and its Maxwell traction drives that stage's
 * mobility solve (rbm_solve_density_dev); stage updates as in rbm_step_rk4, including the
 * contact correction when options.contact_delta > 0.  Needs options.magnetic = 1.
 * stage_info[4] may be NULL.  RBM_E_NOCONV if a mobility solve missed its tolerance (the
 * step is still taken); an error of a magnetostatic solve ends the call with the poses of
 * the stage it was solving. */
rbm_status rbm_step_rk4_magnetic(rbm_ctx* ctx, double dt, const double* H0, double mu_ratio,
                                 double mu0, double tol_mag, rbm_solve_info* stage_info);

/* Device pointers of internal arrays for inspection (valid until the workspace is
 * rebound).  name: "X","N","W" ([3][N]/[N] lab nodes, normals, weights), "mu",
 * "rho", "b" ([3][N]), "r" ([3][N]: the float64 residual b - A mu of the last refinement), "A0","P0" ([n_shapes][3M][3M] column-major body-frame
 * operators), "V0" ([n_shapes][6][3M]), "gx","gn","gr" ([n_shapes][3][M] shape points,
 * normals, recentred points), "gw" ([n_shapes][M] weights), "coef" ([n_shapes][3][(p+1)^2]),
 * "shape" (per shape 32 values: area, xc[3], tau[9], tauinv[9]), "Rm" ([n][9]),
 * "Ftab" ([p^2+2p][M]), "Ytab" ([(p+1)^2][M]), "learned_X" / "learned_T" (captured
 * features [capacity][F] and targets [capacity][O], fp32), "learned_m" / "learned_v" (Adam's first
 * and second moments [n_params], fp32); with p_up > 0 also "U" (band-
 * limited interpolation, column-major [M][Mu], Mu = 2 p_up (p_up+1)), "fr" ([n_shapes][3][Mu]
 * fine nodes minus the centroid), "fw" ([n_shapes][Mu] fine weights), "rb" ([n_shapes]
 * bounding radii), "near_list" ([n][64] int, increasing j) and "near_count" ([n] int).
 * NULL if unknown. */
const void* rbm_debug_ptr(rbm_ctx* ctx, const char* name);

/* Copy `bytes` bytes starting `offset` bytes into the internal array `name` (as for
 * rbm_debug_ptr) to the host buffer dst (synchronous). */
rbm_status rbm_debug_read(rbm_ctx* ctx, const char* name, size_t offset, size_t bytes, void* dst);

/* Low-level kernels behind the solve, exposed for parity tests and benchmarks.  For the
 * three context calls below: X, Nrm, q, add, y, u are device pointers to float64 arrays
 * [3][n_points] (component-major); every point is both a target and a source, and the body
 * of point k is k / M, so the last body may hold fewer than M points; pairs on one body are
 * left out.  precision 0 = float64, 1 = float32 arithmetic (inputs and outputs stay float64).
 * Errors: RBM_E_INVAL for a null pointer (add aside), n_points < 1, M < 1 or a precision
 * other than 0 and 1; RBM_E_NOMEM before rbm_bind_workspace or for more than n_bodies_max * M
 * points of the bound workspace.  They use the workspace's scratch, so they must not
 * overlap a solve on the same context.
 *
 * rbm_far_traction: y = add (may be NULL) + sum over sources b not on the target's body of
 *   -(3/4pi) d (d.N_a)(d.q_b)/|d|^5, d = X_a - X_b (traction of the Stokeslet sum, §2.1,
 *   §3.1).  Issued on the context stream; returns without waiting. */
rbm_status rbm_far_traction(rbm_ctx* ctx, int n_points, int M, const double* X,
                            const double* Nrm, const double* q, const double* add,
                            double* y, int precision);

/* rbm_far_stokeslet: u = sum over sources b not on the target's body of
 *   (1/(8 pi eta)) [q_b/|d| + d (d.q_b)/|d|^3]  (Stokeslet of §2.1).  Issued on the context
 *   stream; returns without waiting. */
rbm_status rbm_far_stokeslet(rbm_ctx* ctx, int n_points, int M, const double* X,
                             const double* q, double* u, int precision);

/* rbm_far_traction_fmm: the sum of rbm_far_traction (add = NULL) approximated by the fast
 *   multipole method of order options.fmm_order (the O(N) far field, §3.1): Stokes through
 *   four harmonic potentials, complex solid-harmonic expansions on a uniform octree whose
 *   leaves are at least d_max wide (d_max >= the largest body diameter, so that every
 *   same-body pair falls in the direct near field), leaf level at most
 *   options.fmm_max_level (to *level, may be NULL).  Error: geometric in the order
 *   (about 5e-4 relative at order 10 for suspensions of spheres).  precision 0 = float64,
 *   1 = float32 arithmetic.  Needs options.fmm_order > 0; RBM_E_INVAL if a leaf would
 *   hold more than 4096 points.  Synchronous. */
rbm_status rbm_far_traction_fmm(rbm_ctx* ctx, int n_points, int M, const double* X, const double* Nrm,
                                const double* q, double d_max, double* y, int precision, int* level);

/* rbm_far_traction_static: the sum of rbm_far_traction (same arguments, same kernels and
 *   split rule, so the same result) for callers that cannot allocate device memory: code
 *   under HIP graph capture, tight serving loops, harnesses that forbid allocation.  It needs
 *   no context and calls no allocator: its scratch (packed sources, the split's partial
 *   sums, float32 copies of X and Nrm) is a 64 MiB array in device memory that every GPU
 *   the library runs on holds until the process ends.  At most about 762,000 points in
 *   float64 (precision 0) and 838,000 in float32 (precision 1); more return RBM_E_NOMEM.
 *   X, Nrm, q, add (may be NULL), y: device pointers, [3][n_points] float64; body of point k
 *   is k / M.  Work is issued on `stream` (hipStream_t, NULL = the default stream) on the
 *   current device and the call returns without waiting.  Every call on one GPU shares that
 *   GPU's scratch, which keeps the last call's contents: calls that overlap on one GPU (other
 *   streams, other host threads) race. */
rbm_status rbm_far_traction_static(int n_points, int M, const double* X, const double* Nrm,
                                   const double* q, const double* add, double* y, int precision,
                                   void* stream);

const char* rbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RBM_H */
