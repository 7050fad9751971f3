// Host side of the C ABI declared in include/rbm.h: context, workspace layout,
// setup, and the GMRES / GMRES-IR drivers that sequence the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <thread>
#include <cmath>
#include <type_traits>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rbm.h"
#include "kernels.h"
#include "far_plan.h"

using namespace rbm;

static thread_local std::string g_err;

static rbm_status fail(rbm_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

// The thread-local message of rbm_last_error(), for the entry points of other translation units.
namespace rbm {
rbm_status set_last_error(rbm_status s, const char* msg) { return fail(s, msg); }
}  // namespace rbm

#define HIPCHECK(expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(RBM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Near-singular correction: at most kNearMax near bodies per body.  The concatenated
// source lists are cut into work items of ch = max(128, ceil(total / kNearWork)) list
// positions, so that even a few near pairs give enough workgroups and there are at most
// kNearWork + n items (which bounds the slot scratch).
constexpr int kMaxPup = 48;
constexpr int kNearMax = 64;
constexpr int kNearWork = 8192;
// contact search: at most kContactCand candidate pairs per body (bounding spheres within delta)
constexpr int kContactCand = 32;

struct rbm_ctx {
  rbm_options opt;
  int p = 0, ps = 0, M = 0, M3 = 0, nc = 0, nB = 0, Ms = 0;
  hipStream_t st = nullptr;
  // shapes (host copy until setup)
  int ns = 0, shape_kind = -1, shape_lmax = 0, nsrc = 0;
  std::vector<double> shape_data;
  // bodies
  int n = 0, nmax = 0;
  std::vector<int> sid_h;
  std::vector<double> cen_h, quat_h;
  bool bodies_dirty = true;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool setup_done = false, have_solution = false, guess_set = false;
  int nblk = 256;
  // tables
  double *gl_t, *gl_w, *glr_t, *glr_w, *Ytab, *Yttab, *Ypstab, *Ftab, *Fttab, *nth, *nph, *nlam,
      *rnodes, *rW;
  // shapes
  double *coef, *rcbuf, *gx, *gn, *gw, *gr, *shp, *A0, *P0, *V0;
  float* P0f;
  uint16_t* P0h;
  int* piv;
  // bodies and nodes
  int* sid;
  double *cen, *quat, *FT, *VW, *Rm, *tauinv, *area_b, *mom, *vws;
  double *cen0, *quat0, *kst, *kacc;
  double *X, *Nn, *W;
  float *Xf, *Nf;
  // vectors
  double *rho, *b, *mu, *r, *t1, *t2, *yb, *guess;
  double* gB = nullptr;  // shared-shape GEMM operand (3N values)
  float* gZ = nullptr;   // shared-shape bf16 GEMM product (3N floats)
  // Krylov
  double *V, *H, *cs, *sn, *g, *y, *scal, *partial;
  // far field; part_u holds the Stokeslet partial sums of a fused residual evaluation,
  // valid for the current mu while vel_ready
  void* src;
  double* part;
  double* part_u = nullptr;
  bool vel_ready = false;
  // near-singular correction by upsampling (p_up > 0)
  int pu = 0, Mu = 0, near_pairs = 0;
  double kappa = 5.0;
  double *glu_t = nullptr, *glu_w = nullptr, *fr = nullptr, *fw = nullptr, *rb = nullptr,
         *U = nullptr, *nslots = nullptr;
  void* srcf = nullptr;
  int *nbr = nullptr, *ncnt = nullptr, *nitem = nullptr, *nfirst = nullptr, *nneed = nullptr;
  int n_items = 0, n_need = 0, item_len = 0;
  std::vector<int> ncnt_h, nbr_h, items_h, first_h, need_h;
  // magnetostatics (option magnetic): Laplace self operators, derivative matrices, tangents,
  // scalar work vectors
  double *SL0 = nullptr, *KL0 = nullptr, *Dth = nullptr, *Dph = nullptr, *tang = nullptr,
         *mq = nullptr, *mphi = nullptr, *mdn = nullptr, *mtmp = nullptr, *mb = nullptr,
         *mrho = nullptr;
  // fast multipole far field (option fmm_order): tree over the current points, sorted
  // geometry, counts per box and level, translation tables and expansions
  int *fleaf = nullptr, *fperm = nullptr, *fstart = nullptr, *ffill = nullptr, *fcnt = nullptr,
      *fmax = nullptr, *ftcnt = nullptr, *ftoff = nullptr;
  int2* ftask = nullptr;
  double* fsrt = nullptr;
  int fmm_ntask = 0;
  double4 *fXs = nullptr, *fNs = nullptr;
  double* fbounds = nullptr;
  void *ftabR = nullptr, *ftabI = nullptr, *fM = nullptr, *fL = nullptr;
  bool fmm_ready = false;
  int fmm_level = 0, fmm_npts = 0;
  double fmm_lo[3] = {0, 0, 0}, fmm_D = 1.0;
  size_t fmm_off[8] = {0};
  int* fmm_cnt[8] = {nullptr};
  int far_nslots = 0, far_base = 0;  // partial-sum slots of the last far sum, near slot index
  // contact search: coarse bounding radius per shape (device and host), candidate pairs
  double *rbc = nullptr, *cres = nullptr;
  int* ccand = nullptr;
  std::vector<double> rbc_h;
  // overlap test: largest nearest-neighbour node spacing per shape (device and host)
  double* hsp = nullptr;
  std::vector<double> hsp_h;
  double* pinned = nullptr;
  double* pinned_dev = nullptr;  // the same pinned buffer as a device pointer
  // learned warm start
  struct Learned {
    bool bound = false, stats_ready = false, capture_on = false;
    rbm_learned_config cfg;
    int F = 0, O = 0, S = 0, L = 0, rows_max = 0, count = 0, head = 0, t = 0, epoch = 0;
    std::vector<int> dims;
    std::vector<size_t> woff, boff;
    size_t nparam = 0;
    float *P, *G, *Mo, *Vo, *mean, *istd, *tsc, *Xbuf, *Tbuf, *Tb, *dA, *feats, *Yout;
    uint16_t *Wb, *Xb;
    int* idx;
    double *lpart, *lsum;
    std::vector<float*> Z, H, dZ;
    std::vector<uint16_t*> Hb, dZb;
  } L;
  double bd_ratio = -1.0;
  bool verbose = false;  // RBM_VERBOSE set: one stderr line per refinement and GMRES cycle
  // events for timing
  std::vector<hipEvent_t> ev;
  int ev_used = 0;
  bool timing = true;
};

extern "C" void rbm_default_options(rbm_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->p = 8;
  o->p_sing = 0;
  o->eta = 1.0;
  o->tol = 1e-12;
  o->max_iter = 100;
  o->max_restart = 4;
  o->precision = RBM_FP64;
  o->guess = RBM_GUESS_BLOCKDIAG;
  o->inner_tol = 1e-4;
  o->stream = nullptr;
  o->p_up = 0;
  o->near_factor = 5.0;
  o->contact_delta = 0.0;
  o->magnetic = 0;
  o->fmm_order = 0;
  o->fmm_max_level = 5;
  o->gmres_lookahead = 1;
  o->ir_stall = 0.5;
  o->velocity_fusion = 1;
}

extern "C" const char* rbm_last_error(void) { return g_err.c_str(); }

extern "C" rbm_status rbm_create(const rbm_options* opt, rbm_ctx** out) {
  if (!opt || !out) return fail(RBM_E_INVAL, "null argument");
  if (opt->p < 2 || opt->p > 20) return fail(RBM_E_INVAL, "p must be in [2, 20]");
  const int ps = opt->p_sing ? opt->p_sing : 2 * opt->p;
  if (ps < opt->p + 1 || ps > 64) return fail(RBM_E_INVAL, "p_sing must be in [p+1, 64]");
  if (!(opt->eta > 0.0) || !std::isfinite(opt->eta)) return fail(RBM_E_INVAL, "eta must be > 0");
  if (!(opt->tol > 0.0) || !std::isfinite(opt->tol)) return fail(RBM_E_INVAL, "tol must be > 0");
  if (opt->max_iter < 1 || opt->max_iter > 400) return fail(RBM_E_INVAL, "max_iter in [1, 400]");
  if (opt->max_restart < 0) return fail(RBM_E_INVAL, "max_restart >= 0");
  if (opt->precision < 0 || opt->precision > 2) return fail(RBM_E_INVAL, "bad precision");
  if (opt->guess < 0 || opt->guess > 3) return fail(RBM_E_INVAL, "bad guess");
  if (opt->p_up != 0 && (opt->p_up < opt->p + 1 || opt->p_up > kMaxPup))
    return fail(RBM_E_INVAL, "p_up must be 0 or in [p+1, 48]");
  if (!(opt->near_factor >= 0.0) || !std::isfinite(opt->near_factor))
    return fail(RBM_E_INVAL, "near_factor must be >= 0");
  if (!(opt->contact_delta >= 0.0) || !std::isfinite(opt->contact_delta))
    return fail(RBM_E_INVAL, "contact_delta must be >= 0");
  if (opt->fmm_order != 0 && (opt->fmm_order < 2 || opt->fmm_order > kFmmMaxOrder))
    return fail(RBM_E_INVAL, "fmm_order must be 0 or in [2, 16]");
  if (opt->fmm_order != 0 && opt->fmm_max_level != 0 && (opt->fmm_max_level < 2 || opt->fmm_max_level > 6))
    return fail(RBM_E_INVAL, "fmm_max_level must be 0 or in [2, 6]");
  if (opt->gmres_lookahead < 0 || opt->gmres_lookahead > 2) return fail(RBM_E_INVAL, "gmres_lookahead in [0, 2]");
  if (!(opt->ir_stall >= 0.0 && opt->ir_stall < 1.0)) return fail(RBM_E_INVAL, "ir_stall in [0, 1)");
  if (opt->velocity_fusion != 0 && opt->velocity_fusion != 1) return fail(RBM_E_INVAL, "velocity_fusion is 0 or 1");
  rbm_ctx* c = new rbm_ctx();
  c->opt = *opt;
  if (c->opt.fmm_max_level == 0) c->opt.fmm_max_level = 5;
  if (!(c->opt.inner_tol > 0.0)) c->opt.inner_tol = 1e-4;
  if (!(c->opt.ir_stall > 0.0)) c->opt.ir_stall = 0.5;
  c->p = opt->p;
  c->ps = ps;
  c->M = (c->p + 1) * 2 * c->p;
  c->M3 = 3 * c->M;
  c->nc = (c->p + 1) * (c->p + 1);
  c->nB = c->p * c->p + 2 * c->p;
  c->Ms = (ps + 1) * 2 * ps;
  c->st = (hipStream_t)opt->stream;
  c->pu = opt->p_up;
  c->Mu = c->pu ? (c->pu + 1) * 2 * c->pu : 0;
  c->kappa = opt->near_factor > 0.0 ? opt->near_factor : 5.0;
  c->verbose = std::getenv("RBM_VERBOSE") != nullptr;
  *out = c;
  return RBM_OK;
}

extern "C" void rbm_destroy(rbm_ctx* c) {
  if (!c) return;
  for (auto e : c->ev) (void)hipEventDestroy(e);
  if (c->pinned) (void)hipHostFree(c->pinned);
  delete c;
}

static bool all_finite(const double* x, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

extern "C" rbm_status rbm_set_shapes(rbm_ctx* c, int n_shapes, int lmax, const double* coef) {
  if (!c || !coef) return fail(RBM_E_INVAL, "null argument");
  if (n_shapes < 1) return fail(RBM_E_INVAL, "n_shapes must be >= 1");
  if (lmax < 1 || lmax > c->p - 1) return fail(RBM_E_INVAL, "coordinate lmax must be in [1, p-1]");
  const size_t k = (size_t)(lmax + 1) * (lmax + 1);
  if (!all_finite(coef, (size_t)n_shapes * 3 * k)) return fail(RBM_E_INVAL, "non-finite coefficient");
  c->shape_data.assign(coef, coef + (size_t)n_shapes * 3 * k);
  c->ns = n_shapes;
  c->shape_kind = 0;
  c->shape_lmax = lmax;
  c->setup_done = false;
  return RBM_OK;
}

extern "C" rbm_status rbm_set_shapes_radial(rbm_ctx* c, int n_shapes, int lmax, const double* rc) {
  if (!c || !rc) return fail(RBM_E_INVAL, "null argument");
  if (n_shapes < 1) return fail(RBM_E_INVAL, "n_shapes must be >= 1");
  if (lmax < 0 || lmax > c->p - 2) return fail(RBM_E_INVAL, "radial lmax must be in [0, p-2]");
  const size_t k = (size_t)(lmax + 1) * (lmax + 1);
  if (!all_finite(rc, (size_t)n_shapes * k)) return fail(RBM_E_INVAL, "non-finite coefficient");
  c->shape_data.assign(rc, rc + (size_t)n_shapes * k);
  c->ns = n_shapes;
  c->shape_kind = 1;
  c->shape_lmax = lmax;
  c->setup_done = false;
  return RBM_OK;
}

extern "C" rbm_status rbm_set_bodies(rbm_ctx* c, int n, const int* shape_id, const double* centre,
                                     const double* quat) {
  if (!c || !shape_id || !centre || !quat) return fail(RBM_E_INVAL, "null argument");
  if (n < 1) return fail(RBM_E_INVAL, "n must be >= 1");
  if (c->ns < 1) return fail(RBM_E_STATE, "set shapes first");
  if (c->ws && n > c->nmax) return fail(RBM_E_NOMEM, "more bodies than the workspace holds");
  if (!all_finite(centre, 3 * (size_t)n) || !all_finite(quat, 4 * (size_t)n))
    return fail(RBM_E_INVAL, "non-finite centre or quaternion");
  for (int i = 0; i < n; ++i) {
    if (shape_id[i] < 0 || shape_id[i] >= c->ns) return fail(RBM_E_INVAL, "unknown shape id");
    const double* q = quat + 4 * i;
    const double nq = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (std::fabs(nq - 1.0) > 1e-6) return fail(RBM_E_INVAL, "quaternion is not unit");
  }
  c->n = n;
  c->sid_h.assign(shape_id, shape_id + n);
  c->cen_h.assign(centre, centre + 3 * (size_t)n);
  c->quat_h.assign(quat, quat + 4 * (size_t)n);
  c->bodies_dirty = true;
  c->have_solution = false;
  return RBM_OK;
}

// Split of the source range for N points, bounded by the partial-sum buffer.
static int split_for(const rbm_ctx* c, int N) {
  const size_t cap = far_part_cap((size_t)c->nmax * c->M);
  int s = far_split(N);
  while (s > 1 && (size_t)s * N > cap) --s;
  return s;
}

// Bump allocation over the bound workspace; with assign == false only sizes.
static size_t layout(rbm_ctx* c, int nmax, bool assign) {
  size_t off = 0;
  auto take = [&](auto*& ptr, size_t count) {
    using T = std::remove_reference_t<decltype(*ptr)>;
    off = (off + 255) & ~(size_t)255;
    if (assign) ptr = reinterpret_cast<T*>(c->ws + off);
    off += count * sizeof(T);
  };
  const int p = c->p, ps = c->ps, M = c->M, M3 = c->M3, nc = c->nc, nB = c->nB, Ms = c->Ms;
  const size_t ns = c->ns;
  take(c->gl_t, p + 1); take(c->gl_w, p + 1); take(c->glr_t, ps + 1); take(c->glr_w, ps + 1);
  take(c->Ytab, (size_t)nc * M); take(c->Yttab, (size_t)nc * M); take(c->Ypstab, (size_t)nc * M);
  take(c->Ftab, (size_t)nB * M); take(c->Fttab, (size_t)nB * M);
  take(c->nth, M); take(c->nph, M); take(c->nlam, M);
  take(c->rnodes, 3 * (size_t)Ms); take(c->rW, Ms);
  take(c->coef, ns * 3 * nc);
  take(c->rcbuf, c->shape_data.size() + 1);
  take(c->gx, ns * 3 * M); take(c->gn, ns * 3 * M); take(c->gr, ns * 3 * M); take(c->gw, ns * M);
  take(c->shp, ns * 32);
  take(c->rbc, ns);
  take(c->hsp, ns);
  take(c->A0, ns * M3 * M3); take(c->P0, ns * M3 * M3); take(c->V0, ns * 6 * M3);
  take(c->piv, ns * M3);
  if (c->opt.precision == RBM_MIXED_FP32) take(c->P0f, ns * M3 * M3); else if (assign) c->P0f = nullptr;
  if (c->opt.precision == RBM_MIXED_BF16) take(c->P0h, ns * M3 * M3); else if (assign) c->P0h = nullptr;
  const size_t nm = nmax, N = nm * M, N3 = 3 * N;
  take(c->sid, nm); take(c->cen, 3 * nm); take(c->quat, 4 * nm); take(c->FT, 6 * nm);
  take(c->VW, 6 * nm); take(c->Rm, 9 * nm); take(c->tauinv, 9 * nm); take(c->area_b, nm);
  take(c->mom, 6 * nm); take(c->vws, 6 * nm);
  take(c->cen0, 3 * nm); take(c->quat0, 4 * nm); take(c->kst, 7 * nm); take(c->kacc, 7 * nm);
  take(c->X, N3); take(c->Nn, N3); take(c->W, N); take(c->Xf, N3); take(c->Nf, N3);
  take(c->rho, N3); take(c->b, N3); take(c->mu, N3); take(c->r, N3); take(c->t1, N3);
  take(c->t2, N3); take(c->yb, N3); take(c->guess, N3);
  if (c->ns == 1) {
    take(c->gB, N3);
    take(c->gZ, N3);
  } else if (assign) {
    c->gB = nullptr;
    c->gZ = nullptr;
  }
  const int m = c->opt.max_iter;
  take(c->V, (size_t)(m + 1) * N3); take(c->H, (size_t)(m + 1) * (m + 1)); take(c->cs, m + 1);
  take(c->sn, m + 1); take(c->g, m + 2); take(c->y, m + 2);
  take(c->scal, 64);
  take(c->partial, 3 * (size_t)(m + 2) * c->nblk);  // three regions for the fused Arnoldi step
  double* srcd = nullptr;
  take(srcd, 8 * N);
  if (assign) c->src = srcd;
  take(c->part, 3 * (far_part_cap(N) + (c->pu ? N : 0)));
  take(c->part_u, 3 * (far_part_cap(N) + (c->pu ? N : 0)));
  take(c->ccand, 2 * (size_t)kContactCand * nm); take(c->cres, 5 * (size_t)kContactCand * nm);
  if (c->opt.magnetic) {
    take(c->SL0, ns * M * M); take(c->KL0, ns * M * M);
    take(c->Dth, (size_t)M * M); take(c->Dph, (size_t)M * M); take(c->tang, ns * 6 * M);
    take(c->mq, N); take(c->mphi, N); take(c->mdn, N); take(c->mtmp, N); take(c->mb, N);
    take(c->mrho, N3);
  }
  if (c->opt.fmm_order > 0) {
    const int Lm = c->opt.fmm_max_level, P = c->opt.fmm_order;
    const size_t nleaf = (size_t)1 << (3 * Lm);
    size_t btot = 0;
    for (int l = 2; l <= Lm; ++l) btot += (size_t)1 << (3 * l);
    // expansions keep m >= 0 ((P+1)(P+2)/2 coefficients); the M2L tables hold all m, (2P+1)^2
    const size_t kc = (size_t)(P + 1) * (P + 2) / 2, kc2 = (size_t)(2 * P + 1) * (2 * P + 1);
    take(c->fleaf, N); take(c->fperm, N); take(c->fstart, nleaf + 1); take(c->ffill, nleaf);
    take(c->fcnt, std::max(btot, nleaf)); take(c->fmax, 64);
    take(c->fXs, N); take(c->fNs, N); take(c->fbounds, 64);
    take(c->ftcnt, nleaf); take(c->ftoff, nleaf + 1); take(c->ftask, N / 64 + nleaf + 1);
    take(c->fsrt, 8 * (size_t)N);
    double *tr = nullptr, *ti = nullptr, *me = nullptr, *le = nullptr;
    take(tr, 2 * (size_t)(Lm - 1) * 8 * kc); take(ti, 2 * (size_t)(Lm - 1) * 343 * kc2);
    take(me, 2 * btot * 4 * kc); take(le, 2 * btot * 4 * kc);
    if (assign) {
      c->ftabR = tr;
      c->ftabI = ti;
      c->fM = me;
      c->fL = le;
    }
  }
  if (c->pu) {
    const size_t Mu = c->Mu;
    take(c->glu_t, c->pu + 1); take(c->glu_w, c->pu + 1);
    take(c->fr, ns * 3 * Mu); take(c->fw, ns * Mu); take(c->rb, ns);
    take(c->U, Mu * M);
    take(c->nslots, (size_t)(kNearWork + nm) * 3 * M);
    double* sf = nullptr;
    take(sf, 8 * nm * Mu);
    if (assign) c->srcf = sf;
    take(c->nbr, nm * kNearMax); take(c->ncnt, nm);
    take(c->nitem, 2 * (kNearWork + nm)); take(c->nfirst, nm + 1); take(c->nneed, nm);
  }
  return off + 256;
}

extern "C" rbm_status rbm_workspace_size(rbm_ctx* c, int n_bodies_max, size_t* bytes) {
  if (!c || !bytes) return fail(RBM_E_INVAL, "null argument");
  if (c->ns < 1) return fail(RBM_E_STATE, "set shapes first");
  if (n_bodies_max < 1) return fail(RBM_E_INVAL, "n_bodies_max >= 1");
  if ((double)n_bodies_max * c->M > 2.0e9) return fail(RBM_E_INVAL, "too many points");
  *bytes = layout(c, n_bodies_max, false);
  return RBM_OK;
}

extern "C" rbm_status rbm_bind_workspace(rbm_ctx* c, void* dptr, size_t bytes) {
  if (!c || !dptr) return fail(RBM_E_INVAL, "null argument");
  if (c->ns < 1) return fail(RBM_E_STATE, "set shapes first");
  if (((uintptr_t)dptr & 255) != 0) return fail(RBM_E_INVAL, "workspace must be 256-byte aligned");
  // largest body count that fits
  int lo = 0, hi = 1;
  while (hi < (1 << 26) && layout(c, hi, false) <= bytes) { lo = hi; hi *= 2; }
  while (hi - lo > 1) {
    const int mid = lo + (hi - lo) / 2;
    if (layout(c, mid, false) <= bytes) lo = mid; else hi = mid;
  }
  if (lo < 1) return fail(RBM_E_NOMEM, "workspace too small for one body");
  if (c->n > lo) return fail(RBM_E_NOMEM, "workspace too small for the bodies already set");
  c->ws = reinterpret_cast<char*>(dptr);
  c->ws_bytes = bytes;
  c->nmax = lo;
  layout(c, lo, true);
  if (!c->pinned) {
    HIPCHECK(hipHostMalloc((void**)&c->pinned, 64 * sizeof(double), 0));
    HIPCHECK(hipHostGetDevicePointer((void**)&c->pinned_dev, c->pinned, 0));
  }
  c->setup_done = false;
  c->bodies_dirty = true;
  return RBM_OK;
}

extern "C" rbm_status rbm_setup(rbm_ctx* c) {
  if (!c) return fail(RBM_E_INVAL, "null argument");
  if (!c->ws) return fail(RBM_E_NOMEM, "bind a workspace first");
  if (c->ns < 1) return fail(RBM_E_STATE, "set shapes first");
  hipStream_t st = c->st;
  const int p = c->p, M = c->M, M3 = c->M3;
  HIPCHECK(launch_gauss_legendre(p + 1, c->gl_t, c->gl_w, st));
  HIPCHECK(launch_gauss_legendre(c->ps + 1, c->glr_t, c->glr_w, st));
  HIPCHECK(launch_grid_tables(p, c->gl_t, c->gl_w, c->Ytab, c->Yttab, c->Ypstab, c->Ftab, c->Fttab,
                              c->nth, c->nph, c->nlam, st));
  HIPCHECK(launch_rotated_rule(c->ps, c->glr_t, c->glr_w, c->rnodes, c->rW, st));
  if (c->shape_kind == 1) {
    const int nrc = (c->shape_lmax + 1) * (c->shape_lmax + 1);
    HIPCHECK(hipMemcpyAsync(c->rcbuf, c->shape_data.data(), c->shape_data.size() * sizeof(double),
                            hipMemcpyHostToDevice, st));
    HIPCHECK(launch_radial_to_coef(c->ns, p, nrc, c->rcbuf, c->Ytab, c->Ftab, c->nth, c->nph,
                                   c->coef, st));
  } else {
    std::vector<double> full((size_t)c->ns * 3 * c->nc, 0.0);
    const int k = (c->shape_lmax + 1) * (c->shape_lmax + 1);
    for (int s = 0; s < c->ns; ++s)
      for (int d = 0; d < 3; ++d)
        for (int i = 0; i < k; ++i)
          full[((size_t)s * 3 + d) * c->nc + i] = c->shape_data[((size_t)s * 3 + d) * k + i];
    HIPCHECK(hipMemcpyAsync(c->coef, full.data(), full.size() * sizeof(double),
                            hipMemcpyHostToDevice, st));
    HIPCHECK(hipStreamSynchronize(st));
  }
  HIPCHECK(launch_shape_geometry(c->ns, p, c->coef, c->Ytab, c->Yttab, c->Ypstab, c->nlam, c->gx,
                                 c->gn, c->gw, c->gr, c->shp, st));
  // S0 into the P0 buffer (temporary), K0 into A0
  HIPCHECK(launch_singular_assemble(c->ns, p, c->ps, c->opt.eta, c->coef, c->gx, c->gn, c->nth,
                                    c->nph, c->rnodes, c->rW, c->Fttab, c->P0, c->A0, st));
  HIPCHECK(launch_finish_A0(c->ns, M, c->gr, c->gw, c->A0, st));
  HIPCHECK(launch_velocity_functional(c->ns, M, c->P0, c->gr, c->gw, c->shp, c->V0, st));
  HIPCHECK(hipMemcpyAsync(c->P0, c->A0, (size_t)c->ns * M3 * M3 * sizeof(double),
                          hipMemcpyDeviceToDevice, st));
  HIPCHECK(launch_gauss_jordan(c->ns, M3, c->P0, c->piv, st));
  if (c->P0f) HIPCHECK(launch_cast_f32((size_t)c->ns * M3 * M3, c->P0, c->P0f, st));
  if (c->P0h) HIPCHECK(launch_cast_bf16((size_t)c->ns * M3 * M3, c->P0, c->P0h, st));
  if (c->opt.magnetic) {
    HIPCHECK(launch_singular_laplace(c->ns, p, c->ps, c->coef, c->gx, c->gn, c->nth, c->nph, c->rnodes,
                                     c->rW, c->Fttab, c->SL0, c->KL0, st));
    HIPCHECK(launch_magnetic_tables(p, c->ns, c->coef, c->Yttab, c->Ypstab, c->Ftab, c->Dth, c->Dph,
                                    c->tang, st));
  }
  HIPCHECK(launch_bound_radius(c->ns, M, c->gr, c->rbc, st));
  HIPCHECK(launch_node_spacing(c->ns, M, c->gr, c->hsp, st));
  c->rbc_h.resize(c->ns);
  c->hsp_h.resize(c->ns);
  HIPCHECK(hipMemcpyAsync(c->rbc_h.data(), c->rbc, c->ns * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipMemcpyAsync(c->hsp_h.data(), c->hsp, c->ns * sizeof(double), hipMemcpyDeviceToHost, st));
  if (c->pu) {
    HIPCHECK(launch_gauss_legendre(c->pu + 1, c->glu_t, c->glu_w, st));
    HIPCHECK(launch_fine_geometry(c->ns, p, c->pu, c->coef, c->glu_t, c->glu_w, c->shp, c->fr, c->fw,
                                  c->rb, st));
    HIPCHECK(launch_interp_matrix(p, c->pu, c->gl_t, c->gl_w, c->glu_t, c->U, st));
  }
  HIPCHECK(hipStreamSynchronize(st));
  c->setup_done = true;
  c->bodies_dirty = true;
  return RBM_OK;
}

// ---------------------------------------------------------------------------------
// Solve

// Near list of the current poses (upsampling on); reads the counts back to check them
// against kNearMax and to report the number of near pairs.
static rbm_status build_near(rbm_ctx* c) {
  if (!c->pu) return RBM_OK;
  HIPCHECK(launch_near_list(c->n, c->M, kNearMax, c->kappa, c->cen, c->sid, c->rb, c->shp, c->nbr,
                            c->ncnt, c->st));
  const int n = c->n;
  c->ncnt_h.resize(n);
  c->nbr_h.resize((size_t)n * kNearMax);
  HIPCHECK(hipMemcpyAsync(c->ncnt_h.data(), c->ncnt, n * sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHECK(hipMemcpyAsync(c->nbr_h.data(), c->nbr, (size_t)n * kNearMax * sizeof(int),
                          hipMemcpyDeviceToHost, c->st));
  HIPCHECK(hipStreamSynchronize(c->st));
  int tot = 0, mx = 0;
  for (int v : c->ncnt_h) { tot += v; mx = std::max(mx, v); }
  if (mx > kNearMax)
    return fail(RBM_E_INVAL, "a body has more than 64 near bodies: lower near_factor");
  c->near_pairs = tot;
  // work items (body, first list position), per-body item ranges, bodies whose fine
  // sources are read
  const long seg = (long)c->Mu + c->M, total = (long)tot * seg;
  c->item_len = (int)std::max<long>(128, (total + kNearWork - 1) / kNearWork);
  std::vector<int> body, pos;
  c->first_h.assign(n + 1, 0);
  std::vector<char> needed(n, 0);
  for (int i = 0; i < n; ++i) {
    c->first_h[i] = (int)body.size();
    const long L = c->ncnt_h[i] * seg;
    for (long p0 = 0; p0 < L; p0 += c->item_len) {
      body.push_back(i);
      pos.push_back((int)p0);
    }
    for (int k = 0; k < c->ncnt_h[i]; ++k) needed[c->nbr_h[(size_t)i * kNearMax + k]] = 1;
  }
  c->first_h[n] = (int)body.size();
  c->n_items = (int)body.size();
  c->items_h = body;
  c->items_h.insert(c->items_h.end(), pos.begin(), pos.end());
  c->need_h.clear();
  for (int j = 0; j < n; ++j)
    if (needed[j]) c->need_h.push_back(j);
  c->n_need = (int)c->need_h.size();
  if (c->n_items > kNearWork + c->nmax) return fail(RBM_E_INVAL, "near-correction work list overflow");
  if (c->n_items)
    HIPCHECK(hipMemcpyAsync(c->nitem, c->items_h.data(), c->items_h.size() * sizeof(int),
                            hipMemcpyHostToDevice, c->st));
  HIPCHECK(hipMemcpyAsync(c->nfirst, c->first_h.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice,
                          c->st));
  if (c->n_need)
    HIPCHECK(hipMemcpyAsync(c->nneed, c->need_h.data(), c->n_need * sizeof(int), hipMemcpyHostToDevice,
                            c->st));
  HIPCHECK(hipStreamSynchronize(c->st));
  return RBM_OK;
}

// Overlap test at the current poses (centres read from the device): bodies whose bounding
// spheres (largest centroid-to-node distance) intersect are compared node by node, and
// RBM_E_OVERLAP is returned when a node of one body lies inside the other by more than the
// allowance h^2, h the largest nearest-neighbour node spacing of the other body's shape.  A
// node outside a smooth body is never below -(covering radius)^2 x curvature / 2 >= -h^2
// (curvature up to 4 for unit-size bodies), so separated bodies pass however close they are.
static rbm_status check_overlap(rbm_ctx* c) {
  const int n = c->n, M = c->M;
  if (n < 2) return RBM_OK;
  hipStream_t st = c->st;
  std::vector<double> cen(3 * (size_t)n);
  HIPCHECK(hipMemcpyAsync(cen.data(), c->cen, cen.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  double rmax = 0.0;
  for (int i = 0; i < n; ++i) rmax = std::max(rmax, c->rbc_h[c->sid_h[i]]);
  // sweep over bodies sorted by x: a pair can intersect only within 2 rmax in x
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) {
    return cen[3 * a] < cen[3 * b] || (cen[3 * a] == cen[3 * b] && a < b);
  });
  std::vector<int> cand;
  for (int ia = 0; ia < n; ++ia) {
    const int a = ord[ia];
    for (int ib = ia + 1; ib < n; ++ib) {
      const int b = ord[ib];
      const double dx = cen[3 * b] - cen[3 * a];
      if (dx >= 2.0 * rmax) break;
      const double dy = cen[3 * b + 1] - cen[3 * a + 1], dz = cen[3 * b + 2] - cen[3 * a + 2];
      const double rr = c->rbc_h[c->sid_h[a]] + c->rbc_h[c->sid_h[b]];
      if (dx * dx + dy * dy + dz * dz < rr * rr) {
        cand.push_back(std::min(a, b));
        cand.push_back(std::max(a, b));
      }
    }
  }
  const int ncand = (int)cand.size() / 2;
  if (ncand == 0) return RBM_OK;
  if ((size_t)ncand > (size_t)kContactCand * c->nmax)
    return fail(RBM_E_OVERLAP, "more than 32 n body pairs with intersecting bounding spheres");
  std::vector<double> res(2 * (size_t)ncand);
  HIPCHECK(hipMemcpyAsync(c->ccand, cand.data(), cand.size() * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHECK(launch_overlap_depth(ncand, n * M, M, c->ccand, c->X, c->Nn, c->cres, st));
  HIPCHECK(hipMemcpyAsync(res.data(), c->cres, res.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  for (int k = 0; k < ncand; ++k) {
    const int a = cand[2 * k], b = cand[2 * k + 1];
    const double ha = c->hsp_h[c->sid_h[a]], hb = c->hsp_h[c->sid_h[b]];
    if (!(res[2 * k] >= -ha * ha) || !(res[2 * k + 1] >= -hb * hb))
      return fail(RBM_E_OVERLAP, "bodies " + std::to_string(a) + " and " + std::to_string(b) + " overlap");
  }
  return RBM_OK;
}

static rbm_status upload_bodies(rbm_ctx* c) {
  if (!c->bodies_dirty) return RBM_OK;
  hipStream_t st = c->st;
  const int n = c->n;
  HIPCHECK(hipMemcpyAsync(c->sid, c->sid_h.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHECK(hipMemcpyAsync(c->cen, c->cen_h.data(), 3 * n * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHECK(hipMemcpyAsync(c->quat, c->quat_h.data(), 4 * n * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHECK(launch_body_prep(n, c->quat, c->sid, c->shp, c->Rm, c->tauinv, c->area_b, st));
  HIPCHECK(launch_nodes(n, c->M, c->sid, c->cen, c->Rm, c->gr, c->gn, c->gw, c->X, c->Nn, c->W,
                        c->Xf, c->Nf, st));
  HIPCHECK(hipStreamSynchronize(st));
  rbm_status s = check_overlap(c);
  if (s != RBM_OK) return s;
  s = build_near(c);
  if (s != RBM_OK) return s;
  c->bodies_dirty = false;
  return RBM_OK;
}

struct Timer {
  rbm_ctx* c;
  hipEvent_t a, b;
  bool on;
  Timer(rbm_ctx* cc) : c(cc), on(cc->timing) {
    if (!on) return;
    while ((int)c->ev.size() < c->ev_used + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
      c->ev.push_back(e);
    }
    a = c->ev[c->ev_used];
    b = c->ev[c->ev_used + 1];
    c->ev_used += 2;
    (void)hipEventRecord(a, c->st);
  }
  void stop() { if (on) (void)hipEventRecord(b, c->st); }
};

struct SolveState {
  // event index pairs: float64 traction sums, float32 (direct or fast multipole) traction
  // sums, Stokeslet sums, self applies, near corrections
  std::vector<std::pair<int, int>> trac_ev, trac32_ev, stok_ev, self_ev, near_ev, fused_ev;
  bool fused_used = false;
  double far_pairs = 0.0;
  int matvecs = 0;
  int fmm_applies = 0;
};

// Partial-sum slots the combine adds for N points: the far sum's split plus, with
// upsampling, the near-correction slot that follows it.
static int far_slots(const rbm_ctx* c, int N) { return split_for(c, N) + (c->pu ? 1 : 0); }

// Near-singular correction of the far sum of kind (0 traction, 1 Stokeslet) for the
// density x whose plain sources are already packed in c->src: fine sources of the needed
// bodies, fine-minus-plain sums per work item, reduced per body into the slot after the
// far split.
static rbm_status near_correction(rbm_ctx* c, SolveState& S, int kind, const double* x,
                                  int x_is_body, int prec, double* part = nullptr) {
  if (!c->pu) return RBM_OK;
  const int n = c->n, M = c->M, N = n * M;
  double* res = (part ? part : c->part) + (size_t)c->far_base * 3 * N;
  const int* ib = c->nitem;
  const int* ip = c->nitem + c->n_items;
  Timer t(c);
  if (prec == 0) {
    HIPCHECK(launch_near_corr<double>(kind, n, M, c->Mu, kNearMax, c->n_need, c->nneed, c->n_items,
                                      c->item_len, ib, ip, c->nfirst, c->X, c->Nn, c->src, x, x_is_body,
                                      c->U, c->sid, c->cen, c->Rm, c->fr, c->fw, c->nbr, c->ncnt, c->srcf,
                                      c->nslots, res, c->st));
  } else {
    HIPCHECK(launch_near_corr<float>(kind, n, M, c->Mu, kNearMax, c->n_need, c->nneed, c->n_items,
                                     c->item_len, ib, ip, c->nfirst, c->Xf, c->Nf, c->src, x, x_is_body,
                                     c->U, c->sid, c->cen, c->Rm, c->fr, c->fw, c->nbr, c->ncnt, c->srcf,
                                     c->nslots, res, c->st));
  }
  t.stop();
  if (t.on) S.near_ev.push_back({c->ev_used - 2, c->ev_used - 1});
  return RBM_OK;
}

// Octree of the fast multipole far field over the points X, N ([3][npts], float64) with
// bodies of M consecutive points and largest body diameter d_max: leaf level = finest level
// whose width is >= d_max (at most fmm_max_level), points sorted by leaf.  Leaves the
// context without a tree (fmm_ready false) when some leaf would hold more than kFmmLeafCap
// points; the far sums are then direct.
static rbm_status fmm_build(rbm_ctx* c, int npts, int M, const double* X, const double* Nn, double d_max) {
  c->fmm_ready = false;
  hipStream_t st = c->st;
  HIPCHECK(launch_fmm_bounds(npts, X, c->fbounds, st));
  HIPCHECK(hipMemcpyAsync(c->pinned, c->fbounds, 6 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  double e = 0.0;
  for (int d = 0; d < 3; ++d) {
    c->fmm_lo[d] = c->pinned[d];
    e = std::max(e, c->pinned[3 + d] - c->pinned[d]);
  }
  c->fmm_D = e > 0.0 ? e * (1.0 + std::ldexp(1.0, -20)) : 1.0;
  int L = 0;
  while (L < c->opt.fmm_max_level && std::ldexp(c->fmm_D, -(L + 1)) >= d_max) ++L;
  c->fmm_level = L;
  const int nb = 1 << L;
  // per-level counts: levels 2..L consecutive (or the single leaf level when L < 2)
  size_t off = 0;
  for (int l = 0; l < 8; ++l) c->fmm_cnt[l] = nullptr;
  if (L >= 2) {
    for (int l = 2; l <= L; ++l) {
      c->fmm_off[l] = off;
      c->fmm_cnt[l] = c->fcnt + off;
      off += (size_t)1 << (3 * l);
    }
  } else {
    c->fmm_off[L] = 0;
    c->fmm_cnt[L] = c->fcnt;
  }
  HIPCHECK(launch_fmm_sort_points(npts, M, X, Nn, c->fmm_lo, std::ldexp(c->fmm_D, -L), nb, c->fleaf,
                                  c->fmm_cnt[L], c->fstart, c->ffill, c->fperm, c->fmax, c->fXs, c->fNs, st));
  int maxcnt = 0;
  HIPCHECK(hipMemcpyAsync(c->pinned, c->fmax, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  std::memcpy(&maxcnt, c->pinned, sizeof(int));
  if (maxcnt > kFmmLeafCap) return RBM_OK;
  HIPCHECK(launch_fmm_finish_tree(npts, M, L, X, Nn, c->fstart, c->fperm, c->fXs, c->fNs, c->fmm_cnt, c->ftcnt,
                                   c->ftoff, c->ftask, c->fmax + 1, st));
  HIPCHECK(hipMemcpyAsync(c->pinned, c->ftoff + ((size_t)1 << (3 * L)), sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  std::memcpy(&c->fmm_ntask, c->pinned, sizeof(int));
  c->fmm_npts = npts;
  c->fmm_ready = true;
  return RBM_OK;
}

// Largest body diameter bound of the current shapes: twice the largest centroid-to-node
// distance.
static double fmm_dmax(const rbm_ctx* c) {
  double r = 0.0;
  for (double v : c->rbc_h) r = std::max(r, v);
  return 2.0 * r;
}

// FMM traction sums of the packed sources c->src (precision prec) into out[3][npts].
static rbm_status fmm_apply(rbm_ctx* c, int prec, double* out) {
  const int P = c->opt.fmm_order, L = c->fmm_level;
  if (prec == 0) {
    if (L >= 2) HIPCHECK(launch_fmm_tables<double>(P, L, c->fmm_D, c->ftabR, c->ftabI, c->st));
    HIPCHECK(launch_fmm_apply<double>(P, L, c->fmm_lo, c->fmm_D, c->fmm_npts, c->fstart, c->fperm, c->fXs,
                                      c->fNs, c->fmm_cnt, c->fmm_off, c->fmm_ntask, c->ftask, c->ftabR, c->ftabI,
                                      c->src, c->fsrt, c->fM, c->fL, out, c->st));
  } else {
    if (L >= 2) HIPCHECK(launch_fmm_tables<float>(P, L, c->fmm_D, c->ftabR, c->ftabI, c->st));
    HIPCHECK(launch_fmm_apply<float>(P, L, c->fmm_lo, c->fmm_D, c->fmm_npts, c->fstart, c->fperm, c->fXs,
                                     c->fNs, c->fmm_cnt, c->fmm_off, c->fmm_ntask, c->ftask, c->ftabR, c->ftabI,
                                     c->src, c->fsrt, c->fM, c->fL, out, c->st));
  }
  return RBM_OK;
}

// Far traction of x (lab [3][N] or body frame), precision prec: part sums in c->part
// (c->far_nslots of them, the near correction included).  prec 0: direct float64; prec 1:
// float32, by the FMM when the context has a tree for the current poses (inner iterations
// of the precision form), else direct.
static rbm_status far_traction(rbm_ctx* c, SolveState& S, const double* x, int x_is_body,
                               int prec) {
  const int N = c->n * c->M;
  const int nsp = split_for(c, N);
  if (prec != 0 && c->fmm_ready && c->fmm_npts == N) {
    HIPCHECK(launch_pack_sources<float>(N, c->M, c->X, c->W, c->Rm, x, x_is_body, nullptr, c->src, c->st));
    Timer t(c);
    rbm_status s = fmm_apply(c, 1, c->part);
    if (s != RBM_OK) return s;
    t.stop();
    if (t.on) S.trac32_ev.push_back({c->ev_used - 2, c->ev_used - 1});
    c->far_base = 1;
    c->far_nslots = 1 + (c->pu ? 1 : 0);
    S.fmm_applies++;
    return near_correction(c, S, 0, x, x_is_body, 1);
  }
  c->far_base = nsp;
  c->far_nslots = nsp + (c->pu ? 1 : 0);
  if (prec == 0) {
    HIPCHECK(launch_pack_sources<double>(N, c->M, c->X, c->W, c->Rm, x, x_is_body, nullptr, c->src, c->st));
    Timer t(c);
    HIPCHECK(launch_far<double>(0, N, c->M, c->X, c->Nn, c->src, c->part, nsp, c->st));
    t.stop();
    if (t.on) S.trac_ev.push_back({c->ev_used - 2, c->ev_used - 1});
  } else {
    HIPCHECK(launch_pack_sources<float>(N, c->M, c->X, c->W, c->Rm, x, x_is_body, nullptr, c->src, c->st));
    Timer t(c);
    HIPCHECK(launch_far<float>(0, N, c->M, c->Xf, c->Nf, c->src, c->part, nsp, c->st));
    t.stop();
    if (t.on) S.trac32_ev.push_back({c->ev_used - 2, c->ev_used - 1});
  }
  S.far_pairs += (double)N * N - (double)c->n * c->M * c->M;
  return near_correction(c, S, 0, x, x_is_body, prec == 0 ? 0 : 1);
}

// y_body = A (R^T x) with A = A0 (which 0), P0 (which 1) in the given precision.  With one
// shape shared by all bodies (and enough of them) this is a GEMM on MFMA.
static rbm_status self_apply(rbm_ctx* c, SolveState& S, int which, int prec, const double* x,
                             double* ybody) {
  Timer t(c);
  if (c->ns == 1 && c->n >= 8 && c->gB) {
    if (which == 0 || prec == 0) {
      HIPCHECK(launch_self_apply_shared<double>(c->n, c->M, which == 0 ? c->A0 : c->P0, c->Rm, x,
                                                c->gB, c->gZ, ybody, c->st));
    } else if (prec == 1) {
      HIPCHECK(launch_self_apply_shared<float>(c->n, c->M, c->P0f, c->Rm, x, c->gB, c->gZ, ybody, c->st));
    } else {
      HIPCHECK(launch_self_apply_shared<uint16_t>(c->n, c->M, c->P0h, c->Rm, x, c->gB, c->gZ, ybody, c->st));
    }
  } else if (which == 0 || prec == 0) {
    HIPCHECK(launch_self_apply<double>(c->n, c->M, c->sid, which == 0 ? c->A0 : c->P0, c->Rm, x,
                                       ybody, c->st));
  } else if (prec == 1) {
    HIPCHECK(launch_self_apply<float>(c->n, c->M, c->sid, c->P0f, c->Rm, x, ybody, c->st));
  } else {
    HIPCHECK(launch_self_apply<uint16_t>(c->n, c->M, c->sid, c->P0h, c->Rm, x, ybody, c->st));
  }
  t.stop();
  if (t.on) S.self_ev.push_back({c->ev_used - 2, c->ev_used - 1});
  return RBM_OK;
}

// out = A x = A_self x + K_far(w x)   (float64; A_self includes 1/2 I and L)
static rbm_status apply_A(rbm_ctx* c, SolveState& S, const double* x, double* out) {
  const int N = c->n * c->M;
  rbm_status s;
  if ((s = self_apply(c, S, 0, 0, x, c->yb)) != RBM_OK) return s;
  if ((s = far_traction(c, S, x, 0, 0)) != RBM_OK) return s;
  HIPCHECK(launch_combine(N, c->M, c->far_nslots, c->part, 1.0, nullptr, 0.0, c->yb, c->Rm, 1.0, out, c->st));
  S.matvecs++;
  return RBM_OK;
}

// out = v + K_far(w R P~^{-1} R^T v): the right-preconditioned operator A P^{-1}
static rbm_status apply_AP(rbm_ctx* c, SolveState& S, int prec, const double* v, double* out) {
  const int N = c->n * c->M;
  rbm_status s;
  if ((s = self_apply(c, S, 1, prec, v, c->yb)) != RBM_OK) return s;
  if ((s = far_traction(c, S, c->yb, 1, prec == 0 ? 0 : 1)) != RBM_OK) return s;
  HIPCHECK(launch_combine(N, c->M, c->far_nslots, c->part, 1.0, v, 1.0, nullptr, nullptr, 0.0, out, c->st));
  S.matvecs++;
  return RBM_OK;
}

// Wait for a value >= 0 (or NaN) that a kernel of the context's stream writes into pinned
// host memory over the sentinel -1, reading it as soon as it lands instead of waiting
// for the stream to drain; between reads the stream is checked for errors, and a
// drained stream without the value is reported.  The host spins for the first 2 ms (an
// iteration at up to ~10^5 points) and then polls every few tens of microseconds, so a
// long iteration does not hold a CPU core.
static rbm_status wait_pinned(rbm_ctx* c, volatile double* p, double* out) {
  const auto t0 = std::chrono::steady_clock::now();
  bool nap = false;
  for (unsigned it = 1;; ++it) {
    const double v = *p;
    if (v != -1.0) {
      *out = v;
      return RBM_OK;
    }
    if (nap) std::this_thread::sleep_for(std::chrono::microseconds(20));
    if ((it & 63) == 0 || nap) {
      if (!nap && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) nap = true;
      const hipError_t q = hipStreamQuery(c->st);
      if (q == hipSuccess) {
        const double v2 = *p;
        if (v2 == -1.0) return fail(RBM_E_DEVICE, "device result not written to pinned memory");
        *out = v2;
        return RBM_OK;
      }
      if (q != hipErrorNotReady) return fail(RBM_E_DEVICE, hipGetErrorString(q));
    }
  }
}

// ||w|| of w[0, len) (len = 0: a traction-sized vector) written by the norm kernel into
// pinned slot `slot` over the sentinel -1; wait_pinned reads it.
static rbm_status norm_to_pinned(rbm_ctx* c, const double* w, int slot, size_t len = 0) {
  if (len == 0) len = 3 * (size_t)c->n * c->M;
  c->pinned[slot] = -1.0;
  HIPCHECK(launch_dots(1, len, w, len, w, c->partial, c->nblk, c->st));
  HIPCHECK(launch_dots_final_sqrt(c->nblk, c->partial, c->pinned_dev + slot, c->st));
  return RBM_OK;
}

static rbm_status read_norm(rbm_ctx* c, const double* w, double* v, size_t len = 0) {
  rbm_status s;
  if ((s = norm_to_pinned(c, w, 24, len)) != RBM_OK) return s;
  return wait_pinned(c, c->pinned + 24, v);
}

static rbm_status read_scalar(rbm_ctx* c, const double* d, double* h) {
  HIPCHECK(hipMemcpyAsync(c->pinned, d, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHECK(hipStreamSynchronize(c->st));
  *h = c->pinned[0];
  return RBM_OK;
}

// One GMRES cycle on A delta = r (right preconditioned, CGS2), starting from 0, with
// V_0 = r/||r||; stops when the residual estimate <= abs_tol or after max_iter.
// On exit mu += P~^{-1} V y (lab frame).  prec: 0 fp64, 1 fp32, 2 bf16 operators.
static rbm_status gmres_cycle(rbm_ctx* c, SolveState& S, int prec, const double* r, double rnorm,
                              double abs_tol, int* iters, double* est = nullptr) {
  const size_t len = 3 * (size_t)c->n * c->M;
  const int m = c->opt.max_iter;
  const int ldh = m + 1;
  const int N = c->n * c->M;
  rbm_status s;
  // g = (rnorm, 0, ...), H = 0, V0 = r / rnorm
  HIPCHECK(launch_gmres_init(len, r, rnorm, c->V, m + 2, c->g, (size_t)(m + 1) * (m + 1), c->H, c->st));
  // Iteration j: w = V[j+1] = A P~^-1 V[j], then CGS2 against V[0..j], normalisation,
  // Givens rotation and |g_{j+1}| in four launches; the residual estimate lands in
  // pinned host memory (two slots, alternating) and is read as soon as it does.
  const auto enqueue = [&](int j) -> rbm_status {
    rbm_status s2;
    if ((s2 = apply_AP(c, S, prec, c->V + (size_t)j * len, c->V + (size_t)(j + 1) * len)) != RBM_OK)
      return s2;
    c->pinned[16 + (j & 1)] = -1.0;
    HIPCHECK(launch_arnoldi(j, len, c->V, len, c->partial, (size_t)(m + 2) * c->nblk, c->nblk, ldh, c->H,
                            c->cs, c->sn, c->g, c->pinned_dev + 16 + (j & 1), c->st));
    return RBM_OK;
  };
  // While the residual estimates fall at a steady rate and the next one is predicted at
  // more than 8 abs_tol, iteration k+1 is queued before iteration k's estimate is read,
  // so the GPU does not idle through the host's round trip.  If k converges after all,
  // k+1 only wrote V[k+2], column k+1 of H, rotation k+1 (cs, sn), g[k+1..k+2] and scratch
  // buffers; the solution over the first k+1 columns reads H and g up to row k only.
  if ((s = enqueue(0)) != RBM_OK) return s;
  double prev1 = rnorm, prev2 = -1.0;  // estimates after iterations k-1 and k-2
  double last = rnorm;
  int k = 0;
  for (k = 0; k < m; ++k) {
    bool ahead = false;
    if (k + 1 < m && c->opt.gmres_lookahead == 2) ahead = true;
    if (k + 1 < m && c->opt.gmres_lookahead == 1 && prev2 > 0.0)
      ahead = prev1 * std::min(1.0, prev1 / prev2) > 8.0 * abs_tol;
    if (ahead && (s = enqueue(k + 1)) != RBM_OK) return s;
    double res;
    if ((s = wait_pinned(c, c->pinned + 16 + (k & 1), &res)) != RBM_OK) return s;
    if (!std::isfinite(res)) return fail(RBM_E_DEVICE, "non-finite GMRES residual");
    last = res;
    if (res <= abs_tol) { ++k; break; }
    if (!ahead && k + 1 < m && (s = enqueue(k + 1)) != RBM_OK) return s;
    prev2 = prev1;
    prev1 = res;
  }
  if (k > m) k = m;
  *iters = k;
  if (est) *est = last;
  HIPCHECK(launch_backsolve(k, ldh, c->H, c->g, c->y, c->st));
  HIPCHECK(launch_vupdate(k, len, c->V, len, c->y, c->t2, 1, c->st));
  if ((s = self_apply(c, S, 1, prec, c->t2, c->yb)) != RBM_OK) return s;
  HIPCHECK(launch_combine(N, c->M, 0, nullptr, 0.0, c->mu, 1.0, c->yb, c->Rm, 1.0, c->mu, c->st));
  return RBM_OK;
}

static rbm_status learned_correction(rbm_ctx* c, const double* dFT);
static rbm_status learned_capture(rbm_ctx* c, const double* dFT);

// Incident density (§2.2) and right-hand side b = -(A_self rho - L rho + K_far rho).
// exact = false evaluates K_far rho in the cheaper precision (float32 direct sum, or the
// fast multipole method when a tree is built): b then serves only the block-diagonal guess
// and the scale ||b|| of the stopping test, while residuals come from residual_exact().
static rbm_status build_rhs(rbm_ctx* c, SolveState& S, const double* dFT, const double* d_rho,
                            double* bnorm, bool exact = true, double* rhonorm = nullptr) {
  hipStream_t st = c->st;
  const int n = c->n, M = c->M, N = n * M;
  rbm_status s;
  if (d_rho)
    HIPCHECK(hipMemcpyAsync(c->rho, d_rho, 3 * (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, st));
  else
    HIPCHECK(launch_rho(n, M, dFT, c->cen, c->X, c->tauinv, c->area_b, c->rho, st));
  if ((s = self_apply(c, S, 0, 0, c->rho, c->yb)) != RBM_OK) return s;
  if ((s = far_traction(c, S, c->rho, 0, exact ? 0 : 1)) != RBM_OK) return s;
  HIPCHECK(launch_combine(N, M, c->far_nslots, c->part, -1.0, nullptr, 0.0, c->yb, c->Rm, -1.0, c->b, st));
  HIPCHECK(launch_moments(n, M, c->rho, c->X, c->W, c->cen, c->mom, st));
  HIPCHECK(launch_add_rigid(n, M, c->mom, c->X, c->cen, 1.0, c->b, st));
  S.matvecs++;
  // ||b|| and ||rho|| in one round trip
  if ((s = norm_to_pinned(c, c->b, 24)) != RBM_OK) return s;
  if ((s = norm_to_pinned(c, c->rho, 25)) != RBM_OK) return s;
  double rh;
  if ((s = wait_pinned(c, c->pinned + 24, bnorm)) != RBM_OK) return s;
  if ((s = wait_pinned(c, c->pinned + 25, &rh)) != RBM_OK) return s;
  if (rhonorm) *rhonorm = rh;
  if (!std::isfinite(*bnorm)) return fail(RBM_E_INVAL, "non-finite right-hand side");
  return RBM_OK;
}

// Float64 residual r = b - A x without forming b: by linearity
//   r = -(A_self (rho + x) - L rho) - K_far (rho + x),
// one exact far sum of rho + x (tmp holds rho + x).
// With `velocity`, the traction and Stokeslet sums of rho + x come from one fused pass: the
// Stokeslet partial sums stay in part_u (vel_ready) for the velocities, should this residual
// end the solve.  With `inner`, the far sum is the inner operators' (float32 direct or fast
// multipole) instead of the float64 one: the starting residual of the precision form's first
// refinement, which decides nothing.
static rbm_status residual_exact(rbm_ctx* c, SolveState& S, const double* x, double* r, double* tmp,
                                 bool velocity = false, bool inner = false) {
  const int n = c->n, M = c->M, N = n * M;
  hipStream_t st = c->st;
  rbm_status s;
  HIPCHECK(launch_axpby(3 * (size_t)N, 1.0, c->rho, 1.0, x, tmp, st));
  if ((s = self_apply(c, S, 0, 0, tmp, c->yb)) != RBM_OK) return s;
  c->vel_ready = false;
  if (velocity) {
    const int nsp = split_for(c, N);
    HIPCHECK(launch_pack_sources<double>(N, M, c->X, c->W, c->Rm, tmp, 0, nullptr, c->src, st));
    Timer t(c);
    HIPCHECK(launch_far_ts(N, M, c->X, c->Nn, c->src, c->part, c->part_u, nsp, st));
    t.stop();
    if (t.on) S.fused_ev.push_back({c->ev_used - 2, c->ev_used - 1});
    S.far_pairs += 2.0 * ((double)N * N - (double)n * M * M);
    c->far_base = nsp;
    c->far_nslots = nsp + (c->pu ? 1 : 0);
    if ((s = near_correction(c, S, 0, tmp, 0, 0)) != RBM_OK) return s;
    if ((s = near_correction(c, S, 1, tmp, 0, 0, c->part_u)) != RBM_OK) return s;
    c->vel_ready = true;
  } else if ((s = far_traction(c, S, tmp, 0, inner ? 1 : 0)) != RBM_OK) {
    return s;
  }
  HIPCHECK(launch_combine(N, M, c->far_nslots, c->part, -1.0, nullptr, 0.0, c->yb, c->Rm, -1.0, r, st));
  HIPCHECK(launch_moments(n, M, c->rho, c->X, c->W, c->cen, c->mom, st));
  HIPCHECK(launch_add_rigid(n, M, c->mom, c->X, c->cen, 1.0, r, st));
  S.matvecs++;
  return RBM_OK;
}

static rbm_status solve_impl(rbm_ctx* c, const double* dFT, double* dVW, rbm_solve_info* info,
                             const double* d_rho = nullptr) {
  if (!c->ws) return fail(RBM_E_NOMEM, "bind a workspace first");
  if (!c->setup_done) return fail(RBM_E_STATE, "call rbm_setup first");
  if (c->n < 1) return fail(RBM_E_STATE, "set bodies first");
  rbm_status s;
  if ((s = upload_bodies(c)) != RBM_OK) return s;
  hipStream_t st = c->st;
  const int n = c->n, M = c->M, N = n * M;
  const size_t len = 3 * (size_t)N;
  SolveState S;
  c->ev_used = 0;
  Timer total(c);
  // tree of the fast multipole far field for the inner iterations at these poses
  if (c->opt.fmm_order > 0 && c->opt.precision != RBM_FP64) {
    if ((s = fmm_build(c, N, M, c->X, c->Nn, fmm_dmax(c))) != RBM_OK) return s;
  } else {
    c->fmm_ready = false;
  }
  // Precision form: b only seeds the guess and scales the tolerance (every residual is
  // exact), so its far sum is the cheap one.  Float64 form, or a zero guess (the first
  // residual is b itself): b is exact.
  double bnorm, rhonorm;
  const bool b_exact = c->opt.precision == RBM_FP64 || c->opt.guess == RBM_GUESS_ZERO;
  if ((s = build_rhs(c, S, dFT, d_rho, &bnorm, b_exact, &rhonorm)) != RBM_OK) return s;
  // b at the rounding level of the terms it is formed from (an isolated sphere, whose incident
  // density already solves the problem, or zero loads) is zero: mu = 0 solves the system to
  // rounding and a relative test on ||b|| would only compare rounding errors
  const bool b_zero = bnorm <= 64.0 * DBL_EPSILON * rhonorm;
  if (b_zero) bnorm = 0.0;
  const double abs_tol = c->opt.tol * bnorm;
  const int prec = c->opt.precision;
  // initial guess
  bool mu_zero = false, learned_active = false;
  int guess_used = c->opt.guess, fallback = 0;
  if (bnorm == 0.0 || c->opt.guess == RBM_GUESS_ZERO) {
    HIPCHECK(hipMemsetAsync(c->mu, 0, len * sizeof(double), st));
    mu_zero = true;
    guess_used = RBM_GUESS_ZERO;
  } else if (c->opt.guess == RBM_GUESS_BLOCKDIAG || c->opt.guess == RBM_GUESS_LEARNED) {
    // block-diagonal (isolated-particle) guess mu_BD = P^{-1} b (§3.2 preconditioner)
    if ((s = self_apply(c, S, 1, prec, c->b, c->yb)) != RBM_OK) return s;
    HIPCHECK(launch_combine(N, M, 0, nullptr, 0.0, nullptr, 0.0, c->yb, c->Rm, 1.0, c->mu, st));
    if (c->opt.guess == RBM_GUESS_LEARNED && c->L.bound && c->L.stats_ready && !d_rho) {
      HIPCHECK(hipMemcpyAsync(c->t2, c->mu, len * sizeof(double), hipMemcpyDeviceToDevice, st));
      if ((s = learned_correction(c, dFT)) != RBM_OK) return s;
      learned_active = true;
    } else {
      guess_used = RBM_GUESS_BLOCKDIAG;
    }
  } else {
    if (!c->guess_set) return fail(RBM_E_STATE, "RBM_GUESS_USER needs rbm_set_guess_dev");
    HIPCHECK(hipMemcpyAsync(c->mu, c->guess, len * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  int total_iters = 0, cycles = 0, refinements = 0, fp64_cycles = 0;
  double rel = 0.0, init_rel = 0.0;
  bool converged = false;
  const int max_outer = prec == 0 ? c->opt.max_restart + 1 : 50;
  // GMRES-IR: inner operators in the form's precision until a refinement stalls (its
  // float64 residual not below ir_stall times the previous one); then float64 operators
  int prec_in = prec;
  double rn_prev = -1.0;
  // The exact residual that ends the solve is evaluated for sigma = rho + mu, the density
  // whose Stokeslet sum gives the velocities: when the next residual is predicted to meet the
  // tolerance, both sums come from one fused pass (a wrong prediction costs the Stokeslet
  // part of that pass, about 0.4 of a traction sum).  Prediction: with float64 operators the
  // GMRES estimate; in the precision form the estimate plus eps_op times the residual the
  // cycle started from (plus ||b|| when that residual was the inner operators' own), eps_op
  // the relative accuracy of the inner operators: at first 1e-4
  // with fast multipole sums, 2^-22 with float32 direct sums and 2^-8 with bf16 blocks, then
  // what the last refinement showed (its exact residual beyond its estimate).
  bool fuse_next = false;
  double eps_op = c->fmm_ready ? 1e-4 : prec == RBM_MIXED_BF16 ? std::ldexp(1.0, -8) : std::ldexp(1.0, -22);
  double est_prev = -1.0, rn_cycle = -1.0;
  int prec_cycle = prec;
  bool cycle_from_inner = false, last_exact = true;
  c->vel_ready = false;
  for (int outer = 0; outer <= max_outer; ++outer) {
    // residual r = b - A mu: float64, except that the precision form starts its first
    // refinement from the residual of its inner operators (every residual that decides
    // convergence is float64; the first comes after the first refinement, which the inner
    // operators' accuracy bounds alike from either starting residual)
    double rn;
    bool exact = true;
    if (mu_zero) {
      HIPCHECK(hipMemcpyAsync(c->r, c->b, len * sizeof(double), hipMemcpyDeviceToDevice, st));
      rn = bnorm;
      mu_zero = false;
    } else {
      exact = !(outer == 0 && prec != 0);
      if ((s = residual_exact(c, S, c->mu, c->r, c->t1, exact && fuse_next, !exact)) != RBM_OK) return s;
      if ((s = read_norm(c, c->r, &rn)) != RBM_OK) return s;
    }
    if (outer == 0 && bnorm > 0.0) {
      if (learned_active) {
        // fallback test against the block-diagonal guess's residual ratio (residuals of the
        // same kind as this one)
        if (c->bd_ratio < 0.0) {
          if ((s = residual_exact(c, S, c->t2, c->t1, c->V, false, !exact)) != RBM_OK) return s;  // V is free before GMRES
          double rbd;
          if ((s = read_norm(c, c->t1, &rbd)) != RBM_OK) return s;
          c->bd_ratio = rbd / bnorm;
        }
        if (!(rn <= c->bd_ratio * bnorm)) {
          fallback = 1;
          HIPCHECK(hipMemcpyAsync(c->mu, c->t2, len * sizeof(double), hipMemcpyDeviceToDevice, st));
          if ((s = residual_exact(c, S, c->mu, c->r, c->t1, false, !exact)) != RBM_OK) return s;
          if ((s = read_norm(c, c->r, &rn)) != RBM_OK) return s;
          c->bd_ratio = rn / bnorm;
        }
      } else if (guess_used == RBM_GUESS_BLOCKDIAG) {
        c->bd_ratio = rn / bnorm;
      }
      init_rel = rn / bnorm;
    }
    last_exact = exact;
    if (c->verbose)
      std::fprintf(stderr, "[rbm] refinement %d: %s residual %.3e (relative), inner precision %d, fused %d\n",
                   outer, exact ? "float64" : "inner", bnorm > 0.0 ? rn / bnorm : 0.0, prec_in,
                   exact && fuse_next ? 1 : 0);
    if (!exact) {
      // an inner-operator residual already at the tolerance: go to the float64 one
      if (rn <= abs_tol) {
        fuse_next = c->opt.velocity_fusion != 0;
        continue;
      }
    } else {
      rel = bnorm > 0.0 ? rn / bnorm : 0.0;
      if (rn <= abs_tol || bnorm == 0.0) { converged = true; break; }
    }
    if (outer == max_outer) break;
    if (prec_in != 0 && rn_prev > 0.0 && !(rn < c->opt.ir_stall * rn_prev)) prec_in = 0;
    // the inner operators' relative accuracy as the last refinement showed it: its float64
    // residual beyond its estimate, over the residual it started from (plus ||b|| when that
    // was the inner operators' own residual, whose error does not recur)
    if (est_prev >= 0.0 && prec_cycle != 0)
      eps_op = std::max(1e-16, (rn - est_prev) / (rn_cycle + (cycle_from_inner ? bnorm : 0.0)));
    rn_prev = rn;
    double inner_abs = prec_in == 0 ? abs_tol : std::max(c->opt.inner_tol * rn, 0.5 * abs_tol);
    // Float32 inner operators (direct far sum, float32 self blocks) are accurate to about
    // 2^-22: when that accuracy times the error this refinement can leave (the residual it
    // starts from, plus ||b|| when that residual is the inner operators' own, whose right-
    // hand side carries their error too) already meets the tolerance, solve the correction
    // to the tolerance itself and finish in this refinement (the exact residual still
    // decides; a miss costs one more refinement, never accuracy).
    if (prec_in == RBM_MIXED_FP32 && !c->fmm_ready &&
        std::ldexp(rn + (last_exact ? 0.0 : bnorm), -22) <= 0.5 * abs_tol)
      inner_abs = 0.5 * abs_tol;
    int it = 0;
    double est = rn;
    if ((s = gmres_cycle(c, S, prec_in, c->r, rn, inner_abs, &it, &est)) != RBM_OK) return s;
    c->vel_ready = false;  // mu has changed
    total_iters += it;
    cycles++;
    if (prec != 0) refinements++;
    if (prec != 0 && prec_in == 0) fp64_cycles++;
    fuse_next = c->opt.velocity_fusion &&
                (prec_in == 0 ? est <= abs_tol : est + eps_op * (rn + (last_exact ? 0.0 : bnorm)) <= abs_tol);
    if (c->verbose)
      std::fprintf(stderr, "[rbm]   cycle: %d iterations, estimate %.3e (relative), eps_op %.2e, next fused %d\n", it,
                   bnorm > 0.0 ? est / bnorm : 0.0, eps_op, fuse_next ? 1 : 0);
    est_prev = est;
    rn_cycle = rn;
    prec_cycle = prec_in;
    cycle_from_inner = !last_exact;
  }
  // velocities u = S[rho + mu]: far Stokeslet sum (from the fused pass of the last residual
  // when it was evaluated for this mu) + self functional, float64
  HIPCHECK(launch_axpby(len, 1.0, c->rho, 1.0, c->mu, c->t2, st));
  if (c->vel_ready) {
    S.fused_used = true;
    HIPCHECK(launch_combine(N, M, far_slots(c, N), c->part_u, 1.0 / c->opt.eta, nullptr, 0.0, nullptr, nullptr,
                            0.0, c->t1, st));
  } else {
    HIPCHECK(launch_pack_sources<double>(N, M, c->X, c->W, c->Rm, c->t2, 0, nullptr, c->src, st));
    Timer t(c);
    HIPCHECK(launch_far<double>(1, N, M, c->X, nullptr, c->src, c->part, split_for(c, N), st));
    t.stop();
    if (t.on) S.stok_ev.push_back({c->ev_used - 2, c->ev_used - 1});
    S.far_pairs += (double)N * N - (double)n * M * M;
    c->far_base = split_for(c, N);
    if ((s = near_correction(c, S, 1, c->t2, 0, 0)) != RBM_OK) return s;
    HIPCHECK(launch_combine(N, M, far_slots(c, N), c->part, 1.0 / c->opt.eta, nullptr, 0.0, nullptr, nullptr,
                            0.0, c->t1, st));
  }
  c->vel_ready = false;
  HIPCHECK(launch_moments(n, M, c->t1, c->X, c->W, c->cen, c->mom, st));
  HIPCHECK(launch_velocity_self(n, M, c->sid, c->V0, c->Rm, c->t2, c->vws, st));
  HIPCHECK(launch_velocity_final(n, c->mom, c->vws, c->tauinv, c->area_b, dVW, st));
  total.stop();
  HIPCHECK(hipStreamSynchronize(st));
  c->have_solution = true;
  if (c->L.bound && c->L.capture_on && !d_rho)
    if ((s = learned_capture(c, dFT)) != RBM_OK) return s;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->guess_used = guess_used;
    info->fallback_used = fallback;
    info->init_rel_residual = init_rel;
    info->iters = total_iters;
    info->matvecs = S.matvecs;
    info->refinements = refinements;
    info->cycles = cycles;
    info->rel_residual = rel;
    info->bnorm = bnorm;
    info->far_pairs = S.far_pairs;
    info->n_traction = (int)S.trac_ev.size();
    info->n_traction32 = (int)S.trac32_ev.size();
    info->n_stokeslet = (int)S.stok_ev.size();
    info->pairs_per_launch = (double)N * N - (double)n * M * M;
    info->near_pairs = c->pu ? c->near_pairs : 0;
    info->fmm_level = c->fmm_ready ? c->fmm_level : -1;
    info->fmm_applies = S.fmm_applies;
    info->fp64_cycles = fp64_cycles;
    info->n_fused = (int)S.fused_ev.size();
    info->fused_used = S.fused_used ? 1 : 0;
    if (total.on) {
      float ms = 0;
      (void)hipEventElapsedTime(&ms, total.a, total.b);
      info->ms_total = ms;
      for (auto& e : S.trac_ev) {
        (void)hipEventElapsedTime(&ms, c->ev[e.first], c->ev[e.second]);
        info->ms_traction += ms;
      }
      for (auto& e : S.trac32_ev) {
        (void)hipEventElapsedTime(&ms, c->ev[e.first], c->ev[e.second]);
        info->ms_traction32 += ms;
      }
      for (auto& e : S.stok_ev) {
        (void)hipEventElapsedTime(&ms, c->ev[e.first], c->ev[e.second]);
        info->ms_stokeslet += ms;
      }
      for (auto& e : S.fused_ev) {
        (void)hipEventElapsedTime(&ms, c->ev[e.first], c->ev[e.second]);
        info->ms_fused += ms;
      }
      info->ms_far = info->ms_traction + info->ms_traction32 + info->ms_stokeslet + info->ms_fused;
      for (auto& e : S.self_ev) {
        (void)hipEventElapsedTime(&ms, c->ev[e.first], c->ev[e.second]);
        info->ms_self += ms;
      }
      for (auto& e : S.near_ev) {
        (void)hipEventElapsedTime(&ms, c->ev[e.first], c->ev[e.second]);
        info->ms_near += ms;
      }
    }
  }
  if (!converged) return fail(RBM_E_NOCONV, "GMRES did not reach tol");
  return RBM_OK;
}

extern "C" rbm_status rbm_solve_dev(rbm_ctx* c, const double* d_FT, double* d_VW,
                                    rbm_solve_info* info) {
  if (!c || !d_FT || !d_VW) return fail(RBM_E_INVAL, "null argument");
  return solve_impl(c, d_FT, d_VW, info);
}

extern "C" rbm_status rbm_solve(rbm_ctx* c, const double* FT, double* VW, rbm_solve_info* info) {
  if (!c || !FT || !VW) return fail(RBM_E_INVAL, "null argument");
  if (!c->ws) return fail(RBM_E_NOMEM, "bind a workspace first");
  if (!all_finite(FT, 6 * (size_t)c->n)) return fail(RBM_E_INVAL, "non-finite load");
  HIPCHECK(hipMemcpyAsync(c->FT, FT, 6 * c->n * sizeof(double), hipMemcpyHostToDevice, c->st));
  rbm_status s = solve_impl(c, c->FT, c->VW, info);
  if (s != RBM_OK && s != RBM_E_NOCONV) return s;
  HIPCHECK(hipMemcpyAsync(VW, c->VW, 6 * c->n * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHECK(hipStreamSynchronize(c->st));
  return s;
}

extern "C" rbm_status rbm_set_guess_dev(rbm_ctx* c, const double* d_mu0) {
  if (!c || !d_mu0) return fail(RBM_E_INVAL, "null argument");
  if (!c->ws) return fail(RBM_E_NOMEM, "bind a workspace first");
  const size_t len = 3 * (size_t)c->n * c->M;
  HIPCHECK(hipMemcpyAsync(c->guess, d_mu0, len * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  HIPCHECK(hipStreamSynchronize(c->st));
  c->guess_set = true;
  return RBM_OK;
}

extern "C" rbm_status rbm_get_density(rbm_ctx* c, double* mu, double* rho) {
  if (!c) return fail(RBM_E_INVAL, "null argument");
  if (!c->have_solution) return fail(RBM_E_STATE, "no solution yet");
  const size_t len = 3 * (size_t)c->n * c->M;
  if (mu) HIPCHECK(hipMemcpy(mu, c->mu, len * sizeof(double), hipMemcpyDeviceToHost));
  if (rho) HIPCHECK(hipMemcpy(rho, c->rho, len * sizeof(double), hipMemcpyDeviceToHost));
  return RBM_OK;
}

extern "C" rbm_status rbm_apply_dev(rbm_ctx* c, const double* d_mu, double* d_y) {
  if (!c || !d_mu || !d_y) return fail(RBM_E_INVAL, "null argument");
  if (!c->ws) return fail(RBM_E_NOMEM, "bind a workspace first");
  if (!c->setup_done) return fail(RBM_E_STATE, "call rbm_setup first");
  if (c->n < 1) return fail(RBM_E_STATE, "set bodies first");
  if (d_mu == d_y) return fail(RBM_E_INVAL, "d_mu and d_y must not alias");
  rbm_status s;
  if ((s = upload_bodies(c)) != RBM_OK) return s;
  SolveState S;
  c->ev_used = 0;
  if ((s = apply_A(c, S, d_mu, d_y)) != RBM_OK) return s;
  HIPCHECK(hipStreamSynchronize(c->st));
  return RBM_OK;
}

extern "C" rbm_status rbm_find_contacts(rbm_ctx* c, double delta, int max_contacts, int* n_found,
                                        int* pairs, double* points) {
  if (!c || !n_found) return fail(RBM_E_INVAL, "null argument");
  if (max_contacts < 0 || (max_contacts > 0 && (!pairs || !points)))
    return fail(RBM_E_INVAL, "max_contacts >= 0 with pairs and points for max_contacts > 0");
  if (!(delta > 0.0) || !std::isfinite(delta)) return fail(RBM_E_INVAL, "delta must be > 0");
  if (!c->ws) return fail(RBM_E_NOMEM, "bind a workspace first");
  if (!c->setup_done) return fail(RBM_E_STATE, "call rbm_setup first");
  if (c->n < 1) return fail(RBM_E_STATE, "set bodies first");
  rbm_status s;
  if ((s = upload_bodies(c)) != RBM_OK) return s;
  const int n = c->n, M = c->M;
  // candidates: bounding spheres (largest centroid-to-node distance) within delta
  std::vector<int> cand;
  for (int a = 0; a < n; ++a)
    for (int b = a + 1; b < n; ++b) {
      const double* ca = &c->cen_h[3 * a];
      const double* cb = &c->cen_h[3 * b];
      const double dx = ca[0] - cb[0], dy = ca[1] - cb[1], dz = ca[2] - cb[2];
      if (std::sqrt(dx * dx + dy * dy + dz * dz) < c->rbc_h[c->sid_h[a]] + c->rbc_h[c->sid_h[b]] + delta) {
        cand.push_back(a);
        cand.push_back(b);
      }
    }
  const int ncand = (int)cand.size() / 2;
  if ((size_t)ncand > (size_t)kContactCand * c->nmax)
    return fail(RBM_E_INVAL, "too many contact candidates: lower delta");
  std::vector<double> res(5 * (size_t)ncand);
  if (ncand) {
    HIPCHECK(hipMemcpyAsync(c->ccand, cand.data(), cand.size() * sizeof(int), hipMemcpyHostToDevice, c->st));
    HIPCHECK(launch_closest_pairs(ncand, n * M, M, c->ccand, c->X, c->cres, c->st));
    HIPCHECK(hipMemcpyAsync(res.data(), c->cres, res.size() * sizeof(double), hipMemcpyDeviceToHost, c->st));
  }
  HIPCHECK(hipStreamSynchronize(c->st));
  int found = 0;
  for (int k = 0; k < ncand; ++k) {
    if (!(std::sqrt(res[5 * k]) < delta)) continue;
    if (found < max_contacts) {
      pairs[2 * found] = cand[2 * k];
      pairs[2 * found + 1] = cand[2 * k + 1];
      for (int e = 0; e < 3; ++e) points[3 * found + e] = res[5 * k + 2 + e];
    }
    ++found;
  }
  *n_found = found;
  return RBM_OK;
}

// LU with partial pivoting of the small dense system A x = b (A row-major n x n,
// overwritten); false if a pivot vanishes.
static bool small_solve(int n, std::vector<double>& A, std::vector<double>& b) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[(size_t)i * n + k]) > std::fabs(A[(size_t)piv * n + k])) piv = i;
    if (!(std::fabs(A[(size_t)piv * n + k]) > 0.0)) return false;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)piv * n + j]);
      std::swap(b[k], b[piv]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = A[(size_t)i * n + k] / A[(size_t)k * n + k];
      for (int j = k; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double v = b[k];
    for (int j = k + 1; j < n; ++j) v -= A[(size_t)k * n + j] * b[j];
    b[k] = v / A[(size_t)k * n + k];
  }
  return true;
}

static rbm_status contact_correct(rbm_ctx* c, const std::vector<double>& V0, rbm_solve_info i0,
                                  int n_contacts, const int* pairs, const double* points, double* VW,
                                  double* Fc, rbm_solve_info* info);

extern "C" rbm_status rbm_solve_contacts(rbm_ctx* c, const double* FT, int n_contacts,
                                         const int* pairs, const double* points, double* VW,
                                         double* Fc, rbm_solve_info* info) {
  if (!c || !FT || !VW) return fail(RBM_E_INVAL, "null argument");
  if (n_contacts < 0 || (n_contacts > 0 && (!pairs || !points || !Fc)))
    return fail(RBM_E_INVAL, "n_contacts >= 0 with pairs, points and Fc for n_contacts > 0");
  const int n = c->n;
  for (int k = 0; k < n_contacts; ++k) {
    const int a = pairs[2 * k], b = pairs[2 * k + 1];
    if (a < 0 || b < 0 || a >= n || b >= n || a == b) return fail(RBM_E_INVAL, "bad contact pair");
    if (!all_finite(points + 3 * k, 3)) return fail(RBM_E_INVAL, "non-finite contact point");
  }
  rbm_solve_info i0;
  std::vector<double> V0(6 * (size_t)n);
  rbm_status s = rbm_solve(c, FT, V0.data(), &i0);
  if (s != RBM_OK) return s;
  return contact_correct(c, V0, i0, n_contacts, pairs, points, VW, Fc, info);
}

// Given the velocities V0 without contact forces (host, [n][6]) and the validated
// contact list: the mobility solves of the unit contact forces, (D M C) F_c = -D V0 and
// VW = V0 + M C F_c.  i0 carries V0's solve statistics and accumulates the rest.
static rbm_status contact_correct(rbm_ctx* c, const std::vector<double>& V0, rbm_solve_info i0,
                                  int n_contacts, const int* pairs, const double* points, double* VW,
                                  double* Fc, rbm_solve_info* info) {
  const int n = c->n;
  rbm_solve_info ik;
  rbm_status s;
  const int m = 3 * n_contacts;
  std::vector<double> Vc((size_t)m * 6 * n), load(6 * (size_t)n);
  // column (k, e) of M C: the solve for a unit force along e at x_k on body a, its
  // opposite on body b, torques about the centroids
  for (int k = 0; k < n_contacts; ++k) {
    const int a = pairs[2 * k], b = pairs[2 * k + 1];
    const double* xs = points + 3 * k;
    double ra[3], rb[3];
    for (int d = 0; d < 3; ++d) {
      ra[d] = xs[d] - c->cen_h[3 * a + d];
      rb[d] = xs[d] - c->cen_h[3 * b + d];
    }
    for (int e = 0; e < 3; ++e) {
      std::fill(load.begin(), load.end(), 0.0);
      double f[3] = {0, 0, 0};
      f[e] = 1.0;
      const double ta[3] = {ra[1] * f[2] - ra[2] * f[1], ra[2] * f[0] - ra[0] * f[2], ra[0] * f[1] - ra[1] * f[0]};
      const double tb[3] = {rb[1] * f[2] - rb[2] * f[1], rb[2] * f[0] - rb[0] * f[2], rb[0] * f[1] - rb[1] * f[0]};
      for (int d = 0; d < 3; ++d) {
        load[6 * a + d] += f[d];
        load[6 * a + 3 + d] += ta[d];
        load[6 * b + d] -= f[d];
        load[6 * b + 3 + d] -= tb[d];
      }
      s = rbm_solve(c, load.data(), &Vc[(size_t)(3 * k + e) * 6 * n], &ik);
      if (s != RBM_OK) return s;
      i0.iters += ik.iters;
      i0.matvecs += ik.matvecs;
      i0.ms_total += ik.ms_total;
      i0.ms_far += ik.ms_far;
      i0.ms_self += ik.ms_self;
      i0.far_pairs += ik.far_pairs;
    }
  }
  // velocity differences at the contact points: D V
  auto dvel = [&](const double* V, int k, double* out) {
    const int a = pairs[2 * k], b = pairs[2 * k + 1];
    const double* xs = points + 3 * k;
    double ra[3], rb[3];
    for (int d = 0; d < 3; ++d) {
      ra[d] = xs[d] - c->cen_h[3 * a + d];
      rb[d] = xs[d] - c->cen_h[3 * b + d];
    }
    const double* va = V + 6 * a;
    const double* vb = V + 6 * b;
    const double ua[3] = {va[0] + va[4] * ra[2] - va[5] * ra[1], va[1] + va[5] * ra[0] - va[3] * ra[2],
                          va[2] + va[3] * ra[1] - va[4] * ra[0]};
    const double ub[3] = {vb[0] + vb[4] * rb[2] - vb[5] * rb[1], vb[1] + vb[5] * rb[0] - vb[3] * rb[2],
                          vb[2] + vb[3] * rb[1] - vb[4] * rb[0]};
    for (int d = 0; d < 3; ++d) out[d] = ua[d] - ub[d];
  };
  std::vector<double> A((size_t)m * m), rhs(m);
  for (int col = 0; col < m; ++col)
    for (int k = 0; k < n_contacts; ++k) {
      double d[3];
      dvel(&Vc[(size_t)col * 6 * n], k, d);
      for (int e = 0; e < 3; ++e) A[(size_t)(3 * k + e) * m + col] = d[e];
    }
  for (int k = 0; k < n_contacts; ++k) {
    double d[3];
    dvel(V0.data(), k, d);
    for (int e = 0; e < 3; ++e) rhs[3 * k + e] = -d[e];
  }
  if (m > 0 && !small_solve(m, A, rhs)) return fail(RBM_E_INVAL, "singular contact system");
  for (size_t i = 0; i < V0.size(); ++i) {
    double v = V0[i];
    for (int col = 0; col < m; ++col) v += rhs[col] * Vc[(size_t)col * 6 * n + i];
    VW[i] = v;
  }
  for (int col = 0; col < m; ++col) Fc[col] = rhs[col];
  if (info) *info = i0;
  return RBM_OK;
}

extern "C" rbm_status rbm_solve_density_dev(rbm_ctx* c, const double* d_rho, double* d_VW,
                                           rbm_solve_info* info) {
  if (!c || !d_rho || !d_VW) return fail(RBM_E_INVAL, "null argument");
  return solve_impl(c, nullptr, d_VW, info, d_rho);
}

// w = 1/2 v + eta (K^L_self v + K^L_far v) on scalar node vectors (float64).
static rbm_status magnetic_apply(rbm_ctx* c, double eta, const double* v, double* w) {
  const int n = c->n, M = c->M, N = n * M;
  const int nsp = split_for(c, N);
  HIPCHECK(launch_scalar_self(n, M, c->sid, c->KL0, v, c->mtmp, c->st));
  HIPCHECK(launch_pack_scalar(N, c->X, c->W, v, c->src, c->st));
  HIPCHECK(launch_far<double>(2, N, M, c->X, c->Nn, c->src, c->part, nsp, c->st));
  HIPCHECK(launch_scalar_combine(N, nsp, c->part, eta, c->mtmp, eta, v, 0.5, w, c->st));
  return RBM_OK;
}

// Unpreconditioned restarted GMRES (CGS2) for (1/2 I + eta K^L) x = b, x starting at 0;
// the operator is second kind with |eta| < 1.
static rbm_status magnetic_gmres(rbm_ctx* c, double eta, const double* b, double* x, double tol,
                                 int* iters) {
  const size_t len = (size_t)c->n * c->M;
  const int m = c->opt.max_iter, ldh = m + 1;
  rbm_status s;
  double bn;
  if ((s = read_norm(c, b, &bn, len)) != RBM_OK) return s;
  HIPCHECK(hipMemsetAsync(x, 0, len * sizeof(double), c->st));
  *iters = 0;
  if (bn == 0.0) return RBM_OK;
  double* r = c->mb;  // residual
  HIPCHECK(hipMemcpyAsync(r, b, len * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  double rn = bn;
  for (int cycle = 0; cycle <= c->opt.max_restart; ++cycle) {
    HIPCHECK(launch_gmres_init(len, r, rn, c->V, m + 2, c->g, (size_t)(m + 1) * (m + 1), c->H, c->st));
    int k;
    for (k = 0; k < m; ++k) {
      // w = V[k+1] = A V[k], then the fused Arnoldi step of the mobility GMRES
      if ((s = magnetic_apply(c, eta, c->V + (size_t)k * len, c->V + (size_t)(k + 1) * len)) != RBM_OK)
        return s;
      c->pinned[16] = -1.0;
      HIPCHECK(launch_arnoldi(k, len, c->V, len, c->partial, (size_t)(m + 2) * c->nblk, c->nblk, ldh, c->H,
                              c->cs, c->sn, c->g, c->pinned_dev + 16, c->st));
      double res;
      if ((s = wait_pinned(c, c->pinned + 16, &res)) != RBM_OK) return s;
      if (!std::isfinite(res)) return fail(RBM_E_DEVICE, "non-finite GMRES residual");
      ++*iters;
      if (res <= tol * bn) { ++k; break; }
    }
    if (k > m) k = m;
    HIPCHECK(launch_backsolve(k, ldh, c->H, c->g, c->y, c->st));
    HIPCHECK(launch_vupdate(k, len, c->V, len, c->y, c->mtmp, 1, c->st));
    HIPCHECK(launch_axpby(len, 1.0, x, 1.0, c->mtmp, x, c->st));
    // true residual r = b - A x
    if ((s = magnetic_apply(c, eta, x, c->mphi)) != RBM_OK) return s;
    HIPCHECK(launch_axpby(len, 1.0, b, -1.0, c->mphi, r, c->st));
    if ((s = read_norm(c, r, &rn, len)) != RBM_OK) return s;
    if (rn <= tol * bn) return RBM_OK;
  }
  return fail(RBM_E_NOCONV, "magnetic GMRES did not reach tol");
}

static rbm_status magnetic_traction_impl(rbm_ctx* c, const double* H0, double mu_ratio, double mu0,
                                         double tol, double* d_rho, double* d_FT, int* iters);

extern "C" rbm_status rbm_magnetic_traction_dev(rbm_ctx* c, const double* H0, double mu_ratio,
                                               double mu0, double tol, double* d_rho, double* d_FT,
                                               int* iters) {
  if (!c || !H0 || !d_rho) return fail(RBM_E_INVAL, "null argument");
  if (!c->opt.magnetic) return fail(RBM_E_STATE, "create the context with options.magnetic = 1");
  if (!(mu_ratio > 0.0) || !std::isfinite(mu_ratio) || !(mu0 > 0.0) || !std::isfinite(mu0) ||
      !(tol > 0.0) || !all_finite(H0, 3))
    return fail(RBM_E_INVAL, "mu_ratio, mu0, tol must be > 0 and H0 finite");
  if (!c->ws) return fail(RBM_E_NOMEM, "bind a workspace first");
  if (!c->setup_done) return fail(RBM_E_STATE, "call rbm_setup first");
  if (c->n < 1) return fail(RBM_E_STATE, "set bodies first");
  rbm_status s;
  if ((s = upload_bodies(c)) != RBM_OK) return s;
  return magnetic_traction_impl(c, H0, mu_ratio, mu0, tol, d_rho, d_FT, iters);
}

// Density q, potential, exterior normal derivative, field and Maxwell traction at the
// current poses (arguments validated by the caller).
static rbm_status magnetic_traction_impl(rbm_ctx* c, const double* H0, double mu_ratio, double mu0,
                                         double tol, double* d_rho, double* d_FT, int* iters) {
  rbm_status s;
  const int n = c->n, M = c->M, N = n * M;
  const int nsp = split_for(c, N);
  const double eta = (mu_ratio - 1.0) / (mu_ratio + 1.0);
  hipStream_t st = c->st;
  // q from (1/2 I + eta K^L) q = eta H0 . n
  HIPCHECK(launch_hdot(N, c->Nn, H0[0], H0[1], H0[2], eta, 0, c->mdn, st));
  int it = 0;
  if ((s = magnetic_gmres(c, eta, c->mdn, c->mq, tol, &it)) != RBM_OK) return s;
  if (iters) *iters = it;
  // phi = -H0 . X + S^L q
  HIPCHECK(launch_scalar_self(n, M, c->sid, c->SL0, c->mq, c->mtmp, st));
  HIPCHECK(launch_pack_scalar(N, c->X, c->W, c->mq, c->src, st));
  HIPCHECK(launch_far<double>(3, N, M, c->X, c->Nn, c->src, c->part, nsp, st));
  HIPCHECK(launch_scalar_combine(N, nsp, c->part, 1.0, c->mtmp, 1.0, nullptr, 0.0, c->mphi, st));
  HIPCHECK(launch_hdot(N, c->X, H0[0], H0[1], H0[2], -1.0, 1, c->mphi, st));
  // exterior normal derivative dn = -H0 . n - q/2 + K^L q
  HIPCHECK(launch_scalar_self(n, M, c->sid, c->KL0, c->mq, c->mtmp, st));
  HIPCHECK(launch_far<double>(2, N, M, c->X, c->Nn, c->src, c->part, nsp, st));
  HIPCHECK(launch_scalar_combine(N, nsp, c->part, 1.0, c->mtmp, 1.0, c->mq, -0.5, c->mdn, st));
  HIPCHECK(launch_hdot(N, c->Nn, H0[0], H0[1], H0[2], -1.0, 1, c->mdn, st));
  // field and Maxwell traction
  HIPCHECK(launch_magnetic_traction(n, M, c->sid, c->Rm, c->Nn, c->tang, c->Dth, c->Dph, c->mphi, c->mdn,
                                    mu0, d_rho, st));
  if (d_FT) {
    HIPCHECK(launch_moments(n, M, d_rho, c->X, c->W, c->cen, c->mom, st));
    HIPCHECK(hipMemcpyAsync(d_FT, c->mom, 6 * (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  HIPCHECK(hipStreamSynchronize(st));
  return RBM_OK;
}

extern "C" const void* rbm_debug_ptr(rbm_ctx* c, const char* name) {
  if (!c || !name || !c->ws) return nullptr;
  const std::string s(name);
  if (s == "X") return c->X;
  if (s == "N") return c->Nn;
  if (s == "W") return c->W;
  if (s == "mu") return c->mu;
  if (s == "rho") return c->rho;
  if (s == "b") return c->b;
  if (s == "r") return c->r;
  if (s == "A0") return c->A0;
  if (s == "P0") return c->P0;
  if (s == "V0") return c->V0;
  if (s == "coef") return c->coef;
  if (s == "gr") return c->gr;
  if (s == "gn") return c->gn;
  if (s == "gw") return c->gw;
  if (s == "gx") return c->gx;
  if (s == "shape") return c->shp;
  if (s == "Rm") return c->Rm;
  if (s == "Ftab") return c->Ftab;
  if (s == "Ytab") return c->Ytab;
  if (s == "mag_q") return c->mq;
  if (s == "mag_phi") return c->mphi;
  if (s == "mag_dn") return c->mdn;
  if (s == "SL0") return c->SL0;
  if (s == "KL0") return c->KL0;
  if (s == "U") return c->U;
  if (s == "fr") return c->fr;
  if (s == "fw") return c->fw;
  if (s == "rb") return c->rb;
  if (s == "near_list") return c->nbr;
  if (s == "near_count") return c->ncnt;
  if (s == "learned_X") return c->L.bound ? c->L.Xbuf : nullptr;
  if (s == "learned_T") return c->L.bound ? c->L.Tbuf : nullptr;
  if (s == "learned_m") return c->L.bound ? c->L.Mo : nullptr;
  if (s == "learned_v") return c->L.bound ? c->L.Vo : nullptr;
  return nullptr;
}

extern "C" rbm_status rbm_far_traction(rbm_ctx* c, int n_points, int M, const double* X,
                                       const double* Nrm, const double* q, const double* add,
                                       double* y, int precision) {
  if (!c || !X || !Nrm || !q || !y) return fail(RBM_E_INVAL, "null argument");
  if (precision != 0 && precision != 1) return fail(RBM_E_INVAL, "precision must be 0 or 1");
  if (!c->ws) return fail(RBM_E_NOMEM, "bind a workspace first");
  if (n_points < 1 || M < 1) return fail(RBM_E_INVAL, "sizes must be >= 1");
  if (n_points > c->nmax * c->M) return fail(RBM_E_NOMEM, "more points than the workspace holds");
  const int nsplit = split_for(c, n_points);
  hipStream_t st = c->st;
  const size_t N3 = 3 * (size_t)n_points;
  if (precision == 0) {
    HIPCHECK(launch_pack_sources<double>(n_points, M, X, nullptr, nullptr, q, 0, nullptr, c->src, st));
    HIPCHECK(launch_far<double>(0, n_points, M, X, Nrm, c->src, c->part, nsplit, st));
  } else {
    HIPCHECK(launch_cast_f32(N3, X, c->Xf, st));
    HIPCHECK(launch_cast_f32(N3, Nrm, c->Nf, st));
    HIPCHECK(launch_pack_sources<float>(n_points, M, X, nullptr, nullptr, q, 0, nullptr, c->src, st));
    HIPCHECK(launch_far<float>(0, n_points, M, c->Xf, c->Nf, c->src, c->part, nsplit, st));
  }
  HIPCHECK(launch_combine(n_points, M, nsplit, c->part, 1.0, add, 1.0, nullptr, nullptr, 0.0, y, st));
  c->bodies_dirty = true;  // Xf/Nf were overwritten
  return RBM_OK;
}

extern "C" rbm_status rbm_far_traction_fmm(rbm_ctx* c, int n_points, int M, const double* X,
                                           const double* Nrm, const double* q, double d_max, double* y,
                                           int precision, int* level) {
  if (!c || !X || !Nrm || !q || !y) return fail(RBM_E_INVAL, "null argument");
  if (precision != 0 && precision != 1) return fail(RBM_E_INVAL, "precision must be 0 or 1");
  if (!c->ws) return fail(RBM_E_NOMEM, "bind a workspace first");
  if (c->opt.fmm_order <= 0) return fail(RBM_E_STATE, "create the context with options.fmm_order > 0");
  if (n_points < 1 || M < 1) return fail(RBM_E_INVAL, "sizes must be >= 1");
  if (n_points > c->nmax * c->M) return fail(RBM_E_NOMEM, "more points than the workspace holds");
  if (!(d_max > 0.0) || !std::isfinite(d_max)) return fail(RBM_E_INVAL, "d_max must be > 0");
  rbm_status s;
  if ((s = fmm_build(c, n_points, M, X, Nrm, d_max)) != RBM_OK) return s;
  if (!c->fmm_ready) return fail(RBM_E_INVAL, "a leaf box would hold more than 4096 points");
  if (level) *level = c->fmm_level;
  if (precision == 0)
    HIPCHECK(launch_pack_sources<double>(n_points, M, X, nullptr, nullptr, q, 0, nullptr, c->src, c->st));
  else
    HIPCHECK(launch_pack_sources<float>(n_points, M, X, nullptr, nullptr, q, 0, nullptr, c->src, c->st));
  s = fmm_apply(c, precision == 0 ? 0 : 1, y);
  c->fmm_ready = false;  // the tree belongs to these points, not to the bodies
  if (s != RBM_OK) return s;
  HIPCHECK(hipStreamSynchronize(c->st));
  return RBM_OK;
}

extern "C" rbm_status rbm_far_stokeslet(rbm_ctx* c, int n_points, int M, const double* X,
                                        const double* q, double* u, int precision) {
  if (!c || !X || !q || !u) return fail(RBM_E_INVAL, "null argument");
  if (precision != 0 && precision != 1) return fail(RBM_E_INVAL, "precision must be 0 or 1");
  if (!c->ws) return fail(RBM_E_NOMEM, "bind a workspace first");
  if (n_points < 1 || M < 1) return fail(RBM_E_INVAL, "sizes must be >= 1");
  if (n_points > c->nmax * c->M) return fail(RBM_E_NOMEM, "more points than the workspace holds");
  const int nsplit = split_for(c, n_points);
  hipStream_t st = c->st;
  const size_t N3 = 3 * (size_t)n_points;
  if (precision == 0) {
    HIPCHECK(launch_pack_sources<double>(n_points, M, X, nullptr, nullptr, q, 0, nullptr, c->src, st));
    HIPCHECK(launch_far<double>(1, n_points, M, X, nullptr, c->src, c->part, nsplit, st));
  } else {
    HIPCHECK(launch_cast_f32(N3, X, c->Xf, st));
    HIPCHECK(launch_pack_sources<float>(n_points, M, X, nullptr, nullptr, q, 0, nullptr, c->src, st));
    HIPCHECK(launch_far<float>(1, n_points, M, c->Xf, nullptr, c->src, c->part, nsplit, st));
  }
  HIPCHECK(launch_combine(n_points, M, nsplit, c->part, 1.0 / c->opt.eta, nullptr, 0.0, nullptr,
                          nullptr, 0.0, u, st));
  c->bodies_dirty = true;
  return RBM_OK;
}

extern "C" rbm_status rbm_debug_read(rbm_ctx* c, const char* name, size_t offset, size_t bytes,
                                     void* dst) {
  if (!c || !name || !dst) return fail(RBM_E_INVAL, "null argument");
  const void* p = rbm_debug_ptr(c, name);
  if (!p) return fail(RBM_E_INVAL, "unknown array name");
  HIPCHECK(hipStreamSynchronize(c->st));
  HIPCHECK(hipMemcpy(dst, (const char*)p + offset, bytes, hipMemcpyDeviceToHost));
  return RBM_OK;
}

static rbm_status refresh_nodes(rbm_ctx* c) {
  c->fmm_ready = false;
  HIPCHECK(launch_body_prep(c->n, c->quat, c->sid, c->shp, c->Rm, c->tauinv, c->area_b, c->st));
  HIPCHECK(launch_nodes(c->n, c->M, c->sid, c->cen, c->Rm, c->gr, c->gn, c->gw, c->X, c->Nn, c->W,
                        c->Xf, c->Nf, c->st));
  rbm_status s = check_overlap(c);
  if (s != RBM_OK) return s;
  return build_near(c);
}

// An RK4 stage (or the step's end) whose poses overlap: put back the poses the step
// started from, so that the context stays at a valid configuration, and return `why`
// with the overlap message.
static rbm_status restore_step_start(rbm_ctx* c, rbm_status why) {
  const std::string msg = g_err;
  const int n = c->n;
  HIPCHECK(hipMemcpyAsync(c->cen, c->cen0, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  HIPCHECK(hipMemcpyAsync(c->quat, c->quat0, 4 * n * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  HIPCHECK(launch_body_prep(n, c->quat, c->sid, c->shp, c->Rm, c->tauinv, c->area_b, c->st));
  HIPCHECK(launch_nodes(n, c->M, c->sid, c->cen, c->Rm, c->gr, c->gn, c->gw, c->X, c->Nn, c->W, c->Xf,
                        c->Nf, c->st));
  HIPCHECK(hipMemcpyAsync(c->cen_h.data(), c->cen0, 3 * n * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHECK(hipMemcpyAsync(c->quat_h.data(), c->quat0, 4 * n * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHECK(hipStreamSynchronize(c->st));
  c->fmm_ready = false;
  c->bodies_dirty = true;  // near lists are rebuilt by the next call that needs them
  return fail(why, msg + " (the step's initial poses are kept)");
}

extern "C" rbm_status rbm_step_rk4(rbm_ctx* c, double dt, const double* d_FT,
                                   rbm_solve_info* stage_info) {
  if (!c || !d_FT) return fail(RBM_E_INVAL, "null argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RBM_E_INVAL, "dt must be > 0");
  if (!c->ws) return fail(RBM_E_NOMEM, "bind a workspace first");
  if (!c->setup_done) return fail(RBM_E_STATE, "call rbm_setup first");
  if (c->n < 1) return fail(RBM_E_STATE, "set bodies first");
  rbm_status s;
  if ((s = upload_bodies(c)) != RBM_OK) return s;
  const int n = c->n;
  hipStream_t st = c->st;
  HIPCHECK(hipMemcpyAsync(c->cen0, c->cen, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHECK(hipMemcpyAsync(c->quat0, c->quat, 4 * n * sizeof(double), hipMemcpyDeviceToDevice, st));
  const double a[4] = {0.0, 0.5, 0.5, 1.0}, wgt[4] = {1.0, 2.0, 2.0, 1.0};
  rbm_status worst = RBM_OK;
  std::vector<double> FT_h;
  if (c->opt.contact_delta > 0.0) {
    FT_h.resize(6 * (size_t)n);
    HIPCHECK(hipMemcpyAsync(FT_h.data(), d_FT, FT_h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
  }
  for (int k = 0; k < 4; ++k) {
    HIPCHECK(launch_rk_stage(n, c->cen0, c->quat0, c->kst, a[k], dt, c->cen, c->quat, st));
    if ((s = refresh_nodes(c)) != RBM_OK) return s == RBM_E_OVERLAP ? restore_step_start(c, s) : s;
    c->bodies_dirty = false;
    if (c->opt.contact_delta > 0.0) {
      // stage poses to the host for the contact search, then the contact-corrected solve
      HIPCHECK(hipMemcpyAsync(c->cen_h.data(), c->cen, 3 * n * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHECK(hipMemcpyAsync(c->quat_h.data(), c->quat, 4 * n * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHECK(hipStreamSynchronize(st));
      int nf = 0;
      if ((s = rbm_find_contacts(c, c->opt.contact_delta, 0, &nf, nullptr, nullptr)) != RBM_OK) return s;
      if (nf > 0) {
        std::vector<int> cp(2 * (size_t)nf);
        std::vector<double> cx(3 * (size_t)nf), fc(3 * (size_t)nf), vw(6 * (size_t)n);
        if ((s = rbm_find_contacts(c, c->opt.contact_delta, nf, &nf, cp.data(), cx.data())) != RBM_OK) return s;
        s = rbm_solve_contacts(c, FT_h.data(), nf, cp.data(), cx.data(), vw.data(), fc.data(),
                               stage_info ? stage_info + k : nullptr);
        if (s != RBM_OK) return s;
        HIPCHECK(hipMemcpyAsync(c->VW, vw.data(), vw.size() * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHECK(launch_rk_deriv(n, c->VW, c->quat, c->kst, c->kacc, wgt[k], k == 0, st));
        HIPCHECK(hipStreamSynchronize(st));
        continue;
      }
    }
    s = solve_impl(c, d_FT, c->VW, stage_info ? stage_info + k : nullptr);
    if (s == RBM_E_NOCONV) worst = s;
    else if (s != RBM_OK) return s;
    HIPCHECK(launch_rk_deriv(n, c->VW, c->quat, c->kst, c->kacc, wgt[k], k == 0, st));
  }
  HIPCHECK(launch_rk_final(n, c->cen0, c->quat0, c->kacc, dt, c->cen, c->quat, st));
  if ((s = refresh_nodes(c)) != RBM_OK) return s == RBM_E_OVERLAP ? restore_step_start(c, s) : s;
  HIPCHECK(hipMemcpyAsync(c->cen_h.data(), c->cen, 3 * n * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipMemcpyAsync(c->quat_h.data(), c->quat, 4 * n * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  c->bodies_dirty = false;
  c->have_solution = true;
  if (worst != RBM_OK) return fail(worst, "a stage solve did not reach tol");
  return RBM_OK;
}

// RK4 step of a magnetorheological suspension (§4): at every stage the magnetostatic
// problem at the stage poses gives the Maxwell traction, which is the incident density of
// that stage's mobility solve; contacts (contact_delta > 0) correct the stage velocities
// as in rbm_step_rk4.
extern "C" rbm_status rbm_step_rk4_magnetic(rbm_ctx* c, double dt, const double* H0, double mu_ratio,
                                            double mu0, double tol_mag, rbm_solve_info* stage_info) {
  if (!c || !H0) return fail(RBM_E_INVAL, "null argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RBM_E_INVAL, "dt must be > 0");
  if (!c->opt.magnetic) return fail(RBM_E_STATE, "create the context with options.magnetic = 1");
  if (!(mu_ratio > 0.0) || !std::isfinite(mu_ratio) || !(mu0 > 0.0) || !std::isfinite(mu0) ||
      !(tol_mag > 0.0) || !all_finite(H0, 3))
    return fail(RBM_E_INVAL, "mu_ratio, mu0, tol_mag must be > 0 and H0 finite");
  if (!c->ws) return fail(RBM_E_NOMEM, "bind a workspace first");
  if (!c->setup_done) return fail(RBM_E_STATE, "call rbm_setup first");
  if (c->n < 1) return fail(RBM_E_STATE, "set bodies first");
  rbm_status s;
  if ((s = upload_bodies(c)) != RBM_OK) return s;
  const int n = c->n;
  hipStream_t st = c->st;
  HIPCHECK(hipMemcpyAsync(c->cen0, c->cen, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHECK(hipMemcpyAsync(c->quat0, c->quat, 4 * n * sizeof(double), hipMemcpyDeviceToDevice, st));
  const double a[4] = {0.0, 0.5, 0.5, 1.0}, wgt[4] = {1.0, 2.0, 2.0, 1.0};
  rbm_status worst = RBM_OK;
  for (int k = 0; k < 4; ++k) {
    HIPCHECK(launch_rk_stage(n, c->cen0, c->quat0, c->kst, a[k], dt, c->cen, c->quat, st));
    if ((s = refresh_nodes(c)) != RBM_OK) return s == RBM_E_OVERLAP ? restore_step_start(c, s) : s;
    c->bodies_dirty = false;
    int it = 0;
    if ((s = magnetic_traction_impl(c, H0, mu_ratio, mu0, tol_mag, c->mrho, nullptr, &it)) != RBM_OK) return s;
    rbm_solve_info i0;
    std::memset(&i0, 0, sizeof(i0));
    s = solve_impl(c, nullptr, c->VW, &i0, c->mrho);
    if (s == RBM_E_NOCONV) worst = s;
    else if (s != RBM_OK) return s;
    if (stage_info) stage_info[k] = i0;
    if (c->opt.contact_delta > 0.0) {
      HIPCHECK(hipMemcpyAsync(c->cen_h.data(), c->cen, 3 * n * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHECK(hipMemcpyAsync(c->quat_h.data(), c->quat, 4 * n * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHECK(hipStreamSynchronize(st));
      int nf = 0;
      if ((s = rbm_find_contacts(c, c->opt.contact_delta, 0, &nf, nullptr, nullptr)) != RBM_OK) return s;
      if (nf > 0) {
        std::vector<int> cp(2 * (size_t)nf);
        std::vector<double> cx(3 * (size_t)nf), fc(3 * (size_t)nf), vw(6 * (size_t)n), V0(6 * (size_t)n);
        if ((s = rbm_find_contacts(c, c->opt.contact_delta, nf, &nf, cp.data(), cx.data())) != RBM_OK) return s;
        HIPCHECK(hipMemcpyAsync(V0.data(), c->VW, V0.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        s = contact_correct(c, V0, i0, nf, cp.data(), cx.data(), vw.data(), fc.data(),
                            stage_info ? stage_info + k : nullptr);
        if (s != RBM_OK) return s;
        HIPCHECK(hipMemcpyAsync(c->VW, vw.data(), vw.size() * sizeof(double), hipMemcpyHostToDevice, st));
      }
    }
    HIPCHECK(launch_rk_deriv(n, c->VW, c->quat, c->kst, c->kacc, wgt[k], k == 0, st));
    HIPCHECK(hipStreamSynchronize(st));
  }
  HIPCHECK(launch_rk_final(n, c->cen0, c->quat0, c->kacc, dt, c->cen, c->quat, st));
  if ((s = refresh_nodes(c)) != RBM_OK) return s == RBM_E_OVERLAP ? restore_step_start(c, s) : s;
  HIPCHECK(hipMemcpyAsync(c->cen_h.data(), c->cen, 3 * n * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipMemcpyAsync(c->quat_h.data(), c->quat, 4 * n * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  c->bodies_dirty = false;
  c->have_solution = true;
  if (worst != RBM_OK) return fail(worst, "a stage solve did not reach tol");
  return RBM_OK;
}

extern "C" rbm_status rbm_get_bodies(rbm_ctx* c, double* centre, double* quat) {
  if (!c || !centre || !quat) return fail(RBM_E_INVAL, "null argument");
  if (c->n < 1) return fail(RBM_E_STATE, "set bodies first");
  std::memcpy(centre, c->cen_h.data(), 3 * c->n * sizeof(double));
  std::memcpy(quat, c->quat_h.data(), 4 * c->n * sizeof(double));
  return RBM_OK;
}

// ---------------------------------------------------------------------------------
// Learned warm start

#include <random>

extern "C" void rbm_learned_default_config(rbm_learned_config* cfg) {
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->k_nbr = 8;
  cfg->hidden = 256;
  cfg->n_hidden = 3;
  cfg->capacity = 65536;
  cfg->batch_max = 1024;
  cfg->seed = 1234;
}

static size_t learned_layout(rbm_ctx* c, const rbm_learned_config& cfg, char* base, bool assign) {
  auto& L = c->L;
  const int S = c->shape_kind == 1 ? (c->shape_lmax + 1) * (c->shape_lmax + 1) : 0;
  const int F = 6 + S + 15 * cfg.k_nbr, O = 3 * c->nB;
  std::vector<int> dims;
  dims.push_back(F);
  for (int h = 0; h < cfg.n_hidden; ++h) dims.push_back(cfg.hidden);
  dims.push_back(O);
  const int nl = (int)dims.size() - 1;
  std::vector<size_t> woff(nl), boff(nl);
  size_t np = 0;
  for (int l = 0; l < nl; ++l) {
    woff[l] = np;
    np += (size_t)dims[l] * dims[l + 1];
    boff[l] = np;
    np += dims[l + 1];
  }
  const int rows = std::max(cfg.batch_max, c->nmax);
  int maxw = 0;
  for (int d : dims) maxw = std::max(maxw, d);
  if (assign) {
    L.S = S; L.F = F; L.O = O; L.L = nl; L.dims = dims; L.woff = woff; L.boff = boff;
    L.nparam = np; L.rows_max = rows; L.Z.assign(nl, nullptr); L.H.assign(nl, nullptr);
    L.dZ.assign(nl, nullptr); L.Hb.assign(nl, nullptr); L.dZb.assign(nl, nullptr);
  }
  size_t off = 0;
  auto take = [&](auto*& ptr, size_t count) {
    using T = std::remove_reference_t<decltype(*ptr)>;
    off = (off + 255) & ~(size_t)255;
    if (assign) ptr = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
  };
  float *P, *G, *Mo, *Vo, *mean, *istd, *tsc, *Xbuf, *Tbuf, *Tb, *dA, *feats, *Yout;
  uint16_t *Wb, *Xb;
  int* idx;
  double *lpart, *lsum;
  take(P, np); take(G, np); take(Mo, np); take(Vo, np); take(Wb, np);
  take(mean, F); take(istd, F); take(tsc, 2);
  take(Xbuf, (size_t)cfg.capacity * F); take(Tbuf, (size_t)cfg.capacity * O);
  take(idx, cfg.capacity);
  take(Xb, (size_t)rows * F); take(Tb, (size_t)rows * O);
  take(dA, (size_t)rows * maxw); take(feats, (size_t)c->nmax * F); take(Yout, (size_t)rows * O);
  take(lpart, (size_t)rows * O / 256 + 2); take(lsum, 4);
  std::vector<float*> Z(nl), H(nl), dZ(nl);
  std::vector<uint16_t*> Hb(nl), dZb(nl);
  for (int l = 0; l < nl; ++l) {
    const size_t cnt = (size_t)rows * dims[l + 1];
    take(Z[l], cnt); take(H[l], cnt); take(dZ[l], cnt); take(Hb[l], cnt); take(dZb[l], cnt);
  }
  if (assign) {
    L.P = P; L.G = G; L.Mo = Mo; L.Vo = Vo; L.Wb = Wb; L.mean = mean; L.istd = istd; L.tsc = tsc;
    L.Xbuf = Xbuf; L.Tbuf = Tbuf; L.idx = idx; L.Xb = Xb; L.Tb = Tb; L.dA = dA; L.feats = feats;
    L.Yout = Yout; L.lpart = lpart; L.lsum = lsum; L.Z = Z; L.H = H; L.dZ = dZ; L.Hb = Hb;
    L.dZb = dZb;
  }
  return off + 256;
}

static rbm_status check_cfg(rbm_ctx* c, const rbm_learned_config* cfg) {
  if (!c || !cfg) return fail(RBM_E_INVAL, "null argument");
  if (!c->ws) return fail(RBM_E_NOMEM, "bind the solver workspace first");
  if (cfg->k_nbr < 1 || cfg->k_nbr > 16) return fail(RBM_E_INVAL, "k_nbr in [1, 16]");
  if (cfg->hidden < 1 || cfg->hidden > 4096) return fail(RBM_E_INVAL, "hidden in [1, 4096]");
  if (cfg->n_hidden < 1 || cfg->n_hidden > 6) return fail(RBM_E_INVAL, "n_hidden in [1, 6]");
  if (cfg->capacity < 1 || cfg->batch_max < 1) return fail(RBM_E_INVAL, "capacity, batch_max >= 1");
  return RBM_OK;
}

extern "C" rbm_status rbm_learned_workspace_size(rbm_ctx* c, const rbm_learned_config* cfg,
                                                 size_t* bytes) {
  rbm_status s = check_cfg(c, cfg);
  if (s != RBM_OK) return s;
  if (!bytes) return fail(RBM_E_INVAL, "null argument");
  *bytes = learned_layout(c, *cfg, nullptr, false);
  return RBM_OK;
}

extern "C" rbm_status rbm_learned_bind(rbm_ctx* c, const rbm_learned_config* cfg, void* dptr,
                                       size_t bytes) {
  rbm_status s = check_cfg(c, cfg);
  if (s != RBM_OK) return s;
  if (!dptr || ((uintptr_t)dptr & 255)) return fail(RBM_E_INVAL, "workspace must be 256-byte aligned");
  if (learned_layout(c, *cfg, nullptr, false) > bytes) return fail(RBM_E_NOMEM, "learned workspace too small");
  learned_layout(c, *cfg, (char*)dptr, true);
  auto& L = c->L;
  L.cfg = *cfg;
  L.bound = true;
  L.stats_ready = false;
  L.count = 0;
  L.head = 0;
  L.t = 0;
  L.epoch = 0;
  // weights ~ N(0, 1/fan_in) (last layer 0.1/fan_in), biases 0
  std::vector<float> P(L.nparam, 0.f);
  std::mt19937_64 rng(cfg->seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (int l = 0; l < L.L; ++l) {
    const double sd = (l == L.L - 1 ? 0.1 : 1.0) / std::sqrt((double)L.dims[l]);
    for (size_t i = 0; i < (size_t)L.dims[l] * L.dims[l + 1]; ++i) P[L.woff[l] + i] = (float)(sd * nd(rng));
  }
  HIPCHECK(hipMemcpyAsync(L.P, P.data(), P.size() * sizeof(float), hipMemcpyHostToDevice, c->st));
  HIPCHECK(hipMemsetAsync(L.Mo, 0, L.nparam * sizeof(float), c->st));
  HIPCHECK(hipMemsetAsync(L.Vo, 0, L.nparam * sizeof(float), c->st));
  HIPCHECK(launch_to_bf16(L.nparam, L.P, L.Wb, c->st));
  std::vector<float> ms(2 * L.F + 2, 0.f);
  for (int f = 0; f < L.F; ++f) ms[L.F + f] = 1.f;
  ms[2 * L.F] = 1.f;
  ms[2 * L.F + 1] = 1.f;
  HIPCHECK(hipMemcpyAsync(L.mean, ms.data(), L.F * sizeof(float), hipMemcpyHostToDevice, c->st));
  HIPCHECK(hipMemcpyAsync(L.istd, ms.data() + L.F, L.F * sizeof(float), hipMemcpyHostToDevice, c->st));
  HIPCHECK(hipMemcpyAsync(L.tsc, ms.data() + 2 * L.F, 2 * sizeof(float), hipMemcpyHostToDevice, c->st));
  HIPCHECK(hipStreamSynchronize(c->st));
  return RBM_OK;
}

// Forward pass on `rows` rows of L.Xb (bf16, standardized); output in L.Z[last].
static rbm_status mlp_forward(rbm_ctx* c, int rows) {
  auto& L = c->L;
  const uint16_t* A = L.Xb;
  for (int l = 0; l < L.L; ++l) {
    const int in = L.dims[l], out = L.dims[l + 1];
    HIPCHECK(launch_gemm_bf16(rows, out, in, A, in, 1, L.Wb + L.woff[l], out, 1, L.Z[l], out,
                              L.P + L.boff[l], 1.f, 0.f, c->st));
    if (l < L.L - 1) {
      HIPCHECK(launch_silu_fwd((size_t)rows * out, L.Z[l], L.H[l], L.Hb[l], c->st));
      A = L.Hb[l];
    }
  }
  return RBM_OK;
}

// Loss against L.Tb (scaled targets) and gradients into L.G; loss value in L.lsum[0], and
// added to the running sum L.lsum[1] when accumulate is set.
static rbm_status mlp_backward(rbm_ctx* c, int rows, int accumulate = 0) {
  auto& L = c->L;
  const int last = L.L - 1, O = L.dims[last + 1];
  const size_t cnt = (size_t)rows * O;
  const int nparts = (int)((cnt + 255) / 256);
  HIPCHECK(launch_mse(cnt, 1.f / (float)cnt, L.Z[last], L.Tb, L.dZ[last], L.dZb[last], L.lpart, c->st));
  HIPCHECK(launch_sum_parts(nparts, L.lpart, 1.0 / (double)cnt, L.lsum, accumulate, c->st));
  for (int l = last; l >= 0; --l) {
    const int in = L.dims[l], out = L.dims[l + 1];
    const uint16_t* Aprev = l == 0 ? L.Xb : L.Hb[l - 1];
    // dW = Aprev^T dZ (in x out), db = colsum(dZ)
    HIPCHECK(launch_gemm_bf16(in, out, rows, Aprev, 1, in, L.dZb[l], out, 1, L.G + L.woff[l], out,
                              nullptr, 1.f, 0.f, c->st));
    HIPCHECK(launch_colsum(rows, out, L.dZ[l], L.G + L.boff[l], c->st));
    if (l > 0) {
      // dA = dZ W^T (rows x in), then dZ_{l-1} = dA * silu'(Z_{l-1})
      HIPCHECK(launch_gemm_bf16(rows, in, out, L.dZb[l], out, 1, L.Wb + L.woff[l], 1, out, L.dA, in,
                                nullptr, 1.f, 0.f, c->st));
      HIPCHECK(launch_silu_bwd((size_t)rows * in, L.dA, L.Z[l - 1], L.dZ[l - 1], L.dZb[l - 1], c->st));
    }
  }
  return RBM_OK;
}

static rbm_status learned_correction(rbm_ctx* c, const double* dFT) {
  auto& L = c->L;
  const int n = c->n;
  if (n > L.rows_max) return fail(RBM_E_NOMEM, "more bodies than the learned workspace holds");
  const double* desc = L.S > 0 ? c->rcbuf : nullptr;
  HIPCHECK(launch_features(n, L.cfg.k_nbr, L.S, c->cen, c->Rm, dFT, c->sid, desc, L.feats, c->st));
  HIPCHECK(launch_gather(n, L.F, L.O, nullptr, L.feats, L.mean, L.istd, L.Xb, nullptr, 1.f, nullptr, c->st));
  rbm_status s;
  if ((s = mlp_forward(c, n)) != RBM_OK) return s;
  HIPCHECK(launch_band_synth(n, c->M, c->p, L.Z[L.L - 1], L.tsc, c->Ytab, c->Rm, c->mu, c->st));
  return RBM_OK;
}

static rbm_status learned_capture(rbm_ctx* c, const double* dFT) {
  auto& L = c->L;
  const int n = c->n, M = c->M, N = n * M;
  const size_t len = 3 * (size_t)N;
  // ring buffer: once full, the newest states overwrite the oldest rows
  if (n > L.cfg.capacity) return RBM_OK;
  if (L.head + n > L.cfg.capacity) L.head = 0;
  const double* desc = L.S > 0 ? c->rcbuf : nullptr;
  HIPCHECK(launch_features(n, L.cfg.k_nbr, L.S, c->cen, c->Rm, dFT, c->sid, desc,
                           L.Xbuf + (size_t)L.head * L.F, c->st));
  // target: body-frame band coefficients of mu - mu_BD, mu_BD = P^{-1} b in float64
  HIPCHECK(launch_self_apply<double>(n, M, c->sid, c->P0, c->Rm, c->b, c->yb, c->st));
  HIPCHECK(launch_combine(N, M, 0, nullptr, 0.0, c->mu, 1.0, c->yb, c->Rm, -1.0, c->t1, c->st));
  HIPCHECK(launch_band_analysis(n, M, c->p, c->t1, c->Rm, c->Ftab, L.Tbuf + (size_t)L.head * L.O, c->st));
  HIPCHECK(hipStreamSynchronize(c->st));
  (void)len;
  L.head += n;
  L.count = std::max(L.count, L.head);
  return RBM_OK;
}

extern "C" rbm_status rbm_learned_capture(rbm_ctx* c, const double* d_FT) {
  if (!c || !d_FT) return fail(RBM_E_INVAL, "null argument");
  if (!c->L.bound) return fail(RBM_E_STATE, "bind the learned workspace first");
  if (!c->have_solution) return fail(RBM_E_STATE, "no solve to capture");
  return learned_capture(c, d_FT);
}

extern "C" rbm_status rbm_learned_set_capture(rbm_ctx* c, int on) {
  if (!c) return fail(RBM_E_INVAL, "null argument");
  if (!c->L.bound) return fail(RBM_E_STATE, "bind the learned workspace first");
  c->L.capture_on = on != 0;
  return RBM_OK;
}

extern "C" rbm_status rbm_learned_train(rbm_ctx* c, int epochs, int batch, double lr, double* loss) {
  if (!c) return fail(RBM_E_INVAL, "null argument");
  auto& L = c->L;
  if (!L.bound) return fail(RBM_E_STATE, "bind the learned workspace first");
  if (L.count < 1) return fail(RBM_E_STATE, "no captured samples");
  if (epochs < 0 || batch < 1 || batch > L.rows_max || !(lr > 0.0))
    return fail(RBM_E_INVAL, "bad training arguments");
  hipStream_t st = c->st;
  if (!L.stats_ready) {
    HIPCHECK(launch_colstats(L.count, L.F, L.Xbuf, L.mean, L.istd, st));
    HIPCHECK(launch_rms((size_t)L.count * L.O, L.Tbuf, L.tsc, st));
    L.stats_ready = true;
  }
  float tsc[2];
  HIPCHECK(hipMemcpyAsync(tsc, L.tsc, 2 * sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  std::vector<int> perm(L.count);
  double last = 0.0;
  for (int e = 0; e < epochs; ++e) {
    std::mt19937_64 rng(L.cfg.seed * 1000003ULL + (unsigned long long)(++L.epoch));
    for (int i = 0; i < L.count; ++i) perm[i] = i;
    std::shuffle(perm.begin(), perm.end(), rng);
    HIPCHECK(hipMemcpyAsync(L.idx, perm.data(), L.count * sizeof(int), hipMemcpyHostToDevice, st));
    // the batch losses are summed on the device (lsum[1]) and read once per epoch
    HIPCHECK(hipMemsetAsync(L.lsum + 1, 0, sizeof(double), st));
    int nb = 0;
    for (int off = 0; off < L.count; off += batch) {
      const int rows = std::min(batch, L.count - off);
      HIPCHECK(launch_gather(rows, L.F, L.O, L.idx + off, L.Xbuf, L.mean, L.istd, L.Xb, L.Tbuf,
                             tsc[1], L.Tb, st));
      rbm_status s;
      if ((s = mlp_forward(c, rows)) != RBM_OK) return s;
      if ((s = mlp_backward(c, rows, 1)) != RBM_OK) return s;
      HIPCHECK(launch_adam(L.nparam, L.P, L.G, L.Mo, L.Vo, (float)lr, 0.9f, 0.999f, 1e-8f, ++L.t,
                           L.Wb, st));
      ++nb;
    }
    double acc;
    rbm_status s;
    if ((s = read_scalar(c, L.lsum + 1, &acc)) != RBM_OK) return s;
    last = acc / nb;
  }
  HIPCHECK(hipStreamSynchronize(st));
  if (loss) *loss = last;
  return RBM_OK;
}

extern "C" rbm_status rbm_learned_info(rbm_ctx* c, int* samples, int* n_features, int* n_outputs,
                                       int* n_params) {
  if (!c) return fail(RBM_E_INVAL, "null argument");
  if (!c->L.bound) return fail(RBM_E_STATE, "bind the learned workspace first");
  if (samples) *samples = c->L.count;
  if (n_features) *n_features = c->L.F;
  if (n_outputs) *n_outputs = c->L.O;
  if (n_params) *n_params = (int)c->L.nparam;
  return RBM_OK;
}

extern "C" rbm_status rbm_learned_get_params(rbm_ctx* c, float* host, size_t count) {
  if (!c || !host) return fail(RBM_E_INVAL, "null argument");
  auto& L = c->L;
  if (!L.bound) return fail(RBM_E_STATE, "bind the learned workspace first");
  if (count != L.nparam + 2 * L.F + 2) return fail(RBM_E_INVAL, "count must be n_params + 2F + 2");
  HIPCHECK(hipStreamSynchronize(c->st));
  HIPCHECK(hipMemcpy(host, L.P, L.nparam * sizeof(float), hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(host + L.nparam, L.mean, L.F * sizeof(float), hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(host + L.nparam + L.F, L.istd, L.F * sizeof(float), hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(host + L.nparam + 2 * L.F, L.tsc, 2 * sizeof(float), hipMemcpyDeviceToHost));
  return RBM_OK;
}

extern "C" rbm_status rbm_learned_set_params(rbm_ctx* c, const float* host, size_t count) {
  if (!c || !host) return fail(RBM_E_INVAL, "null argument");
  auto& L = c->L;
  if (!L.bound) return fail(RBM_E_STATE, "bind the learned workspace first");
  if (count != L.nparam + 2 * L.F + 2) return fail(RBM_E_INVAL, "count must be n_params + 2F + 2");
  for (size_t i = 0; i < count; ++i)
    if (!std::isfinite(host[i])) return fail(RBM_E_INVAL, "non-finite parameter");
  HIPCHECK(hipMemcpy(L.P, host, L.nparam * sizeof(float), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L.mean, host + L.nparam, L.F * sizeof(float), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L.istd, host + L.nparam + L.F, L.F * sizeof(float), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(L.tsc, host + L.nparam + 2 * L.F, 2 * sizeof(float), hipMemcpyHostToDevice));
  HIPCHECK(launch_to_bf16(L.nparam, L.P, L.Wb, c->st));
  HIPCHECK(hipStreamSynchronize(c->st));
  L.stats_ready = true;
  return RBM_OK;
}

extern "C" rbm_status rbm_learned_forward_dev(rbm_ctx* c, const float* d_X, int rows, float* d_Y) {
  if (!c || !d_X || !d_Y) return fail(RBM_E_INVAL, "null argument");
  auto& L = c->L;
  if (!L.bound) return fail(RBM_E_STATE, "bind the learned workspace first");
  if (rows < 1 || rows > L.rows_max) return fail(RBM_E_INVAL, "rows out of range");
  HIPCHECK(launch_gather(rows, L.F, L.O, nullptr, d_X, L.mean, L.istd, L.Xb, nullptr, 1.f, nullptr, c->st));
  rbm_status s;
  if ((s = mlp_forward(c, rows)) != RBM_OK) return s;
  HIPCHECK(hipMemcpyAsync(d_Y, L.Z[L.L - 1], (size_t)rows * L.O * sizeof(float),
                          hipMemcpyDeviceToDevice, c->st));
  HIPCHECK(hipStreamSynchronize(c->st));
  return RBM_OK;
}

extern "C" rbm_status rbm_learned_loss_grad_dev(rbm_ctx* c, const float* d_X, const float* d_T,
                                                int rows, float* d_grad, double* loss) {
  if (!c || !d_X || !d_T || !d_grad) return fail(RBM_E_INVAL, "null argument");
  auto& L = c->L;
  if (!L.bound) return fail(RBM_E_STATE, "bind the learned workspace first");
  if (rows < 1 || rows > L.rows_max) return fail(RBM_E_INVAL, "rows out of range");
  float tsc[2];
  HIPCHECK(hipMemcpyAsync(tsc, L.tsc, 2 * sizeof(float), hipMemcpyDeviceToHost, c->st));
  HIPCHECK(hipStreamSynchronize(c->st));
  HIPCHECK(launch_gather(rows, L.F, L.O, nullptr, d_X, L.mean, L.istd, L.Xb, d_T, tsc[1], L.Tb, c->st));
  rbm_status s;
  if ((s = mlp_forward(c, rows)) != RBM_OK) return s;
  if ((s = mlp_backward(c, rows)) != RBM_OK) return s;
  HIPCHECK(hipMemcpyAsync(d_grad, L.G, L.nparam * sizeof(float), hipMemcpyDeviceToDevice, c->st));
  double lv;
  if ((s = read_scalar(c, L.lsum, &lv)) != RBM_OK) return s;
  if (loss) *loss = lv;
  return RBM_OK;
}

extern "C" rbm_status rbm_learned_features_dev(rbm_ctx* c, const double* d_FT, float* d_X) {
  if (!c || !d_FT || !d_X) return fail(RBM_E_INVAL, "null argument");
  auto& L = c->L;
  if (!L.bound) return fail(RBM_E_STATE, "bind the learned workspace first");
  rbm_status s;
  if ((s = upload_bodies(c)) != RBM_OK) return s;
  const double* desc = L.S > 0 ? c->rcbuf : nullptr;
  HIPCHECK(launch_features(c->n, L.cfg.k_nbr, L.S, c->cen, c->Rm, d_FT, c->sid, desc, d_X, c->st));
  HIPCHECK(hipStreamSynchronize(c->st));
  return RBM_OK;
}

extern "C" rbm_status rbm_learned_guess_dev(rbm_ctx* c, const double* d_FT, double* d_mu0) {
  if (!c || !d_FT || !d_mu0) return fail(RBM_E_INVAL, "null argument");
  if (!c->L.bound) return fail(RBM_E_STATE, "bind the learned workspace first");
  if (!c->setup_done) return fail(RBM_E_STATE, "call rbm_setup first");
  rbm_status s;
  if ((s = upload_bodies(c)) != RBM_OK) return s;
  const int N = c->n * c->M;
  SolveState S;
  c->ev_used = 0;
  double bnorm;
  if ((s = build_rhs(c, S, d_FT, nullptr, &bnorm)) != RBM_OK) return s;
  if ((s = self_apply(c, S, 1, 0, c->b, c->yb)) != RBM_OK) return s;
  HIPCHECK(launch_combine(N, c->M, 0, nullptr, 0.0, nullptr, 0.0, c->yb, c->Rm, 1.0, c->mu, c->st));
  if ((s = learned_correction(c, d_FT)) != RBM_OK) return s;
  HIPCHECK(hipMemcpyAsync(d_mu0, c->mu, 3 * (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  HIPCHECK(hipStreamSynchronize(c->st));
  c->have_solution = false;
  return RBM_OK;
}

extern "C" rbm_status rbm_set_guess(rbm_ctx* c, int guess) {
  if (!c) return fail(RBM_E_INVAL, "null argument");
  if (guess < 0 || guess > 3) return fail(RBM_E_INVAL, "bad guess");
  c->opt.guess = guess;
  return RBM_OK;
}

// ---------------------------------------------------------------------------------
// Mobility matrix (§1: V = M F) by unit-load solves

extern "C" rbm_status rbm_mobility_matrix(rbm_ctx* c, double* Mmat, rbm_solve_info* info) {
  if (!c || !Mmat) return fail(RBM_E_INVAL, "null argument");
  if (!c->ws) return fail(RBM_E_NOMEM, "bind a workspace first");
  if (!c->setup_done) return fail(RBM_E_STATE, "call rbm_setup first");
  if (c->n < 1) return fail(RBM_E_STATE, "set bodies first");
  const int m = 6 * c->n;
  const int guess = c->opt.guess;
  const bool capture = c->L.capture_on;
  // unit loads get the block-diagonal guess and are not captured as training data
  if (guess == RBM_GUESS_LEARNED || guess == RBM_GUESS_USER) c->opt.guess = RBM_GUESS_BLOCKDIAG;
  c->L.capture_on = false;
  std::vector<double> load(m, 0.0), vw(m);
  rbm_solve_info tot, ik;
  std::memset(&tot, 0, sizeof(tot));
  rbm_status s = RBM_OK, worst = RBM_OK;
  for (int k = 0; k < m && (s == RBM_OK || s == RBM_E_NOCONV); ++k) {
    load[k] = 1.0;
    s = rbm_solve(c, load.data(), vw.data(), &ik);
    load[k] = 0.0;
    if (s == RBM_E_NOCONV) worst = s;
    if (s != RBM_OK && s != RBM_E_NOCONV) break;
    for (int r = 0; r < m; ++r) Mmat[(size_t)r * m + k] = vw[r];
    tot.iters += ik.iters;
    tot.matvecs += ik.matvecs;
    tot.cycles += ik.cycles;
    tot.refinements += ik.refinements;
    tot.ms_total += ik.ms_total;
    tot.ms_far += ik.ms_far;
    tot.ms_self += ik.ms_self;
    tot.far_pairs += ik.far_pairs;
    tot.rel_residual = std::max(tot.rel_residual, ik.rel_residual);
  }
  c->opt.guess = guess;
  c->L.capture_on = capture;
  if (info) *info = tot;
  if (s != RBM_OK && s != RBM_E_NOCONV) return s;
  if (worst != RBM_OK) return fail(worst, "a unit-load solve did not reach tol");
  return RBM_OK;
}

// ---------------------------------------------------------------------------------
// Run state (Algorithm 1's loop: poses, densities, learned warm start)

namespace {

constexpr char kStateMagic[8] = {'R', 'B', 'M', 'S', 'T', 'A', 'T', '1'};

struct StateHeader {
  char magic[8];
  uint64_t bytes;        // whole record
  uint64_t shape_hash;   // FNV-1a of the shape input (kind, lmax, coefficients)
  int32_t p, M, ns, n;
  int32_t guess, have_solution, learned, pad0;
  double bd_ratio;
  // learned warm start (zeros when learned == 0)
  int32_t F, O, capacity, count, head, t, epoch, stats_ready, capture_on, pad1;
  uint64_t nparam;
};

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ULL;
  }
  return h;
}

uint64_t shape_hash(const rbm_ctx* c) {
  uint64_t h = 1469598103934665603ULL;
  h = fnv1a(h, &c->shape_kind, sizeof(c->shape_kind));
  h = fnv1a(h, &c->shape_lmax, sizeof(c->shape_lmax));
  return fnv1a(h, c->shape_data.data(), c->shape_data.size() * sizeof(double));
}

// Byte count of the record for the context's current contents.
size_t state_bytes(const rbm_ctx* c, const StateHeader& h) {
  const size_t N = (size_t)h.n * h.M;
  size_t b = sizeof(StateHeader) + (size_t)h.n * (sizeof(int32_t) + 7 * sizeof(double));
  if (h.have_solution) b += 6 * N * sizeof(double);
  if (h.learned)
    b += (3 * h.nparam + 2 * (size_t)h.F + 2 + (size_t)h.count * ((size_t)h.F + (size_t)h.O)) * sizeof(float);
  (void)c;
  return b;
}

}  // namespace

extern "C" rbm_status rbm_get_state(rbm_ctx* c, void* buf, size_t* bytes) {
  if (!c || !bytes) return fail(RBM_E_INVAL, "null argument");
  if (!c->ws || !c->setup_done) return fail(RBM_E_STATE, "call rbm_setup first");
  if (c->n < 1) return fail(RBM_E_STATE, "set bodies first");
  StateHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kStateMagic, 8);
  h.shape_hash = shape_hash(c);
  h.p = c->p;
  h.M = c->M;
  h.ns = c->ns;
  h.n = c->n;
  h.guess = c->opt.guess;
  h.have_solution = c->have_solution ? 1 : 0;
  h.learned = c->L.bound ? 1 : 0;
  h.bd_ratio = c->bd_ratio;
  const auto& L = c->L;
  if (L.bound) {
    h.F = L.F;
    h.O = L.O;
    h.capacity = L.cfg.capacity;
    h.count = L.count;
    h.head = L.head;
    h.t = L.t;
    h.epoch = L.epoch;
    h.stats_ready = L.stats_ready ? 1 : 0;
    h.capture_on = L.capture_on ? 1 : 0;
    h.nparam = L.nparam;
  }
  h.bytes = state_bytes(c, h);
  if (!buf) {
    *bytes = h.bytes;
    return RBM_OK;
  }
  if (*bytes < h.bytes) return fail(RBM_E_INVAL, "state buffer too small (query the size with buf = NULL)");
  *bytes = h.bytes;
  char* o = static_cast<char*>(buf);
  auto put = [&](const void* src, size_t nb) {
    std::memcpy(o, src, nb);
    o += nb;
  };
  auto put_dev = [&](const void* dsrc, size_t nb) -> hipError_t {
    hipError_t e = hipMemcpy(o, dsrc, nb, hipMemcpyDeviceToHost);
    o += nb;
    return e;
  };
  HIPCHECK(hipStreamSynchronize(c->st));
  const int n = c->n;
  const size_t N = (size_t)n * c->M;
  put(&h, sizeof(h));
  std::vector<int32_t> sid(c->sid_h.begin(), c->sid_h.end());
  put(sid.data(), n * sizeof(int32_t));
  put(c->cen_h.data(), 3 * n * sizeof(double));
  put(c->quat_h.data(), 4 * n * sizeof(double));
  if (h.have_solution) {
    HIPCHECK(put_dev(c->mu, 3 * N * sizeof(double)));
    HIPCHECK(put_dev(c->rho, 3 * N * sizeof(double)));
  }
  if (h.learned) {
    HIPCHECK(put_dev(L.P, L.nparam * sizeof(float)));
    HIPCHECK(put_dev(L.Mo, L.nparam * sizeof(float)));
    HIPCHECK(put_dev(L.Vo, L.nparam * sizeof(float)));
    HIPCHECK(put_dev(L.mean, L.F * sizeof(float)));
    HIPCHECK(put_dev(L.istd, L.F * sizeof(float)));
    HIPCHECK(put_dev(L.tsc, 2 * sizeof(float)));
    HIPCHECK(put_dev(L.Xbuf, (size_t)L.count * L.F * sizeof(float)));
    HIPCHECK(put_dev(L.Tbuf, (size_t)L.count * L.O * sizeof(float)));
  }
  return RBM_OK;
}

extern "C" rbm_status rbm_set_state(rbm_ctx* c, const void* buf, size_t bytes) {
  if (!c || !buf) return fail(RBM_E_INVAL, "null argument");
  if (!c->ws || !c->setup_done) return fail(RBM_E_STATE, "call rbm_setup first");
  if (bytes < sizeof(StateHeader)) return fail(RBM_E_INVAL, "state record too short");
  StateHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, kStateMagic, 8) != 0) return fail(RBM_E_INVAL, "not a state record");
  // every field the record's size depends on is checked before the size is computed
  if (h.p != c->p || h.M != c->M || h.ns != c->ns || h.shape_hash != shape_hash(c))
    return fail(RBM_E_INVAL, "state record belongs to other shapes or another order p");
  if (h.n < 1) return fail(RBM_E_INVAL, "bad body count in the state record");
  if (h.n > c->nmax) return fail(RBM_E_NOMEM, "more bodies than the workspace holds");
  if (h.guess < 0 || h.guess > 3) return fail(RBM_E_INVAL, "bad guess mode in the state record");
  if ((h.have_solution != 0 && h.have_solution != 1) || (h.learned != 0 && h.learned != 1))
    return fail(RBM_E_INVAL, "bad flags in the state record");
  auto& L = c->L;
  if (h.learned) {
    if (!L.bound) return fail(RBM_E_STATE, "the record has a learned warm start: bind the learned workspace first");
    if (h.F != L.F || h.O != L.O || h.nparam != L.nparam || h.capacity != L.cfg.capacity)
      return fail(RBM_E_INVAL, "learned configuration of the record differs from the bound one");
    if (h.count < 0 || h.count > h.capacity || h.head < 0 || h.head > h.capacity)
      return fail(RBM_E_INVAL, "bad sample counts in the state record");
  }
  if (h.bytes != bytes || state_bytes(c, h) != bytes) return fail(RBM_E_INVAL, "state record size mismatch");
  const char* in = static_cast<const char*>(buf) + sizeof(h);
  const int n = h.n;
  const size_t N = (size_t)n * c->M;
  std::vector<int32_t> sid(n);
  std::memcpy(sid.data(), in, n * sizeof(int32_t));
  in += n * sizeof(int32_t);
  for (int i = 0; i < n; ++i)
    if (sid[i] < 0 || sid[i] >= c->ns) return fail(RBM_E_INVAL, "unknown shape id in the state record");
  std::vector<double> cen(3 * (size_t)n), quat(4 * (size_t)n);
  std::memcpy(cen.data(), in, cen.size() * sizeof(double));
  in += cen.size() * sizeof(double);
  std::memcpy(quat.data(), in, quat.size() * sizeof(double));
  in += quat.size() * sizeof(double);
  if (!all_finite(cen.data(), cen.size()) || !all_finite(quat.data(), quat.size()))
    return fail(RBM_E_INVAL, "non-finite pose in the state record");
  hipStream_t st = c->st;
  HIPCHECK(hipStreamSynchronize(st));
  c->n = n;
  c->sid_h.assign(sid.begin(), sid.end());
  c->cen_h = cen;
  c->quat_h = quat;
  c->bodies_dirty = true;
  c->fmm_ready = false;
  c->opt.guess = h.guess;
  c->bd_ratio = h.bd_ratio;
  if (h.have_solution) {
    HIPCHECK(hipMemcpy(c->mu, in, 3 * N * sizeof(double), hipMemcpyHostToDevice));
    in += 3 * N * sizeof(double);
    HIPCHECK(hipMemcpy(c->rho, in, 3 * N * sizeof(double), hipMemcpyHostToDevice));
    in += 3 * N * sizeof(double);
  }
  c->have_solution = h.have_solution != 0;
  if (h.learned) {
    auto get = [&](void* ddst, size_t nb) -> hipError_t {
      hipError_t e = hipMemcpy(ddst, in, nb, hipMemcpyHostToDevice);
      in += nb;
      return e;
    };
    HIPCHECK(get(L.P, L.nparam * sizeof(float)));
    HIPCHECK(get(L.Mo, L.nparam * sizeof(float)));
    HIPCHECK(get(L.Vo, L.nparam * sizeof(float)));
    HIPCHECK(get(L.mean, L.F * sizeof(float)));
    HIPCHECK(get(L.istd, L.F * sizeof(float)));
    HIPCHECK(get(L.tsc, 2 * sizeof(float)));
    HIPCHECK(get(L.Xbuf, (size_t)h.count * L.F * sizeof(float)));
    HIPCHECK(get(L.Tbuf, (size_t)h.count * L.O * sizeof(float)));
    HIPCHECK(launch_to_bf16(L.nparam, L.P, L.Wb, st));
    HIPCHECK(hipStreamSynchronize(st));
    L.count = h.count;
    L.head = h.head;
    L.t = h.t;
    L.epoch = h.epoch;
    L.stats_ready = h.stats_ready != 0;
    L.capture_on = h.capture_on != 0;
  }
  return RBM_OK;
}
