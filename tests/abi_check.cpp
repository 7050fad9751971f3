// Host-side check of the C ABI in include/rbm.h, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code of the library (rbm_api.cpp, rbm_static.cpp)
// and of this program; the kernels are the ordinary gfx950 code objects.  It walks every
// family of calls once on small inputs, including the error paths whose host logic parses
// caller data (argument validation, run-state records that are truncated or of another
// context, overlapping poses), and exits 0 when every expectation holds.  A sanitizer
// report ends the run with a non-zero status.
//
//   usage: abi_check            (needs a GPU)
//          abi_check --host     (calls that fail before any device work; no GPU needed)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "rbm.h"

extern "C" const char* __asan_default_options() { return "detect_leaks=0"; }

static int g_fail = 0;

#define EXPECT(cond, what)                                                         \
  do {                                                                             \
    if (!(cond)) {                                                                 \
      std::printf("abi_check: FAILED %s (%s:%d) last error: %s\n", what, __FILE__, \
                  __LINE__, rbm_last_error());                                     \
      ++g_fail;                                                                    \
    }                                                                              \
  } while (0)

#define STEP(msg) std::printf("abi_check: %s\n", msg), std::fflush(stdout)

static const double kY00 = 3.5449077018110318;  // sqrt(4 pi): r = 1 for a unit sphere

// Calls that return before any device work: option validation and null arguments.
static void host_checks() {
  STEP("host: option validation");
  rbm_options o;
  rbm_default_options(&o);
  rbm_ctx* c = nullptr;
  rbm_options bad = o;
  bad.p = 1;
  EXPECT(rbm_create(&bad, &c) == RBM_E_INVAL && c == nullptr, "p = 1 refused");
  bad = o;
  bad.p = 21;
  EXPECT(rbm_create(&bad, &c) == RBM_E_INVAL, "p = 21 refused");
  bad = o;
  bad.eta = -1.0;
  EXPECT(rbm_create(&bad, &c) == RBM_E_INVAL, "eta < 0 refused");
  bad = o;
  bad.tol = std::nan("");
  EXPECT(rbm_create(&bad, &c) == RBM_E_INVAL, "NaN tol refused");
  bad = o;
  bad.max_iter = 0;
  EXPECT(rbm_create(&bad, &c) == RBM_E_INVAL, "max_iter 0 refused");
  bad = o;
  bad.fmm_order = 17;
  EXPECT(rbm_create(&bad, &c) == RBM_E_INVAL, "fmm order 17 refused");
  bad = o;
  bad.p_up = o.p;
  EXPECT(rbm_create(&bad, &c) == RBM_E_INVAL, "p_up = p refused");
  EXPECT(rbm_create(nullptr, &c) == RBM_E_INVAL, "null options refused");
  EXPECT(rbm_create(&o, nullptr) == RBM_E_INVAL, "null out refused");
  rbm_destroy(nullptr);

  STEP("host: calls on a context without shapes");
  EXPECT(rbm_create(&o, &c) == RBM_OK && c != nullptr, "create");
  if (!c) return;
  double rc[4] = {kY00, 0, 0, 0};
  EXPECT(rbm_set_shapes_radial(c, 0, 0, rc) == RBM_E_INVAL, "zero shapes refused");
  EXPECT(rbm_set_shapes_radial(c, 1, o.p - 1, rc) == RBM_E_INVAL, "radial lmax > p-2 refused");
  EXPECT(rbm_set_shapes_radial(c, 1, 0, nullptr) == RBM_E_INVAL, "null coefficients refused");
  size_t bytes = 0;
  EXPECT(rbm_workspace_size(c, 4, &bytes) != RBM_OK, "workspace size before shapes refused");
  EXPECT(rbm_setup(c) != RBM_OK, "setup before shapes refused");
  double FT[6] = {1, 0, 0, 0, 0, 0}, VW[6];
  EXPECT(rbm_solve(c, FT, VW, nullptr) != RBM_OK, "solve before setup refused");
  EXPECT(rbm_set_state(c, nullptr, 0) == RBM_E_INVAL, "null state record refused");
  unsigned char junk[64];
  std::memset(junk, 0x5a, sizeof junk);
  EXPECT(rbm_set_state(c, junk, sizeof junk) != RBM_OK, "junk state record refused");
  // low-level sums: argument checks come before the workspace check, and without a
  // workspace the call stops there (the pointers below are never dereferenced)
  const double* h = FT;
  double* o6 = VW;
  EXPECT(rbm_far_traction(c, 2, 1, h, h, nullptr, nullptr, o6, 0) == RBM_E_INVAL, "null strengths refused");
  EXPECT(rbm_far_traction(c, 2, 1, h, h, h, nullptr, o6, 2) == RBM_E_INVAL, "sum precision 2 refused");
  EXPECT(rbm_far_stokeslet(c, 2, 1, h, h, o6, -1) == RBM_E_INVAL, "Stokeslet precision -1 refused");
  EXPECT(rbm_far_traction(c, 2, 1, h, h, h, nullptr, o6, 0) == RBM_E_NOMEM, "sum before a workspace refused");
  EXPECT(rbm_far_stokeslet(c, 2, 1, h, h, o6, 1) == RBM_E_NOMEM, "Stokeslet before a workspace refused");
  EXPECT(std::strlen(rbm_last_error()) > 0, "error message set");
  rbm_destroy(c);
}

struct Dev {
  void* p = nullptr;
  explicit Dev(size_t bytes) {
    if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
  }
  ~Dev() {
    if (p) (void)hipFree(p);
  }
};

// Three unit spheres (and a perturbed second shape), p = 6: setup, solve, mobility matrix,
// run state, RK4, overlap, learned warm start, low-level sums.
static void device_checks() {
  STEP("device: context, shapes, workspace, setup");
  rbm_options o;
  rbm_default_options(&o);
  o.p = 6;
  o.tol = 1e-10;
  rbm_ctx* c = nullptr;
  EXPECT(rbm_create(&o, &c) == RBM_OK, "create");
  if (!c) return;
  const int L = 2, nc = (L + 1) * (L + 1);
  std::vector<double> rc(2 * nc, 0.0);
  rc[0] = kY00;
  rc[nc] = kY00;
  rc[nc + 6] = 0.1;  // (l, m) = (2, 0) on the second shape
  EXPECT(rbm_set_shapes_radial(c, 2, L, rc.data()) == RBM_OK, "radial shapes");
  const int n = 3;
  int sid[n] = {0, 1, 0};
  double cen[n * 3] = {0, 0, 0, 3.0, 0, 0, 0, 3.2, 0.5};
  double q[n * 4] = {1, 0, 0, 0, std::cos(0.3), std::sin(0.3), 0, 0, 1, 0, 0, 0};
  double qbad[n * 4] = {2, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0};
  EXPECT(rbm_set_bodies(c, n, sid, cen, qbad) == RBM_E_INVAL, "quaternion of norm 2 refused");
  int sid_bad[n] = {0, 2, 0};
  EXPECT(rbm_set_bodies(c, n, sid_bad, cen, q) == RBM_E_INVAL, "unknown shape id refused");
  EXPECT(rbm_set_bodies(c, n, sid, cen, q) == RBM_OK, "bodies");
  size_t bytes = 0;
  EXPECT(rbm_workspace_size(c, n, &bytes) == RBM_OK && bytes > 0, "workspace size");
  Dev ws(bytes);
  EXPECT(ws.p != nullptr, "hipMalloc workspace");
  if (!ws.p) {
    rbm_destroy(c);
    return;
  }
  EXPECT(rbm_bind_workspace(c, ws.p, bytes / 2) == RBM_E_NOMEM, "small workspace refused");
  EXPECT(rbm_bind_workspace(c, ws.p, bytes) == RBM_OK, "bind workspace");
  EXPECT(rbm_setup(c) == RBM_OK, "setup");

  STEP("device: solve");
  double FT[n * 6] = {1, 0, 0, 0, 0, 1, 0, -1, 0, 0.2, 0, 0, 0, 0, 1, 0, 0.3, 0};
  double VW[n * 6];
  rbm_solve_info info;
  EXPECT(rbm_solve(c, FT, VW, &info) == RBM_OK, "solve");
  EXPECT(info.rel_residual <= 1e-10 && info.iters > 0, "solve converged");
  double FTnan[n * 6];
  std::memcpy(FTnan, FT, sizeof FT);
  FTnan[4] = std::nan("");
  EXPECT(rbm_solve(c, FTnan, VW, nullptr) == RBM_E_INVAL, "NaN load refused");

  STEP("device: mobility matrix");
  std::vector<double> Mm(36 * n * n);
  EXPECT(rbm_mobility_matrix(c, Mm.data(), &info) == RBM_OK, "mobility matrix");
  double asym = 0, mx = 0;
  for (int i = 0; i < 6 * n; ++i)
    for (int j = 0; j < 6 * n; ++j) {
      asym = std::fmax(asym, std::fabs(Mm[i * 6 * n + j] - Mm[j * 6 * n + i]));
      mx = std::fmax(mx, std::fabs(Mm[i * 6 * n + j]));
    }
  EXPECT(mx > 0 && asym < 1e-3 * mx, "mobility matrix nearly symmetric");
  for (int i = 0; i < 6 * n; ++i) EXPECT(Mm[i * 6 * n + i] > 0, "positive diagonal");

  STEP("device: run state");
  size_t sb = 0;
  EXPECT(rbm_get_state(c, nullptr, &sb) == RBM_OK && sb > 0, "state size");
  std::vector<unsigned char> rec(sb);
  size_t small = sb - 1;
  EXPECT(rbm_get_state(c, rec.data(), &small) != RBM_OK, "short state buffer refused");
  EXPECT(rbm_get_state(c, rec.data(), &sb) == RBM_OK, "get state");
  EXPECT(rbm_set_state(c, rec.data(), sb) == RBM_OK, "set state");
  for (size_t cut : {(size_t)0, (size_t)8, sb / 2, sb - 1})
    EXPECT(rbm_set_state(c, rec.data(), cut) != RBM_OK, "truncated state refused");
  std::vector<unsigned char> bad = rec;
  bad[0] ^= 0xff;
  EXPECT(rbm_set_state(c, bad.data(), sb) != RBM_OK, "state with another tag refused");
  bad = rec;
  for (size_t k = 8; k < std::min<size_t>(sb, 64); ++k) bad[k] = 0xff;
  EXPECT(rbm_set_state(c, bad.data(), sb) != RBM_OK, "state with garbage sizes refused");

  STEP("device: RK4 step and poses");
  Dev dFT(sizeof FT);
  EXPECT(hipMemcpy(dFT.p, FT, sizeof FT, hipMemcpyHostToDevice) == hipSuccess, "copy loads");
  rbm_solve_info st[4];
  EXPECT(rbm_step_rk4(c, 0.05, (const double*)dFT.p, st) == RBM_OK, "RK4 step");
  double cen2[n * 3], q2[n * 4];
  EXPECT(rbm_get_bodies(c, cen2, q2) == RBM_OK, "get bodies");
  for (int i = 0; i < n; ++i) {
    double qq = 0;
    for (int k = 0; k < 4; ++k) qq += q2[4 * i + k] * q2[4 * i + k];
    EXPECT(std::fabs(qq - 1) < 1e-12, "unit quaternions after the step");
  }
  EXPECT(rbm_set_state(c, rec.data(), sb) == RBM_OK, "restore state");
  double cen3[n * 3], q3[n * 4];
  EXPECT(rbm_get_bodies(c, cen3, q3) == RBM_OK && std::memcmp(cen3, cen, sizeof cen) == 0,
         "restored poses");

  STEP("device: overlap");
  double cov[n * 3] = {0, 0, 0, 1.2, 0, 0, 0, 3.2, 0.5};
  EXPECT(rbm_set_bodies(c, n, sid, cov, q) == RBM_OK, "overlapping bodies accepted by set_bodies");
  EXPECT(rbm_solve(c, FT, VW, nullptr) == RBM_E_OVERLAP, "overlap reported by the solve");
  EXPECT(rbm_set_bodies(c, n, sid, cen, q) == RBM_OK, "separated bodies again");
  EXPECT(rbm_solve(c, FT, VW, nullptr) == RBM_OK, "solve after the overlap");

  STEP("device: learned warm start");
  rbm_learned_config lc;
  rbm_learned_default_config(&lc);
  lc.k_nbr = 2;
  lc.hidden = 32;
  lc.n_hidden = 2;
  lc.capacity = 64;
  lc.batch_max = 32;
  size_t lb = 0;
  EXPECT(rbm_learned_workspace_size(c, &lc, &lb) == RBM_OK && lb > 0, "learned workspace size");
  Dev lw(lb);
  EXPECT(lw.p && rbm_learned_bind(c, &lc, lw.p, lb) == RBM_OK, "learned bind");
  EXPECT(rbm_learned_set_capture(c, 1) == RBM_OK, "capture on");
  EXPECT(rbm_step_rk4(c, 0.05, (const double*)dFT.p, st) == RBM_OK, "RK4 step with capture");
  EXPECT(rbm_learned_set_capture(c, 0) == RBM_OK, "capture off");
  double loss = -1;
  EXPECT(rbm_learned_train(c, 2, 8, 1e-3, &loss) == RBM_OK && loss >= 0, "train");
  int samples = 0, F = 0, O = 0, P = 0;
  EXPECT(rbm_learned_info(c, &samples, &F, &O, &P) == RBM_OK && samples == 4 * n, "learned info");
  std::vector<float> par((size_t)P + 2 * F + 2);
  EXPECT(rbm_learned_get_params(c, par.data(), par.size()) == RBM_OK, "get params");
  EXPECT(rbm_learned_get_params(c, par.data(), par.size() - 1) == RBM_E_INVAL, "short params refused");
  EXPECT(rbm_learned_set_params(c, par.data(), par.size()) == RBM_OK, "set params");
  EXPECT(rbm_set_guess(c, RBM_GUESS_LEARNED) == RBM_OK, "learned guess mode");
  EXPECT(rbm_solve(c, FT, VW, &info) == RBM_OK && info.rel_residual <= 1e-10, "learned solve");
  size_t sb2 = 0;
  EXPECT(rbm_get_state(c, nullptr, &sb2) == RBM_OK && sb2 > sb, "state with the learned part");
  std::vector<unsigned char> rec2(sb2);
  EXPECT(rbm_get_state(c, rec2.data(), &sb2) == RBM_OK, "get learned state");
  EXPECT(rbm_set_state(c, rec2.data(), sb2) == RBM_OK, "set learned state");
  EXPECT(rbm_set_state(c, rec2.data(), sb2 - 4) != RBM_OK, "truncated learned state refused");

  STEP("device: low-level sums");
  const int np = 2 * 84;  // two bodies of M = 84 points
  std::vector<double> X(3 * np), Nn(3 * np), qv(3 * np);
  for (int a = 0; a < np; ++a)
    for (int k = 0; k < 3; ++k) {
      X[k * np + a] = std::sin(0.37 * a + k) + (a >= 84 && k == 0 ? 4.0 : 0.0);
      Nn[k * np + a] = std::cos(0.11 * a + 2 * k);
      qv[k * np + a] = std::sin(0.05 * a * (k + 1));
    }
  Dev dX(X.size() * 8), dN(X.size() * 8), dq(X.size() * 8), dy(X.size() * 8), dy2(X.size() * 8);
  EXPECT(hipMemcpy(dX.p, X.data(), X.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(dN.p, Nn.data(), X.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(dq.p, qv.data(), X.size() * 8, hipMemcpyHostToDevice) == hipSuccess,
         "copy sum inputs");
  EXPECT(rbm_far_traction(c, np, 84, (const double*)dX.p, (const double*)dN.p, (const double*)dq.p,
                          nullptr, (double*)dy.p, 0) == RBM_OK, "far traction");
  EXPECT(rbm_far_traction_static(np, 84, (const double*)dX.p, (const double*)dN.p, (const double*)dq.p,
                                 nullptr, (double*)dy2.p, 0, nullptr) == RBM_OK, "static far traction");
  EXPECT(rbm_far_traction_static(np, 84, (const double*)dX.p, (const double*)dN.p, (const double*)dq.p,
                                 nullptr, (double*)dy2.p, 2, nullptr) == RBM_E_INVAL, "precision 2 refused");
  EXPECT(rbm_far_traction_static(1 << 24, 84, (const double*)dX.p, (const double*)dN.p,
                                 (const double*)dq.p, nullptr, (double*)dy2.p, 0, nullptr) == RBM_E_NOMEM,
         "static sum beyond its scratch refused");
  std::vector<double> y(X.size()), y2(X.size());
  EXPECT(hipDeviceSynchronize() == hipSuccess &&
             hipMemcpy(y.data(), dy.p, X.size() * 8, hipMemcpyDeviceToHost) == hipSuccess &&
             hipMemcpy(y2.data(), dy2.p, X.size() * 8, hipMemcpyDeviceToHost) == hipSuccess,
         "copy sums back");
  double d = 0, m = 0;
  for (size_t k = 0; k < y.size(); ++k) {
    d = std::fmax(d, std::fabs(y[k] - y2[k]));
    m = std::fmax(m, std::fabs(y[k]));
  }
  EXPECT(m > 0 && d <= 1e-12 * m, "static sum equals the context's");
  rbm_destroy(c);
}

int main(int argc, char** argv) {
  const bool host_only = argc > 1 && std::strcmp(argv[1], "--host") == 0;
  host_checks();
  if (!host_only) device_checks();
  if (g_fail) {
    std::printf("abi_check: %d expectation(s) failed\n", g_fail);
    return 1;
  }
  std::printf("abi_check: ok\n");
  return 0;
}
