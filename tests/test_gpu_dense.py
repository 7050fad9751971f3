"""Full-size solves in the configuration the benchmark times, checked against the oracle:
the 4000-body suspension at 20 % with a true surface gap of 0.1 (p = 12, 1.25 M points), the
1000-ellipsoid suspension (p = 16, 544 k points) and the 512 sedimenting spheres (p = 12,
160 k points) after three RK4 steps.  The GPU solves in the precision form (float32 far sums
with fast multipole inner iterations of order 12 at the two larger sizes, direct float32
sums at 512 bodies, float32 block preconditioner, float64 refinement residuals) with the
learned warm start, to a relative residual of 1e-8, with near-singular upsampling where
bodies are closer than a node spacing.  On sampled bodies the oracle then applies its own float64 operator to the
GPU density (§2.3, §3.2): the residual rows b - A mu against its own right-hand side, the
GPU's float64 residual vector at those rows, and the velocities it computes from the GPU
density (§3.3) against the GPU's.  The oracle's off-body sums at the sampled targets run in
threads over chunks of targets."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_1606_07428_amd import inputs, rbm
from oracle import singular as sg
from tests.helpers import oracle_problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

THREADS = max(1, min(16, os.cpu_count() or 1))


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _par_rows(prob, fn, idx):
    """fn over chunks of the targets idx in threads (plain rule); with upsampling the oracle
    walks every source body per call, so one call takes the whole body."""
    if prob.upsample is not None:
        return fn(np.asarray(idx))
    parts = [p for p in np.array_split(np.asarray(idx), THREADS) if len(p)]
    with ThreadPoolExecutor(len(parts)) as ex:
        return np.concatenate(list(ex.map(fn, parts)))


# Near-singular upsampling (§3) per configuration: the 20 % suspension has surfaces 0.1
# apart, half a node spacing, where the plain smooth rule leaves the discrete system too
# ill-conditioned for GMRES; the 10 % ellipsoids do not need it.
P_UP = {"dense4000": 24, "ellipsoids1000": 0, "sediment512": 0}
FMM = {"dense4000": 12, "ellipsoids1000": 12, "sediment512": 0}
# RK4 steps (their stage solves captured for training) before the checked solve
STEPS = {"dense4000": 0, "ellipsoids1000": 0, "sediment512": 3}


def _gpu_solve(name):
    w = inputs.workload(name)
    _case(f"{name}: setup, block-diagonal mixed solve (captured), training, learned mixed solve")
    s = rbm.solver_for(w, tol=1e-8, precision=rbm.MIXED_FP32, guess=rbm.GUESS_BLOCKDIAG, fmm_order=FMM[name],
                       p_up=P_UP[name])
    s.learned_bind(k_nbr=8, hidden=256, n_hidden=3, capacity=s.n * (1 + 4 * STEPS[name]), batch_max=1024, seed=7)
    FT = torch.as_tensor(np.asarray(w["FT"], dtype=np.float64), device="cuda")
    VW = torch.zeros_like(FT)
    s.learned_set_capture(True)
    for k in range(STEPS[name]):
        s.step_rk4(0.1, FT)
        print(f"[case] {name}: RK4 step {k + 1}/{STEPS[name]}", flush=True)
    if STEPS[name]:
        c, q = s.bodies()
        w = dict(w, centres=c, quats=q)
    i_bd = s.solve_dev(FT, VW)
    s.learned_set_capture(False)
    s.learned_train(20, 256, 1e-3)
    s.set_guess_mode(rbm.GUESS_LEARNED)
    info = s.solve_dev(FT, VW)
    torch.cuda.synchronize()
    print(f"[case] {name}: block-diagonal {i_bd['iters']} it ({i_bd['ms_total']:.0f} ms), learned "
          f"{info['iters']} it ({info['ms_total']:.0f} ms, fused pass used {info['fused_used']}), near pairs "
          f"{info['near_pairs']}, init residual "
          f"{i_bd['init_rel_residual']:.3f} -> {info['init_rel_residual']:.3f}, fallback {info['fallback_used']}, "
          f"rel residual {info['rel_residual']:.2e}", flush=True)
    mu, rho = s.density()
    out = {"w": w, "info": info, "VW": VW.cpu().numpy(), "mu": mu.T.copy(), "rho": rho.T.copy(), "s": s}
    return out


@pytest.fixture(scope="module", params=["dense4000", "ellipsoids1000", "sediment512"])
def solved(request):
    out = _gpu_solve(request.param)
    out["name"] = request.param
    print(f"[case] {request.param}: oracle geometry", flush=True)
    pu = P_UP[request.param]
    out["prob"] = oracle_problem(out["w"], with_ops=False, upsample=(pu, 5.0) if pu else None)
    yield out
    out["s"].close()


def _ops(prob, i):
    sh = prob.shapes[prob.shape_id[i]]
    if sh.ops is None:
        sh.ops = sg.singular_operators(sh.coef, sh.p, sh.ps, sh.eta)
    return sh


SAMPLES = {"dense4000": [7, 2711], "ellipsoids1000": [12, 640], "sediment512": [3, 300]}


def test_learned_mixed_solve_meets_the_tolerance_against_the_oracle(solved):
    prob, info, s = solved["prob"], solved["info"], solved["s"]
    w, mu_g, rho_g, VW = solved["w"], solved["mu"], solved["rho"], solved["VW"]
    assert info["rel_residual"] <= 1e-8 and info["guess_used"] == rbm.GUESS_LEARNED
    bnorm = info["bnorm"]
    N, M = prob.N, prob.M
    for i in SAMPLES[solved["name"]]:
        _case(f"{solved['name']}: oracle rows of body {i}")
        _ops(prob, i)
        sl = prob.sl(i)
        idx = np.arange(sl.start, sl.stop)
        rho_o = prob.incident_density(w["FT"])[sl]
        assert np.abs(rho_g[sl] - rho_o).max() <= 1e-12 * np.abs(rho_o).max()
        sig = rho_g + mu_g
        # b - A mu = -(1/2 sigma + K_self sigma + K_far sigma) - L mu, sigma = rho + mu
        kf = _par_rows(prob, lambda ix: prob.K_far(sig, ix), idx)
        ks = prob._apply_body_op("K", i, sig[sl])
        rr = prob.X[sl] - prob.c[i]
        wi = prob.w[sl][:, None]
        Lmu = np.sum(wi * mu_g[sl], 0)[None] + np.cross(np.sum(wi * np.cross(rr, mu_g[sl]), 0)[None], rr)
        r_o = -(0.5 * sig[sl] + ks + kf) - Lmu
        r_g = np.stack([s.read("r", M, offset=(c * N + i * M) * 8) for c in range(3)], axis=1)
        print(f"[case] body {i}: |r| oracle {np.linalg.norm(r_o):.3e}, |r_gpu - r_oracle| "
              f"{np.abs(r_g - r_o).max():.3e}, |b| {bnorm:.3e}", flush=True)
        assert np.linalg.norm(r_o) <= 1e-8 * bnorm
        assert np.abs(r_g - r_o).max() <= 1e-11 * bnorm
        # velocities of body i from the GPU density (§3.3)
        sf = _par_rows(prob, lambda ix: prob.S_far(sig, ix), idx)
        u = prob._apply_body_op("S", i, sig[sl]) + sf
        v = np.sum(wi * u, 0) / prob.area[i]
        om = np.linalg.solve(prob.tau[i], np.sum(wi * np.cross(rr, u), 0))
        err = np.abs(VW[i] - np.concatenate([v, om])).max() / np.abs(VW).max()
        print(f"[case] body {i}: velocity difference {err:.2e}", flush=True)
        assert err < 1e-10
