"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Every test prints the case it runs before touching the GPU."""
import math

import numpy as np
import pytest

from paper_1606_07428_amd import inputs, rbm
from oracle import farfield as ff
from oracle import geometry as geo
from oracle import singular as sg
from tests.helpers import oracle_problem, oracle_shapes, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _sum_solver(n_points, M):
    """A context whose workspace holds n_points points (one shared unit sphere)."""
    p = 2
    while 2 * p * (p + 1) < M:
        p += 1
    nb = -(-n_points // (2 * p * (p + 1)))
    w = {"p": p, "shapes": [("radial", [math.sqrt(4 * math.pi)])], "shape_id": np.zeros(nb, np.int32),
         "centres": np.arange(nb)[:, None] * np.array([[3.0, 0, 0]]), "quats": np.tile([1.0, 0, 0, 0], (nb, 1))}
    return rbm.solver_for(w)


@pytest.mark.parametrize("n_points,M,prec", [(5 * 84, 84, 0), (1037, 84, 0), (9 * 512 + 77, 144, 0),
                                             (1037, 84, 1), (9 * 512 + 77, 144, 1),
                                             (70001, 312, 0), (70001, 312, 1)])
def test_far_sums_match_oracle(n_points, M, prec):
    _case(f"far sums n={n_points} M={M} precision={prec}")
    rng = np.random.default_rng(n_points + M)
    X = rng.uniform(-4, 4, (n_points, 3))
    Nn = rng.standard_normal((n_points, 3))
    Nn /= np.linalg.norm(Nn, axis=1)[:, None]
    q = rng.standard_normal((n_points, 3))
    add = rng.standard_normal((n_points, 3))
    body = np.arange(n_points) // M
    s = _sum_solver(n_points, M)
    yt = s.far_traction(_dev(X.T), _dev(Nn.T), _dev(q.T), M, add=_dev(add.T), precision=prec)
    us = s.far_stokeslet(_dev(X.T), _dev(q.T), M, precision=prec)
    torch.cuda.synchronize()
    idx = np.arange(n_points) if n_points < 2000 else rng.choice(n_points, 300, replace=False)
    # The float32 kernel reads positions, normals and strengths rounded to float32; the
    # oracle takes the same rounded inputs (in float64 arithmetic), so what remains is the
    # float32 arithmetic of the pair terms and their sums, held to 1e-5 relative.
    Xo, No, qo = (X, Nn, q) if prec == 0 else (a.astype(np.float32).astype(np.float64) for a in (X, Nn, q))
    ref_t = add[idx] + ff.traction_sum(Xo[idx], No[idx], Xo, qo, body[idx], body)
    ref_u = ff.stokeslet_sum(Xo[idx], Xo, qo, body[idx], body)
    tol = 1e-12 if prec == 0 else 1e-5
    et = rel_err(yt.cpu().numpy().T[idx], ref_t)
    eu = rel_err(us.cpu().numpy().T[idx], ref_u)
    print(f"[case] traction {et:.2e}, Stokeslet {eu:.2e}", flush=True)
    assert et < tol and eu < tol
    s.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_far_sums_degenerate_cases(prec):
    """Cases the all-pairs sum must get right beyond the tiles: every point on one body (a full
    body and a ragged one shorter than M), where no pair survives and the sums are add and
    zero exactly; two one-point bodies, where each sum is the single pair term of §2.1 written
    out here; and a precision the calls do not know."""
    _case(f"far sums, degenerate cases, precision={prec}")
    rng = np.random.default_rng(11)
    for n, M in [(84, 84), (37, 84)]:
        X, Nn, q, add = (rng.standard_normal((3, n)) for _ in range(4))
        s = _sum_solver(n, M)
        y = s.far_traction(_dev(X), _dev(Nn), _dev(q), M, add=_dev(add), precision=prec)
        u = s.far_stokeslet(_dev(X), _dev(q), M, precision=prec)
        ys = rbm.far_traction_static(_dev(X), _dev(Nn), _dev(q), M, add=_dev(add), precision=prec)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), add) and np.array_equal(ys.cpu().numpy(), add)
        assert not u.cpu().numpy().any()
        s.close()
    # two bodies of one point each
    X = np.array([[0.3, -0.9], [0.2, 0.4], [-0.5, 0.7]])
    Nn = np.array([[0.6, 0.0], [0.0, 0.8], [0.8, 0.6]])
    q = np.array([[1.5, -0.4], [0.3, 0.9], [-0.7, 0.2]])
    s = _sum_solver(2, 1)
    y = s.far_traction(_dev(X), _dev(Nn), _dev(q), 1, precision=prec).cpu().numpy()
    u = s.far_stokeslet(_dev(X), _dev(q), 1, precision=prec).cpu().numpy()
    for a, b in [(0, 1), (1, 0)]:
        d = X[:, a] - X[:, b]
        r = np.sqrt(d @ d)
        t = -3.0 / (4 * math.pi) * d * (d @ Nn[:, a]) * (d @ q[:, b]) / r ** 5
        v = (q[:, b] / r + d * (d @ q[:, b]) / r ** 3) / (8 * math.pi)
        tol = 1e-14 if prec == 0 else 1e-6
        assert np.abs(y[:, a] - t).max() <= tol * np.abs(t).max()
        assert np.abs(u[:, a] - v).max() <= tol * np.abs(v).max()
    with pytest.raises(rbm.RbmError) as e:
        s.far_traction(_dev(X), _dev(Nn), _dev(q), 1, precision=2)
    assert e.value.status == rbm.RBM_E_INVAL
    s.close()


def _body_frame_ops(shape):
    ops = shape.ops
    A0 = 0.5 * np.eye(ops["K"].shape[0]) + ops["K"] + sg.L_operator(shape.geom)
    return ops["S"], A0


@pytest.mark.parametrize("name,p", [("tiny", 6), ("two_spheres", 8)])
def test_setup_operators_match_oracle(name, p):
    _case(f"setup operators {name} p={p}")
    w = inputs.tiny(3, p, seed=21) if name == "tiny" else inputs.workload(name)
    s = rbm.solver_for(w)
    M = 2 * p * (p + 1)
    M3 = 3 * M
    shapes = oracle_shapes(w)
    for k, sh in enumerate(shapes):
        S0, A0 = _body_frame_ops(sh)
        A_gpu = s.read("A0", M3 * M3, offset=k * M3 * M3 * 8).reshape(M3, M3).T
        P_gpu = s.read("P0", M3 * M3, offset=k * M3 * M3 * 8).reshape(M3, M3).T
        assert rel_err(A_gpu, A0) < 1e-12
        assert rel_err(P_gpu, np.linalg.inv(A0)) < 1e-11
        g = sh.geom
        assert rel_err(s.read("gw", M, offset=k * M * 8), g["w"]) < 1e-13
        assert rel_err(s.read("gr", 3 * M, offset=k * 3 * M * 8).reshape(3, M), g["r"]) < 1e-12
        shp = s.read("shape", 32, offset=k * 32 * 8)
        assert abs(shp[0] - g["area"]) < 1e-12 * g["area"]
        assert rel_err(shp[4:13].reshape(3, 3), g["tau"]) < 1e-12
        # velocity functional G' S0
        r, wq = g["r"], g["w"]
        G = np.zeros((6, M3))
        for c in range(3):
            G[c, c * M:(c + 1) * M] = wq / g["area"]
        ti = np.linalg.inv(g["tau"])
        for kk in range(3):
            for c in range(3):
                # (r x u)_e = eps_{efc} r_f u_c
                col = np.zeros(M)
                for e in range(3):
                    f = [ff_ for ff_ in range(3) if ff_ not in (e, c)]
                    if e == c or not f:
                        continue
                    f = f[0]
                    sign = 1.0 if (e, f, c) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)) else -1.0
                    col += ti[kk, e] * sign * r[f]
                G[3 + kk, c * M:(c + 1) * M] = wq * col
        V_gpu = s.read("V0", 6 * M3, offset=k * 6 * M3 * 8).reshape(6, M3)
        assert rel_err(V_gpu, G @ S0) < 1e-12
    s.close()


def test_single_sphere_drag_laws():
    _case("single sphere drag")
    w = inputs.workload("single_sphere")
    s = rbm.solver_for(w)
    FT = np.array([[1.0, -0.5, 0.25, 0.3, 0.0, 1.0]])
    VW, info = s.solve(FT)
    assert np.abs(VW[0, :3] - FT[0, :3] / (6 * math.pi)).max() < 1e-13
    assert np.abs(VW[0, 3:] - FT[0, 3:] / (8 * math.pi)).max() < 1e-13
    s.close()


def test_two_spheres_match_oracle_dense_solve():
    _case("two spheres p=8 dense oracle")
    w = inputs.workload("two_spheres")
    s = rbm.solver_for(w, tol=1e-13)
    VW, info = s.solve(w["FT"])
    prob = oracle_problem(w)
    rho, mu, VW_o = __import__("oracle.system", fromlist=["x"]).solve_dense(prob, w["FT"])
    assert info["rel_residual"] < 1e-13
    # the converging residual was predicted, so its pass also gave the velocities' Stokeslet sum
    assert info["fused_used"] == 1 and info["n_fused"] == 1 and info["n_stokeslet"] == 0
    assert rel_err(VW, VW_o) < 1e-11
    mu_g, rho_g = s.density()
    assert rel_err(rho_g.T, rho) < 1e-13
    assert rel_err(mu_g.T, mu) < 1e-10
    # reflection symmetry zeros
    assert np.abs(VW[:, [2, 3, 4]]).max() < 1e-14
    s.close()


@pytest.mark.parametrize("n,p,seed,guess", [(4, 6, 3, rbm.GUESS_BLOCKDIAG), (3, 5, 4, rbm.GUESS_ZERO),
                                            (7, 5, 5, rbm.GUESS_BLOCKDIAG)])
def test_random_bodies_match_oracle(n, p, seed, guess):
    _case(f"random bodies n={n} p={p} seed={seed} guess={guess}")
    from oracle import system as sy
    w = inputs.tiny(n, p, seed=seed)
    s = rbm.solver_for(w, tol=1e-13, guess=guess)
    VW, info = s.solve(w["FT"])
    prob = oracle_problem(w)
    _, mu_o, VW_o = sy.solve_dense(prob, w["FT"])
    assert info["rel_residual"] < 1e-13
    assert rel_err(VW, VW_o) < 1e-10
    mu_g, _ = s.density()
    assert rel_err(mu_g.T, mu_o) < 1e-9
    s.close()


@pytest.mark.parametrize("prec", [rbm.FP64, rbm.MIXED_FP32])
def test_velocities_with_and_without_the_fused_pass_match(prec):
    """The same solve with the fused traction + Stokeslet pass for the converging residual and
    with a separate Stokeslet sum (velocity_fusion = 0): the same iterations, the same density
    and the same velocities to rounding, both matching the oracle."""
    _case(f"fused vs separate velocity sums, tiny n=5 p=6, precision={prec}")
    from oracle import system as sy
    w = inputs.tiny(5, 6, seed=8)
    s1 = rbm.solver_for(w, tol=1e-11, precision=prec)
    VW1, i1 = s1.solve(w["FT"])
    s2 = rbm.solver_for(w, tol=1e-11, precision=prec, velocity_fusion=0)
    VW2, i2 = s2.solve(w["FT"])
    print(f"[case] fused {i1['n_fused']} (used {i1['fused_used']}), separate {i2['n_stokeslet']}", flush=True)
    assert i1["fused_used"] == 1 and i1["n_stokeslet"] == 0
    assert i2["n_fused"] == 0 and i2["fused_used"] == 0 and i2["n_stokeslet"] == 1
    assert i1["iters"] == i2["iters"]
    assert rel_err(VW1, VW2) < 1e-12
    _, _, VW_o = sy.solve_dense(oracle_problem(w), w["FT"])
    assert rel_err(VW1, VW_o) < 1e-9
    s1.close()
    s2.close()


@pytest.mark.parametrize("prec", [rbm.MIXED_FP32, rbm.MIXED_BF16])
def test_mixed_precision_reaches_fp64_answer(prec):
    _case(f"mixed precision {prec} tiny")
    from oracle import system as sy
    w = inputs.tiny(5, 6, seed=8)
    s = rbm.solver_for(w, tol=1e-11, precision=prec)
    VW, info = s.solve(w["FT"])
    _, _, VW_o = sy.solve_dense(oracle_problem(w), w["FT"])
    assert info["rel_residual"] < 1e-11
    assert info["refinements"] >= 1
    # one float64 residual per refinement: the first refinement starts from the inner
    # operators' residual
    assert info["n_traction"] + info["n_fused"] == info["refinements"]
    assert rel_err(VW, VW_o) < 1e-9
    s.close()


@pytest.mark.parametrize("prec", [rbm.FP64, rbm.MIXED_FP32, rbm.MIXED_BF16])
def test_shared_shape_gemm_path_matches_oracle(prec):
    # one shape for all 20 bodies: the self apply runs as an MFMA GEMM (ragged 64x64 tiles)
    _case(f"shared shape n=20 p=6 precision={prec}")
    from oracle import system as sy
    w = inputs.tiny(20, 6, seed=61, shared=True)
    s = rbm.solver_for(w, tol=1e-12, precision=prec)
    VW, info = s.solve(w["FT"])
    _, mu_o, VW_o = sy.solve_dense(oracle_problem(w), w["FT"])
    assert info["rel_residual"] < 1e-12
    assert rel_err(VW, VW_o) < 1e-10
    s.close()


@pytest.mark.parametrize("p", [2, 20])
def test_sphere_drag_laws_at_the_order_limits(p):
    """Smallest and largest expansion orders the library accepts: the isolated sphere's
    drag laws v = F/(6 pi), w = T/(8 pi) are exact at every order."""
    _case(f"single sphere drag, p={p}")
    w = dict(inputs.workload("single_sphere"), p=p)
    s = rbm.solver_for(w, tol=1e-13)
    FT = np.array([[0.4, 1.0, -0.7, -0.2, 0.9, 0.5]])
    VW, info = s.solve(FT)
    assert info["rel_residual"] < 1e-13
    assert np.abs(VW[0, :3] - FT[0, :3] / (6 * math.pi)).max() < 1e-12
    assert np.abs(VW[0, 3:] - FT[0, 3:] / (8 * math.pi)).max() < 1e-12
    s.close()


def test_ellipsoid_mobility_against_oberbeck_and_jeffery():
    """Tri-axial ellipsoid (1, 0.8, 0.6) at p = 16: the GPU mobility is diagonal in the body
    frame with Oberbeck's translational and Jeffery's rotational coefficients (closed forms
    by elliptic integrals), to the discretization's accuracy."""
    from tests.test_oracle_system import _oberbeck
    _case("ellipsoid (1, 0.8, 0.6) p=16 vs Oberbeck/Jeffery")
    k = math.sqrt(4 * math.pi / 3)
    a = np.zeros((3, 4))
    a[0, 3], a[1, 1], a[2, 2] = 1.0 * k, 0.8 * k, 0.6 * k
    w = {"p": 16, "eta": 1.0, "shapes": [("coef", a)], "shape_id": np.zeros(1, np.int32),
         "centres": np.zeros((1, 3)), "quats": np.array([[1.0, 0, 0, 0]])}
    s = rbm.solver_for(w, tol=1e-13)
    Mm = np.zeros((6, 6))
    for j in range(6):
        FT = np.zeros((1, 6))
        FT[0, j] = 1.0
        Mm[:, j] = s.solve(FT)[0][0]
    ref = _oberbeck(1.0, 0.8, 0.6)
    assert np.abs(np.diag(Mm) / ref - 1).max() < 1e-8
    assert np.abs(Mm - np.diag(np.diag(Mm))).max() < 1e-11
    s.close()


@pytest.mark.parametrize("prec", [rbm.FP64, rbm.MIXED_FP32])
def test_gmres_lookahead_modes_give_the_same_solution(prec):
    """Queueing GMRES iteration k+1 before iteration k's residual estimate is read (never,
    when predicted safe, always) changes the schedule only: a queued iteration after
    convergence writes nothing the solution reads, so the velocities are bitwise equal."""
    _case(f"gmres lookahead 0/1/2, tiny n=5 p=6, precision={prec}")
    from oracle import system as sy
    w = inputs.tiny(5, 6, seed=8)
    out = []
    for mode in (0, 1, 2):
        s = rbm.solver_for(w, tol=1e-11, precision=prec, gmres_lookahead=mode)
        VW, info = s.solve(w["FT"])
        assert info["rel_residual"] < 1e-11 and info["iters"] >= 3
        out.append((VW, info))
        s.close()
    for VW, info in out[1:]:
        assert np.array_equal(VW, out[0][0])
        assert info["iters"] == out[0][1]["iters"]
    assert out[2][1]["matvecs"] >= out[0][1]["matvecs"]
    _, _, VW_o = sy.solve_dense(oracle_problem(w), w["FT"])
    assert rel_err(out[2][0], VW_o) < 1e-9


@pytest.mark.parametrize("p,p_sing", [(6, 7), (6, 18), (5, 6)])
def test_singular_rule_orders_match_oracle(p, p_sing):
    """The rotated-grid rule at orders other than the default 2p (the smallest allowed, p+1,
    and 3p): operators and dense-solve velocities against the oracle with the same order."""
    _case(f"p={p} p_sing={p_sing}: setup operators and solve vs oracle")
    from oracle import system as sy
    w = inputs.tiny(3, p, seed=30 + p_sing)
    s = rbm.solver_for(w, tol=1e-13, p_sing=p_sing)
    M3 = 3 * 2 * p * (p + 1)
    shapes = oracle_shapes(w, ps=p_sing)
    for k, sh in enumerate(shapes):
        _, A0 = _body_frame_ops(sh)
        A_gpu = s.read("A0", M3 * M3, offset=k * M3 * M3 * 8).reshape(M3, M3).T
        assert rel_err(A_gpu, A0) < 1e-12
    VW, info = s.solve(w["FT"])
    _, _, VW_o = sy.solve_dense(oracle_problem(w, ps=p_sing), w["FT"])
    assert info["rel_residual"] < 1e-13
    assert rel_err(VW, VW_o) < 1e-10
    s.close()


@pytest.mark.parametrize("max_iter,guess", [(3, rbm.GUESS_BLOCKDIAG), (2, rbm.GUESS_ZERO)])
def test_restarted_gmres_matches_oracle(max_iter, guess):
    """Float64 GMRES restarted every max_iter iterations (several cycles, each starting from
    the exact residual of the previous one) reaches the oracle's dense solution."""
    _case(f"restarted GMRES max_iter={max_iter} guess={guess}, tiny n=5 p=6")
    from oracle import system as sy
    w = inputs.tiny(5, 6, seed=8)
    s = rbm.solver_for(w, tol=1e-12, max_iter=max_iter, max_restart=60, guess=guess)
    VW, info = s.solve(w["FT"])
    print(f"[case] cycles {info['cycles']}, iterations {info['iters']}", flush=True)
    assert info["rel_residual"] < 1e-12
    assert info["cycles"] >= 3
    _, mu_o, VW_o = sy.solve_dense(oracle_problem(w), w["FT"])
    assert rel_err(VW, VW_o) < 1e-10
    mu_g, _ = s.density()
    assert rel_err(mu_g.T, mu_o) < 1e-9
    s.close()


def test_stalled_refinement_switches_to_float64_cycles():
    """Precision form with the stall threshold forced from the host (ir_stall = 1e-9: every
    refinement after the first counts as stalled): the remaining cycles run with float64
    operators and the solve still reaches the oracle's dense solution."""
    _case("GMRES-IR stall fallback, tiny n=5 p=6, ir_stall=1e-9")
    from oracle import system as sy
    w = inputs.tiny(5, 6, seed=8)
    s = rbm.solver_for(w, tol=1e-11, precision=rbm.MIXED_FP32, inner_tol=1e-3, ir_stall=1e-9)
    VW, info = s.solve(w["FT"])
    print(f"[case] refinements {info['refinements']}, float64 cycles {info['fp64_cycles']}", flush=True)
    assert info["rel_residual"] < 1e-11
    assert info["fp64_cycles"] >= 1 and info["refinements"] >= 2
    _, _, VW_o = sy.solve_dense(oracle_problem(w), w["FT"])
    assert rel_err(VW, VW_o) < 1e-9
    s2 = rbm.solver_for(w, tol=1e-11, precision=rbm.MIXED_FP32, inner_tol=1e-3)
    _, info2 = s2.solve(w["FT"])
    assert info2["fp64_cycles"] == 0
    s.close()
    s2.close()


@pytest.mark.parametrize("prec", [rbm.FP64, rbm.MIXED_FP32])
def test_zero_loads_give_zero_velocities(prec):
    """No load on any body: the incident density and the right-hand side vanish (§2.2), so
    mu = 0 and every velocity is exactly zero, without a GMRES iteration; a load on one body
    afterwards is solved normally."""
    _case(f"zero loads, precision {prec}")
    w = inputs.tiny(4, 5, seed=3)
    s = rbm.solver_for(w, tol=1e-10, precision=prec)
    VW, info = s.solve(np.zeros((4, 6)))
    assert np.all(VW == 0.0) and info["iters"] == 0 and info["rel_residual"] == 0.0
    FT = np.zeros((4, 6))
    FT[2, 1] = 1.0
    VW, info = s.solve(FT)
    assert info["rel_residual"] <= 1e-10 and info["iters"] > 0 and VW[2, 1] > 0
    s.close()
