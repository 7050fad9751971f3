"""GPU parity of the near-singular correction by upsampling (§3) against the oracle's
upsampled rule: setup tables, near lists, the operator itself (element by element),
solves in every precision form, an RK4 step, and sampled targets at the 64-body
p = 12 workload.  Every test prints its case before touching the GPU."""
import numpy as np
import pytest

from paper_1606_07428_amd import inputs, rbm
from oracle import nearfield as nf
from oracle import system as sy
from oracle import timestep as ts
from tests.helpers import oracle_problem, oracle_shapes, rel_err, shape_coef

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


# (bodies, p, seed, p_up, kappa): small clusters with near and non-near pairs; every
# kappa is at least 0.3 away from the value at which some pair changes status
CASES = [(5, 6, 71, 12, 6.0), (4, 5, 72, 13, 5.0), (6, 6, 73, 15, 6.0)]


@pytest.mark.parametrize("n,p,seed,pu,kappa", CASES)
def test_setup_tables_match_oracle(n, p, seed, pu, kappa):
    _case(f"near setup tables n={n} p={p} seed={seed} p_up={pu}")
    w = inputs.tiny(n, p, seed=seed)
    s = rbm.solver_for(w, p_up=pu, near_factor=kappa)
    M, Mu = 2 * p * (p + 1), 2 * pu * (pu + 1)
    U = s.read("U", M * Mu).reshape(M, Mu).T
    U_o = nf.interp_matrix(p, pu)
    assert np.abs(U - U_o).max() < 1e-13 * np.abs(U_o).max()
    prob = oracle_problem(w, with_ops=False, upsample=(pu, kappa))
    for k in range(len(w["shapes"])):
        fo = prob.fine(k)
        fr = s.read("fr", 3 * Mu, offset=k * 3 * Mu * 8).reshape(3, Mu)
        fw = s.read("fw", Mu, offset=k * Mu * 8)
        rb = s.read("rb", 1, offset=k * 8)[0]
        assert np.abs(fr - fo["r"]).max() < 1e-13
        assert rel_err(fw, fo["w"]) < 1e-13
        assert abs(rb - fo["R"]) < 1e-13
    s.close()


@pytest.mark.parametrize("n,p,seed,pu,kappa", CASES)
def test_near_list_matches_oracle(n, p, seed, pu, kappa):
    _case(f"near list n={n} p={p} seed={seed} kappa={kappa}")
    w = inputs.tiny(n, p, seed=seed)
    s = rbm.solver_for(w, p_up=pu, near_factor=kappa)
    VW, info = s.solve(w["FT"])
    near_o = oracle_problem(w, with_ops=False, upsample=(pu, kappa)).near
    off = ~np.eye(n, dtype=bool)
    assert near_o[off].any() and not near_o[off].all()
    cnt = s.read("near_count", n, dtype=np.int32)
    lst = s.read("near_list", n * 64, dtype=np.int32).reshape(n, 64)
    assert info["near_pairs"] == int(near_o.sum())
    for i in range(n):
        assert cnt[i] == near_o[i].sum()
        assert list(lst[i, :cnt[i]]) == list(np.nonzero(near_o[i])[0])
    s.close()


@pytest.mark.parametrize("n,p,seed,pu,kappa", CASES)
def test_operator_matches_oracle(n, p, seed, pu, kappa):
    _case(f"upsampled operator n={n} p={p} seed={seed} p_up={pu} kappa={kappa}")
    w = inputs.tiny(n, p, seed=seed)
    s = rbm.solver_for(w, p_up=pu, near_factor=kappa)
    prob = oracle_problem(w, upsample=(pu, kappa))
    rng = np.random.default_rng(seed)
    mu = rng.standard_normal((prob.N, 3))
    y = s.apply_dev(_dev(mu.T)).cpu().numpy().T
    y_o = prob.apply_A(mu)
    assert rel_err(y, y_o) < 1e-12
    # the plain operator differs by the near correction (a check that it is applied)
    s0 = rbm.solver_for(w)
    y0 = s0.apply_dev(_dev(mu.T)).cpu().numpy().T
    assert rel_err(y0, y_o) > 1e-6
    s.close()
    s0.close()


@pytest.mark.parametrize("n,p,seed,pu,kappa", CASES)
def test_fp64_solve_matches_oracle_dense(n, p, seed, pu, kappa):
    _case(f"upsampled fp64 solve n={n} p={p} seed={seed}")
    w = inputs.tiny(n, p, seed=seed)
    s = rbm.solver_for(w, tol=1e-13, p_up=pu, near_factor=kappa)
    VW, info = s.solve(w["FT"])
    _, mu_o, VW_o = sy.solve_dense(oracle_problem(w, upsample=(pu, kappa)), w["FT"])
    assert info["rel_residual"] < 1e-13
    assert info["near_pairs"] > 0 and info["ms_near"] > 0.0
    assert rel_err(VW, VW_o) < 1e-10
    mu_g, _ = s.density()
    assert rel_err(mu_g.T, mu_o) < 1e-9
    s.close()


@pytest.mark.parametrize("prec", [rbm.MIXED_FP32, rbm.MIXED_BF16])
def test_mixed_precision_with_upsampling(prec):
    _case(f"upsampled mixed precision {prec}")
    n, p, seed, pu, kappa = CASES[0]
    w = inputs.tiny(n, p, seed=seed)
    s = rbm.solver_for(w, tol=1e-11, precision=prec, p_up=pu, near_factor=kappa)
    VW, info = s.solve(w["FT"])
    _, _, VW_o = sy.solve_dense(oracle_problem(w, upsample=(pu, kappa)), w["FT"])
    assert info["rel_residual"] < 1e-11 and info["refinements"] >= 1
    assert rel_err(VW, VW_o) < 1e-9
    s.close()


def test_shared_shape_gemm_path_with_upsampling():
    _case("upsampled shared shape n=20 p=6 p_up=12")
    w = inputs.tiny(20, 6, seed=61, shared=True)
    s = rbm.solver_for(w, tol=1e-12, p_up=12, near_factor=3.4)
    VW, info = s.solve(w["FT"])
    prob = oracle_problem(w, upsample=(12, 3.4))
    assert prob.near.sum() == info["near_pairs"] > 0
    _, _, VW_o = sy.solve_dense(prob, w["FT"])
    assert info["rel_residual"] < 1e-12
    assert rel_err(VW, VW_o) < 1e-10
    s.close()


def test_rk4_step_with_upsampling():
    _case("upsampled rk4 n=4 p=5 seed=72")
    n, p, seed, pu, kappa = CASES[1]
    w = inputs.tiny(n, p, seed=seed)
    s = rbm.solver_for(w, tol=1e-13, p_up=pu, near_factor=kappa)
    FT = torch.as_tensor(np.asarray(w["FT"]), device="cuda")
    dt = 0.3
    infos = s.step_rk4(dt, FT)
    assert all(i["rel_residual"] < 1e-13 for i in infos)
    c_g, q_g = s.bodies()
    shapes = oracle_shapes(w)

    def vel(c, q):
        return sy.solve_dense(sy.Problem(shapes, w["shape_id"], c, q, upsample=(pu, kappa)), w["FT"])[2]

    c, q = ts.rk4_step(vel, np.asarray(w["centres"], float), ts.normalize(np.asarray(w["quats"], float)), dt)
    assert np.abs(c_g - c).max() < 1e-11
    Rg = np.array([sy.quat_to_rot(x) for x in q_g])
    Ro = np.array([sy.quat_to_rot(x) for x in q])
    assert np.abs(Rg - Ro).max() < 1e-11
    s.close()


def test_full_size_correction_at_sampled_targets():
    """64 bodies, p = 12, p_up = 24: the GPU operator with upsampling minus the plain one
    equals the oracle's upsampled minus plain off-body sum at sampled targets."""
    _case("random64 p=12 p_up=24: near correction at sampled targets")
    w = inputs.workload("random64")
    s_up = rbm.solver_for(w, p_up=24, near_factor=5.0)
    s_pl = rbm.solver_for(w)
    prob_up = oracle_problem(w, with_ops=False, upsample=(24, 5.0))
    prob_pl = oracle_problem(w, with_ops=False)
    rng = np.random.default_rng(640)
    mu = rng.standard_normal((prob_up.N, 3))
    d = (s_up.apply_dev(_dev(mu.T)) - s_pl.apply_dev(_dev(mu.T))).cpu().numpy().T
    near_bodies = np.nonzero(prob_up.near.any(axis=1))[0]
    assert len(near_bodies) > 0
    idx = np.sort(np.concatenate([rng.choice(np.arange(i * prob_up.M, (i + 1) * prob_up.M), 12, replace=False)
                                  for i in rng.choice(near_bodies, min(8, len(near_bodies)), replace=False)]))
    d_o = prob_up.K_far(mu, idx) - prob_pl.K_far(mu, idx)
    scale = np.abs(prob_pl.K_far(mu, idx)).max()
    assert np.abs(d[idx] - d_o).max() < 1e-12 * scale
    assert np.abs(d_o).max() > 1e-6 * scale
    # bodies without near neighbours see exactly the plain operator
    far_bodies = np.nonzero(~prob_up.near.any(axis=1))[0]
    for i in far_bodies[:4]:
        assert np.abs(d[i * prob_up.M:(i + 1) * prob_up.M]).max() == 0.0
    s_up.close()
    s_pl.close()
