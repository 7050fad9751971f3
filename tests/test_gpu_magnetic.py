"""GPU magnetostatics (§4) against the oracle: Laplace self operators, density q,
potential, normal derivative, Maxwell traction and net loads on small clusters; the
isolated permeable sphere's closed form; the density-driven mobility solve; the
induced-dipole force between two spheres."""
import math

import numpy as np
import pytest

from paper_1606_07428_amd import inputs, rbm
from oracle import magnetic as mg
from oracle import system as sy
from tests.helpers import oracle_problem, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


UNIT = ("radial", np.array([math.sqrt(4 * math.pi)]))


def _pair(d, p=8):
    return {"p": p, "eta": 1.0, "shapes": [UNIT], "shape_id": np.zeros(2, np.int32),
            "centres": np.array([[0.0, 0, 0], [d, 0, 0]]), "quats": np.array([[1.0, 0, 0, 0]] * 2)}


@pytest.mark.parametrize("n,p,seed", [(3, 6, 101), (4, 5, 102)])
def test_magnetics_match_oracle(n, p, seed):
    _case(f"magnetics n={n} p={p} seed={seed}")
    w = inputs.tiny(n, p, seed=seed)
    H0, mu_r = np.array([0.4, -1.0, 0.7]), 3.0
    s = rbm.solver_for(w, magnetic=1)
    rho, FT, it = s.magnetic_traction(H0, mu_r, tol=1e-13)
    assert it > 0
    prob = oracle_problem(w, with_ops=False)
    mag = mg.Magnetic(prob, mu_r, H0)
    M = 2 * p * (p + 1)
    for k in range(len(w["shapes"])):
        SL = s.read("SL0", M * M, offset=k * M * M * 8).reshape(M, M).T
        KL = s.read("KL0", M * M, offset=k * M * M * 8).reshape(M, M).T
        assert np.abs(SL - mag.ops[k]["S"]).max() < 1e-12 * np.abs(mag.ops[k]["S"]).max()
        assert np.abs(KL - mag.ops[k]["K"]).max() < 1e-12 * np.abs(mag.ops[k]["K"]).max()
    q = mag.density()
    assert rel_err(s.read("mag_q", prob.N), q) < 1e-11
    phi_o = -(prob.X @ H0) + mag.SL(q)
    dn_o = -(prob.Nn @ H0) - 0.5 * q + mag.KL(q)
    assert rel_err(s.read("mag_phi", prob.N), phi_o) < 1e-11
    assert rel_err(s.read("mag_dn", prob.N), dn_o) < 1e-11
    rho_o = mag.traction(mag.field(q))
    assert rel_err(rho.cpu().numpy().T, rho_o) < 1e-10
    assert rel_err(FT.cpu().numpy(), mag.forces(rho_o)) < 1e-10
    # the mobility problem driven by the oracle's traction
    VW = torch.zeros((n, 6), dtype=torch.float64, device="cuda")
    s2 = rbm.solver_for(w, tol=1e-13)
    info = s2.solve_density_dev(torch.as_tensor(np.ascontiguousarray(rho_o.T), device="cuda"), VW)
    _, VW_o = sy.solve_dense_density(oracle_problem(w), rho_o)
    assert info["rel_residual"] < 1e-13
    assert rel_err(VW.cpu().numpy(), VW_o) < 1e-10
    s.close()
    s2.close()


@pytest.mark.parametrize("mu_r", [2.0, 0.5])
def test_isolated_sphere_closed_form_on_gpu(mu_r):
    _case(f"isolated sphere mu_r={mu_r}")
    w = {"p": 8, "eta": 1.0, "shapes": [UNIT], "shape_id": np.zeros(1, np.int32),
         "centres": np.zeros((1, 3)), "quats": np.array([[1.0, 0, 0, 0]])}
    H0 = np.array([0.3, -1.2, 0.7])
    s = rbm.solver_for(w, magnetic=1)
    rho, FT, _ = s.magnetic_traction(H0, mu_r, tol=1e-13)
    n = s.read("N", 3 * s.N).reshape(3, s.N).T
    eta = (mu_r - 1) / (mu_r + 1)
    q = s.read("mag_q", s.N)
    assert np.abs(q - 6 * eta / (3 - eta) * (n @ H0)).max() < 1e-12
    Hin = 3 * H0 / (mu_r + 2)
    H = Hin[None, :] - (n @ Hin)[:, None] * n + mu_r * (n @ Hin)[:, None] * n
    rho_exact = (np.sum(H * n, 1)[:, None] * H - 0.5 * np.sum(H * H, 1)[:, None] * n)
    assert np.abs(rho.cpu().numpy().T - rho_exact).max() < 1e-10
    assert np.abs(FT.cpu().numpy()).max() < 1e-11
    s.close()


def test_two_spheres_dipole_force_on_gpu():
    _case("two spheres d=8 mu_r=2: dipole force law")
    mu_r, d = 2.0, 8.0
    beta = (mu_r - 1) / (mu_r + 2)
    m = 4 * math.pi * beta
    s = rbm.solver_for(_pair(d), magnetic=1)
    for H0, k in ((np.array([0.0, 1.0, 0.0]), 3.0), (np.array([1.0, 0.0, 0.0]), -6.0)):
        _, FT, _ = s.magnetic_traction(H0, mu_r, tol=1e-13)
        F = FT.cpu().numpy()
        ref = k * m * m / (4 * math.pi * d**4)
        assert abs(F[1, 0] / ref - 1) < 0.05
        assert np.abs(F[0, :3] + F[1, :3]).max() < 1e-8 * abs(ref)
    s.close()


def _oracle_mhd_velocity(w, H0, mu_r, delta=0.0):
    from oracle import contact as ct
    shapes = oracle_problem(w).shapes

    def vel(c, q):
        prob = sy.Problem(shapes, w["shape_id"], c, q)
        mag = mg.Magnetic(prob, mu_r, H0)
        rho = mag.traction(mag.field(mag.density()))
        V0 = sy.solve_dense_density(prob, rho)[1]
        contacts = ct.find_contacts(prob, delta) if delta > 0 else []
        if not contacts:
            return V0
        return ct.solve_with_contacts(prob, None, contacts, lambda FT: sy.solve_dense(prob, FT)[2], V0=V0)[2]
    return vel


def _compare_poses(s, c, q, tol):
    c_g, q_g = s.bodies()
    assert np.abs(c_g - c).max() < tol
    Rg = np.array([sy.quat_to_rot(x) for x in q_g])
    Ro = np.array([sy.quat_to_rot(x) for x in q])
    assert np.abs(Rg - Ro).max() < tol


@pytest.mark.parametrize("n,p,seed,dt", [(3, 5, 41, 0.5)])
def test_magnetic_rk4_step_matches_oracle(n, p, seed, dt):
    from oracle import timestep as ts
    _case(f"magnetic rk4 n={n} p={p} seed={seed} dt={dt}")
    w = inputs.tiny(n, p, seed=seed)
    H0, mu_r = 3.0 * np.array([1.0, -1.0, -1.0]) / math.sqrt(3.0), 2.0
    s = rbm.solver_for(w, tol=1e-13, magnetic=1)
    infos = s.step_rk4_magnetic(dt, H0, mu_r, tol_mag=1e-13)
    assert all(i["rel_residual"] < 1e-13 for i in infos)
    c, q = np.asarray(w["centres"], float), ts.normalize(np.asarray(w["quats"], float))
    c1, q1 = ts.rk4_step(_oracle_mhd_velocity(w, H0, mu_r), c, q, dt)
    assert np.abs(c1 - c).max() > 1e-4          # the bodies did move
    _compare_poses(s, c1, q1, 1e-11)
    s.close()


def test_magnetic_rk4_step_with_contacts_matches_oracle():
    """Two spheres touching along the field attract; the contact forces of §3.3 hold them."""
    from oracle import timestep as ts
    _case("magnetic rk4 with contacts: two spheres along H0, gap 0.03, delta 0.05")
    w = _pair(2.03, p=6)
    H0, mu_r, dt, delta = np.array([4.0, 0.0, 0.0]), 2.0, 0.2, 0.05
    s = rbm.solver_for(w, tol=1e-13, magnetic=1, contact_delta=delta)
    s.step_rk4_magnetic(dt, H0, mu_r, tol_mag=1e-13)
    c, q = np.asarray(w["centres"], float), np.asarray(w["quats"], float)
    c1, q1 = ts.rk4_step(_oracle_mhd_velocity(w, H0, mu_r, delta), c, q, dt)
    _compare_poses(s, c1, q1, 1e-11)
    # without the contact forces the pair closes the gap
    s2 = rbm.solver_for(w, tol=1e-13, magnetic=1)
    s2.step_rk4_magnetic(dt, H0, mu_r, tol_mag=1e-13)
    gap_free = s2.bodies()[0][1, 0] - s2.bodies()[0][0, 0]
    gap_held = s.bodies()[0][1, 0] - s.bodies()[0][0, 0]
    assert gap_free < 2.03 - 1e-4 and abs(gap_held - 2.03) < 1e-3 * (2.03 - gap_free)
    s.close()
    s2.close()
