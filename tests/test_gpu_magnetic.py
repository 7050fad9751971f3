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
