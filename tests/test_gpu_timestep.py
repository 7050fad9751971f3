"""GPU RK4 step (four device solves, device pose update) against the oracle's RK4
with dense oracle solves at every stage (§3.3)."""
import numpy as np
import pytest

from paper_1606_07428_amd import inputs, rbm
from oracle import system as sy
from oracle import timestep as ts
from tests.helpers import oracle_shapes, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("n,p,seed,dt,steps", [(3, 5, 31, 0.4, 2), (4, 6, 32, 0.25, 1)])
def test_rk4_steps_match_oracle(n, p, seed, dt, steps):
    print(f"\n[case] rk4 n={n} p={p} seed={seed} dt={dt} steps={steps}", flush=True)
    w = inputs.tiny(n, p, seed=seed)
    s = rbm.solver_for(w, tol=1e-13)
    FT = torch.as_tensor(np.asarray(w["FT"]), device="cuda")
    for _ in range(steps):
        infos = s.step_rk4(dt, FT)
        assert all(i["rel_residual"] < 1e-13 for i in infos)
    c_g, q_g = s.bodies()
    shapes = oracle_shapes(w)

    def vel(c, q):
        return sy.solve_dense(sy.Problem(shapes, w["shape_id"], c, q), w["FT"])[2]

    c, q = np.asarray(w["centres"], float), ts.normalize(np.asarray(w["quats"], float))
    for _ in range(steps):
        c, q = ts.rk4_step(vel, c, q, dt)
    assert np.abs(c_g - c).max() < 1e-11
    # q and -q are the same rotation; compare rotation matrices
    Rg = np.array([sy.quat_to_rot(x) for x in q_g])
    Ro = np.array([sy.quat_to_rot(x) for x in q])
    assert np.abs(Rg - Ro).max() < 1e-11
    assert np.abs(np.linalg.norm(q_g, axis=1) - 1).max() < 1e-14
    # the context's next solve uses the evolved poses
    VW, _ = s.solve(w["FT"])
    assert rel_err(VW, vel(c, q)) < 1e-10
    s.close()
