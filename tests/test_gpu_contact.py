"""GPU contact search and contact-force solves (§3.3) against the oracle's contact
algorithm with dense oracle mobility solves, and the pushed-pair pin (two touching
spheres pushed together stop, with the contact force cancelling the push)."""
import math

import numpy as np
import pytest

from paper_1606_07428_amd import inputs, rbm
from oracle import contact as ct
from oracle import system as sy
from tests.helpers import oracle_problem, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _min_node_distances(prob):
    out = []
    for a in range(prob.n):
        for b in range(a + 1, prob.n):
            d = np.sqrt(np.sum((prob.X[prob.sl(a)][:, None] - prob.X[prob.sl(b)][None]) ** 2, axis=2)).min()
            out.append(d)
    return np.sort(out)


def _contact_case(n, p, seed):
    w = inputs.tiny(n, p, seed=seed)
    prob = oracle_problem(w)
    d = _min_node_distances(prob)
    delta = 0.5 * (d[1] + d[2])          # two contacts, away from the threshold of a third
    return w, prob, delta


@pytest.mark.parametrize("n,p,seed", [(5, 6, 91), (6, 6, 92)])
def test_contact_search_matches_oracle(n, p, seed):
    _case(f"contact search n={n} p={p} seed={seed}")
    w, prob, delta = _contact_case(n, p, seed)
    s = rbm.solver_for(w)
    pairs, pts = s.find_contacts(delta)
    ref = ct.find_contacts(prob, delta)
    assert len(ref) == 2
    assert [tuple(x) for x in pairs] == [r[:2] for r in ref]
    assert np.abs(pts - np.array([r[2] for r in ref])).max() < 1e-13
    s.close()


@pytest.mark.parametrize("n,p,seed", [(5, 6, 91), (6, 6, 92)])
def test_contact_solve_matches_oracle(n, p, seed):
    _case(f"contact solve n={n} p={p} seed={seed}")
    w, prob, delta = _contact_case(n, p, seed)
    s = rbm.solver_for(w, tol=1e-13)
    pairs, pts = s.find_contacts(delta)
    VW, Fc, info = s.solve_contacts(w["FT"], pairs, pts)
    V0_o, Fc_o, V_o = ct.solve_with_contacts(prob, w["FT"], ct.find_contacts(prob, delta),
                                             lambda FT: sy.solve_dense(prob, FT)[2])
    assert rel_err(VW, V_o) < 1e-9
    assert rel_err(Fc, Fc_o) < 1e-8
    assert info["iters"] > 0
    s.close()


def test_pushed_pair_stops_on_gpu():
    _case("pushed pair p=8 gap=0.02")
    w = {"p": 8, "eta": 1.0, "shapes": [("radial", np.array([math.sqrt(4 * math.pi)]))],
         "shape_id": np.zeros(2, np.int32), "centres": np.array([[0.0, 0, 0], [2.02, 0, 0]]),
         "quats": np.array([[1.0, 0, 0, 0]] * 2)}
    s = rbm.solver_for(w, tol=1e-13)
    pairs, pts = s.find_contacts(0.05)
    assert len(pairs) == 1 and abs(pts[0, 0] - 1.01) < 1e-14 and np.abs(pts[0, 1:]).max() < 1e-14
    FT = np.zeros((2, 6))
    FT[0, 0], FT[1, 0] = 0.7, -0.7
    VW, Fc, _ = s.solve_contacts(FT, pairs, pts)
    assert np.abs(VW).max() < 1e-11
    assert np.abs(Fc[0] - np.array([-0.7, 0.0, 0.0])).max() < 1e-10
    s.close()


def test_rk4_step_with_contacts_matches_oracle():
    _case("rk4 with contacts: sheared pair p=6 gap=0.03")
    from oracle import timestep as ts
    w = {"p": 6, "eta": 1.0, "shapes": [("radial", np.array([math.sqrt(4 * math.pi)]))],
         "shape_id": np.zeros(2, np.int32), "centres": np.array([[0.0, 0, 0], [2.03, 0, 0]]),
         "quats": np.array([[1.0, 0, 0, 0]] * 2), "FT": np.array([[0.0, 1.0, 0, 0, 0, 0], [0.0, -1.0, 0, 0, 0, 0]])}
    s = rbm.solver_for(w, tol=1e-13, contact_delta=0.05)
    dt = 0.2
    infos = s.step_rk4(dt, torch.as_tensor(w["FT"], device="cuda"))
    assert all(i["iters"] > 0 for i in infos)
    c_g, q_g = s.bodies()
    shapes = [sy.Shape(np.array([[0, 0, 0, math.sqrt(4 * math.pi / 3)], [0, math.sqrt(4 * math.pi / 3), 0, 0],
                                 [0, 0, math.sqrt(4 * math.pi / 3), 0]]), 6)]

    def vel(c, q):
        prob = sy.Problem(shapes, w["shape_id"], c, q)
        contacts = ct.find_contacts(prob, 0.05)
        assert len(contacts) == 1
        return ct.solve_with_contacts(prob, w["FT"], contacts, lambda FT: sy.solve_dense(prob, FT)[2])[2]

    c, q = ts.rk4_step(vel, w["centres"], w["quats"], dt)
    assert np.abs(c_g - c).max() < 1e-10
    Rg = np.array([sy.quat_to_rot(x) for x in q_g])
    Ro = np.array([sy.quat_to_rot(x) for x in q])
    assert np.abs(Rg - Ro).max() < 1e-10
    s.close()
