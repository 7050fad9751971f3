"""Pins of the oracle's RK4 evolution (§3.3; convergence rates of the paper's RK4 table)."""
import math

import numpy as np

from oracle import geometry as geo
from oracle import system as sy
from oracle import timestep as ts


def test_quaternion_product_matches_rotation_composition():
    rng = np.random.default_rng(0)
    a, b = ts.normalize(rng.standard_normal(4)), ts.normalize(rng.standard_normal(4))
    Ra, Rb = sy.quat_to_rot(a), sy.quat_to_rot(b)
    assert np.abs(sy.quat_to_rot(ts.quat_mul(a, b)) - Ra @ Rb).max() < 1e-14


def test_constant_rotation_matches_rodrigues():
    # constant omega, constant v: RK4 must reproduce exp(t [omega]x) R0 to O(dt^4)
    om = np.array([0.3, -1.1, 0.7])
    v = np.array([0.2, 0.0, -0.5])
    q0 = ts.normalize(np.array([[0.9, 0.1, -0.2, 0.3]]))
    fn = lambda c, q: np.concatenate([v, om])[None, :]  # noqa: E731
    T = 2.0
    errs = []
    for nsteps in (16, 32, 64):
        c, q = np.zeros((1, 3)), q0.copy()
        for _ in range(nsteps):
            c, q = ts.rk4_step(fn, c, q, T / nsteps)
        Rex = ts.rodrigues(om, T) @ sy.quat_to_rot(q0[0])
        errs.append(np.abs(sy.quat_to_rot(q[0]) - Rex).max())
        assert np.abs(c[0] - v * T).max() < 1e-14
    assert errs[-1] < 1e-7
    assert 12 < errs[0] / errs[1] < 20 and 12 < errs[1] / errs[2] < 20


def test_rk4_fourth_order_on_two_sphere_dynamics():
    # self-convergence as in the paper's RK4 table: ~4 bits gained per halving of dt
    p = 4
    shape = sy.Shape(geo.ellipsoid_coef(1.0, 0.8, 0.6), p)
    FT = np.array([[1.0, 0.2, 0.0, 0.0, 0.5, 1.0], [-1.0, 0.0, 0.3, 0.4, 0.0, 0.0]])

    def velocity(c, q):
        prob = sy.Problem([shape], [0, 0], c, q)
        return sy.solve_dense(prob, FT)[2]

    c0 = np.array([[0.0, 0.0, 0.0], [3.2, 0.3, -0.2]])
    q0 = ts.normalize(np.array([[1.0, 0.0, 0.0, 0.0], [0.8, 0.3, 0.1, -0.2]]))
    T = 4.0
    finals = []
    for nsteps in (2, 4, 8):
        c, q = c0.copy(), q0.copy()
        for _ in range(nsteps):
            c, q = ts.rk4_step(velocity, c, q, T / nsteps)
        finals.append((c, np.array([sy.quat_to_rot(x) for x in q])))
    eC = [np.abs(finals[i][0] - finals[i + 1][0]).max() for i in range(2)]
    eR = [np.abs(finals[i][1] - finals[i + 1][1]).max() for i in range(2)]
    gainC = math.log2(eC[0] / eC[1])
    gainR = math.log2(eR[0] / eR[1])
    assert 3.3 < gainC < 4.8, (eC, gainC)
    assert 3.3 < gainR < 4.8, (eR, gainR)
