"""Pins of the oracle's assembled mobility solve (§2.2, §2.3, §3.2, §3.3)."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import geometry as geo
from oracle import system as sy


def _sphere(p, a=1.0):
    return sy.Shape(geo.ellipsoid_coef(a, a, a), p)


@pytest.mark.parametrize("a", [1.0, 0.6])
def test_isolated_sphere_drag_laws(a):
    # v = F/(6 pi eta a), omega = T/(8 pi eta a^3)  (rho lies in the null space of 1/2 I + K)
    for eta in (1.0, 2.5):
        s = sy.Shape(geo.ellipsoid_coef(a, a, a), 8, eta=eta)
        prob = sy.Problem([s], [0], [[0.5, -1, 2]], [[0.9, 0.1, -0.3, 0.2]], eta=eta)
        FT = np.array([1.0, -0.4, 0.3, 0.2, 0.0, 1.0])
        rho, mu, VW = sy.solve_dense(prob, FT)
        assert np.abs(mu).max() < 1e-13
        assert np.abs(VW[0, :3] - FT[:3] / (6 * math.pi * eta * a)).max() < 1e-13
        assert np.abs(VW[0, 3:] - FT[3:] / (8 * math.pi * eta * a ** 3)).max() < 1e-13


def test_unit_sphere_worked_values():
    prob = sy.Problem([_sphere(8)], [0], [[0, 0, 0]], [[1, 0, 0, 0]])
    _, _, VW = sy.solve_dense(prob, [1, 0, 0, 0, 0, 1])
    assert abs(VW[0, 0] - 0.05305164769729845) < 1e-15
    assert abs(VW[0, 5] - 0.039788735772973836) < 1e-15


def _oberbeck(a, b, c):
    ax = [a, b, c]

    def D(l):
        return math.sqrt((a * a + l) * (b * b + l) * (c * c + l))

    kw = dict(epsabs=1e-15, epsrel=1e-13, limit=400)
    chi = quad(lambda l: 1 / D(l), 0, np.inf, **kw)[0]
    al = [quad(lambda l, ai=ai: 1 / ((ai * ai + l) * D(l)), 0, np.inf, **kw)[0] for ai in ax]
    mt = [(chi + ax[i] ** 2 * al[i]) / (16 * math.pi) for i in range(3)]
    mr = []
    for i in range(3):
        j, k = (i + 1) % 3, (i + 2) % 3
        mr.append(3 * (ax[j] ** 2 * al[j] + ax[k] ** 2 * al[k]) / (16 * math.pi * (ax[j] ** 2 + ax[k] ** 2)))
    return np.array(mt + mr)


def test_oberbeck_jeffery_ellipsoid_mobility():
    # Oberbeck (translation) and Jeffery (rotation) closed forms for a tri-axial ellipsoid
    a, b, c = 1.0, 0.8, 0.6
    ref = _oberbeck(a, b, c)
    errs = []
    for p in (6, 12):
        prob = sy.Problem([sy.Shape(geo.ellipsoid_coef(a, b, c), p)], [0], [[0, 0, 0]], [[1, 0, 0, 0]])
        Mm = sy.mobility_matrix(prob)
        errs.append(np.abs(np.diag(Mm) / ref - 1).max())
        assert np.abs(Mm - np.diag(np.diag(Mm))).max() < 1e-12
    assert errs[1] < 1e-8 and errs[1] < 0.01 * errs[0]


def test_two_spheres_symmetry_and_far_field_coupling():
    prob = sy.Problem([_sphere(8)], [0, 0], [[0, 0, 0], [3, 0, 0]], [[1, 0, 0, 0]] * 2)
    _, mu, VW = sy.solve_dense(prob, [1, 0, 0, 0, 0, 1] + [0] * 6)
    # reflection z -> -z: v_z = 0 and omega_x = omega_y = 0
    assert np.abs(VW[:, [2, 3, 4]]).max() < 1e-14
    # leading-order (Rotne-Prager) coupling: v2.x ~ 0.02456, rotlet v2.y ~ 1/(8 pi 9) = 0.00442
    assert abs(VW[1, 0] - 0.02456) < 0.02 * 0.02456
    assert abs(VW[1, 1] - 1 / (72 * math.pi)) < 0.02 / (72 * math.pi)


def _random_bodies(n, p, seed):
    rng = np.random.default_rng(seed)
    shapes = []
    for i in range(n):
        rc = np.zeros(9)
        rc[0] = math.sqrt(4 * math.pi)
        rc[1:] = 0.05 * rng.standard_normal(8)
        shapes.append(sy.Shape(geo.radial_to_coef(rc, p), p))
    centres = np.array([[0, 0, 0], [2.8, 0.4, -0.3], [0.5, 2.9, 0.6]])[:n]
    quats = rng.standard_normal((n, 4))
    return sy.Problem(shapes, range(n), centres, quats)


def test_mobility_matrix_symmetric_positive_definite():
    prob = _random_bodies(3, 5, 11)
    Mm = sy.mobility_matrix(prob)
    sym = np.abs(Mm - Mm.T).max() / np.abs(Mm).max()
    assert sym < 1e-4
    ev = np.linalg.eigvalsh(0.5 * (Mm + Mm.T))
    assert ev.min() > 0


def test_mobility_symmetry_converges_in_p():
    errs = []
    for p in (4, 8):
        Mm = sy.mobility_matrix(_random_bodies(2, p, 12))
        errs.append(np.abs(Mm - Mm.T).max() / np.abs(Mm).max())
    assert errs[1] < 0.1 * errs[0]


def test_scattered_density_carries_no_force_or_torque():
    prob = _random_bodies(3, 6, 13)
    FT = np.random.default_rng(0).standard_normal(18)
    rho, mu, _ = sy.solve_dense(prob, FT)
    for i in range(prob.n):
        sl = prob.sl(i)
        w = prob.w[sl][:, None]
        rr = prob.X[sl] - prob.c[i]
        # mu: zero net force/torque; rho: exactly F_i, T_i
        assert np.abs(np.sum(w * mu[sl], 0)).max() < 1e-5
        assert np.abs(np.sum(w * np.cross(rr, mu[sl]), 0)).max() < 1e-5
        assert np.abs(np.sum(w * rho[sl], 0) - FT[6 * i:6 * i + 3]).max() < 1e-13
        assert np.abs(np.sum(w * np.cross(rr, rho[sl]), 0) - FT[6 * i + 3:6 * i + 6]).max() < 1e-13


def test_gmres_matches_dense_lu_and_residual():
    prob = _random_bodies(3, 5, 14)
    FT = np.random.default_rng(1).standard_normal(18)
    rho, mu_d, V_d = sy.solve_dense(prob, FT)
    rho2, mu_g, V_g, its = sy.solve_gmres(prob, FT, tol=1e-13)
    b = prob.rhs(rho)
    res = np.linalg.norm(b - prob.apply_A(mu_g)) / np.linalg.norm(b)
    assert res < 1e-13 and its > 3
    assert np.abs(mu_g - mu_d).max() < 1e-11 * np.abs(mu_d).max()
    assert np.abs(V_g - V_d).max() < 1e-11 * np.abs(V_d).max()


def test_linear_in_loads_and_viscosity_scaling():
    prob = _random_bodies(2, 5, 15)
    rng = np.random.default_rng(2)
    F1, F2 = rng.standard_normal(12), rng.standard_normal(12)
    _, _, V1 = sy.solve_dense(prob, F1)
    _, _, V2 = sy.solve_dense(prob, F2)
    _, _, V12 = sy.solve_dense(prob, 2 * F1 - F2)
    assert np.abs(V12 - (2 * V1 - V2)).max() < 1e-12
    shapes = [sy.Shape(s.coef, s.p, eta=3.0) for s in prob.shapes]
    probe = sy.Problem(shapes, prob.shape_id, prob.c, [np.array([1.0, 0, 0, 0])] * 2, eta=3.0)
    probe2 = sy.Problem(prob.shapes, prob.shape_id, prob.c, [np.array([1.0, 0, 0, 0])] * 2)
    _, mu_a, Va = sy.solve_dense(probe, F1)
    _, mu_b, Vb = sy.solve_dense(probe2, F1)
    assert np.abs(mu_a - mu_b).max() < 1e-13
    assert np.abs(3.0 * Va - Vb).max() < 1e-13
