"""Pins of the oracle's magnetostatics (§4): the Laplace self operators on a sphere
(diagonal in spherical harmonics), the isolated permeable sphere in a uniform field
(classical closed form: interior field 3 H0/(mu_r + 2), exterior surface field, Maxwell
traction with zero net force and torque), zero net force on any isolated body in a
uniform field, and the induced-dipole force law between two distant spheres (repulsive
across the field, attractive along it)."""
import math

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import magnetic as mg
from oracle import sphharm as sh
from oracle import system as sysm


def sphere_coef(a=1.0):
    k = math.sqrt(4.0 * math.pi / 3.0) * a
    c = np.zeros((3, 4))
    c[0, 3], c[1, 1], c[2, 2] = k, k, k
    return c


def problem(coefs, centres, quats=None, p=8):
    shapes = [sysm.Shape(c, p, with_ops=False) for c in coefs]
    n = len(centres)
    q = np.array([[1.0, 0, 0, 0]] * n) if quats is None else np.asarray(quats)
    sid = list(range(len(coefs))) if len(coefs) == n else [0] * n
    return sysm.Problem(shapes, sid, np.asarray(centres, float), q)


def test_laplace_self_operators_on_a_sphere():
    """S^L Y_l = a/(2l+1) Y_l and K^L Y_l = -Y_l/(2(2l+1)) on a sphere of radius a."""
    a, p = 1.3, 6
    ops = mg.laplace_operators(sphere_coef(a), p)
    g = sh.grid(p)
    Y, _, _ = sh.real_sh(p, g["theta_a"], g["phi_a"])
    for l in range(p):
        for m in (-l, 0, l):
            y = Y[sh.sh_index(l, m)]
            assert np.abs(ops["S"] @ y - a / (2 * l + 1) * y).max() < 1e-12
            assert np.abs(ops["K"] @ y + y / (2 * (2 * l + 1))).max() < 1e-12


def test_derivative_matrices_exact_on_the_band():
    p = 7
    g = sh.grid(p)
    Y, Yt, Yps = sh.real_sh(p, g["theta_a"], g["phi_a"])
    Dt, Dp = mg.derivative_matrices(p)
    for l, m in ((1, 0), (3, -2), (5, 4), (6, 6)):
        k = sh.sh_index(l, m)
        assert np.abs(Dt @ Y[k] - Yt[k]).max() < 1e-11
        assert np.abs(Dp @ Y[k] - Yps[k]).max() < 1e-11


@pytest.mark.parametrize("mu_ratio", [2.0, 10.0, 0.5])
def test_isolated_sphere_in_a_uniform_field(mu_ratio):
    H0 = np.array([0.3, -1.2, 0.7])
    prob = problem([sphere_coef()], [[0.0, 0, 0]])
    mag = mg.Magnetic(prob, mu_ratio, H0)
    q = mag.density()
    eta = (mu_ratio - 1) / (mu_ratio + 1)
    C = 6 * eta / (3 - eta)
    n = prob.Nn
    Hn0 = n @ H0
    assert np.abs(q - C * Hn0).max() < 1e-12
    H = mag.field(q)
    # classical: interior field 3 H0/(mu_r+2); exterior tangential field equals it,
    # exterior normal field is mu_r times its normal part
    Hin = 3.0 * H0 / (mu_ratio + 2.0)
    Ht = Hin[None, :] - (n @ Hin)[:, None] * n
    exact = Ht + mu_ratio * (n @ Hin)[:, None] * n
    assert np.abs(H - exact).max() < 1e-10 * np.abs(H0).max()
    rho = mag.traction(H)
    FT = mag.forces(rho)
    assert np.abs(FT).max() < 1e-11 * np.abs(H0).max() ** 2


def test_no_net_force_on_an_isolated_body_in_a_uniform_field():
    rc = np.zeros(16)
    rc[0] = math.sqrt(4 * math.pi)
    rc[4], rc[6], rc[12] = 0.15, -0.1, 0.08
    coef = geo.radial_to_coef(rc, 10)
    prob = problem([coef], [[0.0, 0, 0]], quats=[[0.9, 0.3, -0.2, 0.1]], p=10)
    mag = mg.Magnetic(prob, 3.0, np.array([0.0, 1.0, 0.4]))
    FT = mag.forces(mag.traction(mag.field(mag.density())))
    assert np.abs(FT[0, :3]).max() < 1e-6
    assert np.abs(FT[0, 3:]).max() > 1e-3      # a non-spherical body feels a torque


def test_two_spheres_follow_the_induced_dipole_force_law():
    """Force on sphere 2 at distance d along x from sphere 1: with dipoles m = 4 pi a^3
    beta H0 (beta = (mu_r - 1)/(mu_r + 2)), F = 3 m^2/(4 pi d^4) x (repulsion) for H0
    along y and -6 m^2/(4 pi d^4) x (attraction) for H0 along x (mu0 = 1)."""
    mu_r, a = 2.0, 1.0
    beta = (mu_r - 1) / (mu_r + 2)
    errs = []
    for d in (5.0, 8.0, 12.0):
        prob = problem([sphere_coef(a)], [[0.0, 0, 0], [d, 0, 0]])
        row = []
        for H0, k in ((np.array([0.0, 1.0, 0.0]), 3.0), (np.array([1.0, 0.0, 0.0]), -6.0)):
            mag = mg.Magnetic(prob, mu_r, H0)
            FT = mag.forces(mag.traction(mag.field(mag.density())))
            m = 4 * math.pi * a**3 * beta
            F = k * m * m / (4 * math.pi * d**4)
            assert np.abs(FT[0, :3] + FT[1, :3]).max() < 1e-8 * abs(F)   # equal and opposite
            row.append(abs(FT[1, 0] / F - 1.0))
            assert np.sign(FT[1, 0]) == np.sign(F)
        errs.append(max(row))
    assert errs[0] < 0.15 and errs[1] < 0.05 and errs[2] < 0.015
    assert errs[2] < errs[1] < errs[0]


def test_magnetic_traction_drives_the_mobility_problem():
    """Two spheres across the field repel: with the Maxwell traction as the incident
    density of the Stokes problem they move apart, symmetrically."""
    prob_s = sysm.Problem([sysm.Shape(sphere_coef(), 8)], [0, 0], np.array([[0.0, 0, 0], [3.0, 0, 0]]),
                          np.array([[1.0, 0, 0, 0]] * 2))
    mag = mg.Magnetic(prob_s, 2.0, np.array([0.0, 1.0, 0.0]))
    rho = mag.traction(mag.field(mag.density()))
    FT = mag.forces(rho)
    _, VW = sysm.solve_dense_density(prob_s, rho)
    assert FT[1, 0] > 0 and VW[1, 0] > 0 and VW[0, 0] < 0
    assert abs(VW[0, 0] + VW[1, 0]) < 1e-12 * abs(VW[1, 0])
    # the same velocities as the mobility problem driven by the net loads alone, up to the
    # difference between the traction and its rigid-body part (small for a sphere)
    V_rigid = sysm.solve_dense(prob_s, FT)[2]
    assert np.abs(VW[:, :3] - V_rigid[:, :3]).max() < 0.05 * np.abs(V_rigid[:, :3]).max()
