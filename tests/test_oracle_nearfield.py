"""Pins of the oracle's near-singular rule (upsampling, §3).

The rule is pinned against closed forms and identities that hold for the exact
layer potentials: the exterior flow and stress of a translating sphere (the
single layer of a uniform density), the vanishing of the layer potentials of the
normal field off the surface, exact interpolation of band-limited data, and the
agreement of the operator's matrix form with its matrix-free form.
"""
import math

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import nearfield as nf
from oracle import sphharm as sh
from oracle import system as sysm


def unit_sphere_coef(a=1.0):
    k = math.sqrt(4.0 * math.pi / 3.0)
    c = np.zeros((3, 4))
    c[0, 3], c[1, 1], c[2, 2] = a * k, a * k, a * k
    return c


def translating_sphere_velocity(x, c, a, eta=1.0):
    """Single layer of the uniform density c on a sphere of radius a centred at 0,
    at exterior points x (n, 3): the flow of a sphere translating with velocity
    U = 2 a c / (3 eta) (force 6 pi eta a U = 4 pi a^2 c on the fluid)."""
    r = np.linalg.norm(x, axis=1)[:, None]
    xc = (x @ c)[:, None]
    k = 2.0 * a / (3.0 * eta)
    return k * (0.75 * a * (c[None, :] / r + xc * x / r**3)
                + 0.25 * a**3 * (c[None, :] / r**3 - 3.0 * xc * x / r**5))


def translating_sphere_pressure(x, c, a):
    """Pressure of the same single layer: (1/4pi) c . int (x-y)/|x-y|^3 dS_y
    = a^2 (c . x) / r^3 outside the sphere."""
    r = np.linalg.norm(x, axis=1)
    return a * a * (x @ c) / r**3


def two_spheres(gap, p, upsample, a=1.0):
    shape = sysm.Shape(unit_sphere_coef(a), p, with_ops=False)
    cen = np.array([[0.0, 0.0, 0.0], [2 * a + gap, 0.1, -0.05]])
    quats = np.array([[1.0, 0, 0, 0], [0.9, 0.1, -0.3, 0.2]])
    quats /= np.linalg.norm(quats, axis=1)[:, None]
    return sysm.Problem([shape], [0, 0], cen, quats, upsample=upsample)


def test_interpolation_exact_for_band_limited_data():
    """The band-limited interpolant reproduces every function of the band B_p exactly
    at the fine nodes (the forward transform is the exact left inverse of synthesis)."""
    rng = np.random.default_rng(5)
    for p, p_u in ((4, 9), (6, 12), (8, 20)):
        g, gu = sh.grid(p), sh.grid(p_u)
        cB = rng.standard_normal(len(sh.band_indices(p)))
        f = sh.synthesis_matrix(p, g["theta_a"], g["phi_a"]).T @ cB
        fu = sh.synthesis_matrix(p, gu["theta_a"], gu["phi_a"]).T @ cB
        U = nf.interp_matrix(p, p_u)
        assert np.abs(U @ f - fu).max() < 1e-12 * np.abs(fu).max()
        assert np.abs(U @ np.ones(g["M"]) - 1.0).max() < 1e-13


def test_fine_geometry_of_a_sphere():
    a = 1.3
    for p_u in (10, 17):
        fg = nf.fine_geometry(unit_sphere_coef(a), np.zeros(3), p_u)
        assert abs(fg["w"].sum() - 4 * math.pi * a * a) < 1e-12
        assert abs(fg["R"] - a) < 1e-13
        assert fg["M"] == 2 * p_u * (p_u + 1)


def test_near_matrix_by_hand():
    """Unit spheres at x = 0, 3, 10 with p = 8: h = sqrt(4 pi / 144); the first pair's
    gap 1 is below kappa h exactly when kappa > 1 / h = 3.385..."""
    shape = sysm.Shape(unit_sphere_coef(), 8, with_ops=False)
    cen = np.array([[0.0, 0, 0], [3.0, 0, 0], [10.0, 0, 0]])
    q = np.array([[1.0, 0, 0, 0]] * 3)
    h = math.sqrt(4 * math.pi / 144)
    assert abs(1 / h - 3.3851) < 1e-4
    near3 = sysm.Problem([shape], [0, 0, 0], cen, q, upsample=(16, 3.3)).near
    near4 = sysm.Problem([shape], [0, 0, 0], cen, q, upsample=(16, 3.5)).near
    assert not near3.any()
    expect = np.zeros((3, 3), dtype=bool)
    expect[0, 1] = expect[1, 0] = True
    assert (near4 == expect).all()


@pytest.mark.parametrize("gap", [0.15, 0.3])
def test_upsampled_stokeslet_sum_matches_translating_sphere(gap):
    """S_far of a uniform density on sphere 1 at the nodes of sphere 0 (distance
    ~gap from sphere 1) against the exterior flow of a translating sphere."""
    c = np.array([0.3, -0.7, 0.5])
    errs = {}
    for up in (None, (24, 5.0), (32, 5.0)):
        prob = two_spheres(gap, 8, up)
        sig = np.zeros((prob.N, 3))
        sig[prob.sl(1)] = c
        u = prob.S_far(sig, targets=np.arange(prob.M))
        exact = translating_sphere_velocity(prob.X[:prob.M] - prob.c[1], c, 1.0)
        errs[up] = np.abs(u - exact).max() / np.abs(exact).max()
    assert errs[(24, 5.0)] < errs[None] / 20
    assert errs[(32, 5.0)] < errs[(24, 5.0)]
    assert errs[(32, 5.0)] < (3e-5 if gap < 0.2 else 2e-7)


def test_upsampled_traction_sum_matches_stress_of_translating_sphere():
    """K_far (the traction of the Stokeslet sum on the target's normal) against
    [-p I + grad u + grad u^T] N of the translating-sphere flow (eta = 1),
    gradients by central differences of the closed form."""
    c = np.array([-0.4, 0.2, 0.9])
    prob = two_spheres(0.25, 8, (32, 5.0))
    mu = np.zeros((prob.N, 3))
    mu[prob.sl(1)] = c
    tgt = np.arange(0, prob.M, 5)
    y = prob.K_far(mu, targets=tgt)
    x = prob.X[tgt] - prob.c[1]
    Nt = prob.Nn[tgt]
    hh = 1e-5
    grad = np.zeros((len(tgt), 3, 3))  # grad[a, i, k] = d u_i / d x_k
    for k in range(3):
        e = np.zeros(3)
        e[k] = hh
        grad[:, :, k] = (translating_sphere_velocity(x + e, c, 1.0)
                         - translating_sphere_velocity(x - e, c, 1.0)) / (2 * hh)
    pres = translating_sphere_pressure(x, c, 1.0)
    sigma = -pres[:, None, None] * np.eye(3)[None] + grad + np.transpose(grad, (0, 2, 1))
    exact = np.einsum("aik,ak->ai", sigma, Nt)
    err_up = np.abs(y - exact).max() / np.abs(exact).max()
    plain = two_spheres(0.25, 8, None).K_far(mu, targets=tgt)
    err_plain = np.abs(plain - exact).max() / np.abs(exact).max()
    assert err_up < 1e-5
    assert err_up < err_plain / 50


def test_normal_field_gives_zero_off_the_surface():
    """K_far[n_j] = 0 and S_far[n_j] = 0 at targets off Gamma_j (for the exact
    potentials); on a perturbed body close to another one the upsampled rule is far
    closer to zero than the plain one."""
    rc = np.zeros(16)
    rc[0] = math.sqrt(4 * math.pi)
    rc[5], rc[10], rc[14] = 0.08, -0.05, 0.04
    coef = geo.radial_to_coef(rc, 8)
    shape = sysm.Shape(coef, 8, with_ops=False)
    cen = np.array([[0.0, 0, 0], [2.45, 0.2, 0.1]])
    q = np.array([[1.0, 0, 0, 0], [0.8, 0.2, 0.5, -0.1]])
    q /= np.linalg.norm(q, axis=1)[:, None]
    vals = {}
    for up in (None, (32, 5.0)):
        prob = sysm.Problem([shape], [0, 0], cen, q, upsample=up)
        nvec = np.zeros((prob.N, 3))
        nvec[prob.sl(1)] = prob.Nn[prob.sl(1)]
        t = np.arange(prob.M)
        vals[up] = (np.abs(prob.K_far(nvec, targets=t)).max(), np.abs(prob.S_far(nvec, targets=t)).max())
    assert vals[(32, 5.0)][0] < vals[None][0] / 20
    assert vals[(32, 5.0)][1] < vals[None][1] / 20
    assert vals[(32, 5.0)][0] < 1e-4 and vals[(32, 5.0)][1] < 1e-5


def test_dense_matrix_matches_apply_with_upsampling():
    rng = np.random.default_rng(9)
    rc = np.zeros(9)
    rc[0] = math.sqrt(4 * math.pi)
    rc[4], rc[7] = 0.06, -0.04
    shapes = [sysm.Shape(geo.radial_to_coef(rc, 5), 5), sysm.Shape(unit_sphere_coef(0.9), 5)]
    cen = np.array([[0.0, 0, 0], [2.3, 0.3, 0.0], [0.4, 2.4, 0.3], [6.0, 6.0, 6.0]])
    q = rng.standard_normal((4, 4))
    q /= np.linalg.norm(q, axis=1)[:, None]
    prob = sysm.Problem(shapes, [0, 1, 0, 1], cen, q, upsample=(11, 5.0))
    assert prob.near.sum() >= 4 and not prob.near[3].any() and not prob.near[:, 3].any()
    mu = rng.standard_normal((prob.N, 3))
    A = prob.dense_matrix()
    y1 = (A @ mu.reshape(-1)).reshape(prob.N, 3)
    y2 = prob.apply_A(mu)
    assert np.abs(y1 - y2).max() < 1e-12 * np.abs(y2).max()


def test_upsampling_moves_the_mobility_toward_the_converged_one():
    """Two close spheres (gap 0.2): the p = 8 mobility with upsampling is closer to
    the converged (p = 12, upsampled) one than the plain p = 8 mobility, and closer
    than even the plain p = 12 one, whose error is dominated by the near pair."""
    FT = np.array([[1.0, 0.2, -0.3, 0.1, 0.0, 0.4], [0.0, 0.0, 0.0, 0.0, 0.0, 0.0]])

    def vel(p, up):
        shape = sysm.Shape(unit_sphere_coef(), p)
        cen = np.array([[0.0, 0, 0], [2.2, 0.0, 0.0]])
        prob = sysm.Problem([shape], [0, 0], cen, np.array([[1.0, 0, 0, 0]] * 2), upsample=up)
        return sysm.solve_dense(prob, FT)[2]

    ref = vel(12, (36, 5.0))
    e_plain8 = np.abs(vel(8, None) - ref).max()
    e_plain12 = np.abs(vel(12, None) - ref).max()
    e_up8 = np.abs(vel(8, (24, 5.0)) - ref).max()
    assert e_up8 < e_plain8 / 5
    assert e_up8 < e_plain12 / 5
