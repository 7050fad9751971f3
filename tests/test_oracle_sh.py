"""Pins of the oracle's spherical-harmonic machinery (§3) against mathematics and
library routines that do not share its code."""
import math

import numpy as np
import pytest
import scipy.special as sps

from oracle import sphharm as sh


@pytest.mark.parametrize("n", [1, 2, 5, 9, 17, 33])
def test_gauss_legendre_exactness(n):
    t, w = sh.gauss_legendre(n)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * t ** k) - exact) < 1e-14
    if n == 1:
        assert abs(t[0]) < 1e-15


def test_gl2_nodes_closed_form():
    t, w = sh.gauss_legendre(2)
    assert np.allclose(t, [-1 / math.sqrt(3), 1 / math.sqrt(3)], atol=1e-16)
    assert np.allclose(w, [1.0, 1.0], atol=1e-15)


def _scipy_real(l, m, th, ph):
    k = abs(m)
    c = sps.sph_harm_y(l, k, th, ph) * (-1) ** k   # remove the Condon-Shortley phase
    if m == 0:
        return c.real
    return math.sqrt(2) * (c.real if m > 0 else c.imag)


def test_real_sh_matches_scipy():
    rng = np.random.default_rng(0)
    th = rng.uniform(0, math.pi, 50)
    ph = rng.uniform(-math.pi, 2 * math.pi, 50)
    L = 16
    Y, _, _ = sh.real_sh(L, th, ph)
    for l in range(L + 1):
        for m in range(-l, l + 1):
            ref = _scipy_real(l, m, th, ph)
            assert np.abs(Y[sh.sh_index(l, m)] - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


def test_derivatives_against_finite_differences():
    rng = np.random.default_rng(1)
    th = rng.uniform(0.2, math.pi - 0.2, 20)
    ph = rng.uniform(0, 2 * math.pi, 20)
    L, h = 10, 1e-5
    _, Yt, Yps = sh.real_sh(L, th, ph)
    Yp, _, _ = sh.real_sh(L, th + h, ph)
    Ym, _, _ = sh.real_sh(L, th - h, ph)
    assert np.abs((Yp - Ym) / (2 * h) - Yt).max() < 1e-7
    Yp, _, _ = sh.real_sh(L, th, ph + h)
    Ym, _, _ = sh.real_sh(L, th, ph - h)
    assert np.abs((Yp - Ym) / (2 * h) / np.sin(th) - Yps).max() < 1e-7


def test_pole_limits_are_regular():
    # at the pole the pole-regular quantities must equal their limits from nearby
    L = 9
    for th0 in (0.0, math.pi):
        for ph in (0.0, 1.3):
            Y0, Yt0, Yps0 = sh.real_sh(L, np.array([th0]), np.array([ph]))
            eps = 1e-7 if th0 == 0.0 else -1e-7
            Y1, Yt1, Yps1 = sh.real_sh(L, np.array([th0 + eps]), np.array([ph]))
            assert np.all(np.isfinite(Yps0))
            assert np.abs(Y0 - Y1).max() < 1e-5
            assert np.abs(Yt0 - Yt1).max() < 1e-5
            assert np.abs(Yps0 - Yps1).max() < 1e-5


@pytest.mark.parametrize("p", [2, 3, 8, 12])
def test_forward_is_left_inverse_of_synthesis(p):
    g = sh.grid(p)
    F = sh.forward_matrix(p)
    YB = sh.synthesis_matrix(p, g["theta_a"], g["phi_a"])
    assert F.shape == (p * p + 2 * p, (p + 1) * 2 * p)
    assert np.abs(F @ YB.T - np.eye(F.shape[0])).max() < 1e-13


def test_dropped_mode_vanishes_on_grid():
    p = 6
    g = sh.grid(p)
    Y, _, _ = sh.real_sh(p, g["theta_a"], g["phi_a"])
    assert np.abs(Y[sh.sh_index(p, -p)]).max() < 1e-13


def test_quadrature_orthonormality_below_nyquist():
    # the GL(p+1) x trapezoid(2p) rule integrates Y_a Y_b exactly when |m_a|+|m_b| < 2p
    p = 7
    g = sh.grid(p)
    Y, _, _ = sh.real_sh(p - 1, g["theta_a"], g["phi_a"])
    w = (math.pi / p) * g["lam_a"]
    G = (Y * w) @ Y.T
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-13
