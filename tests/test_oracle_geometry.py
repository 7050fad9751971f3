"""Pins of the oracle's surface geometry (§2.2, §3) against closed forms."""
import math

import numpy as np
import pytest
import scipy.special as sps

from oracle import geometry as geo


@pytest.mark.parametrize("a", [1.0, 0.7, 2.5])
@pytest.mark.parametrize("p", [2, 5, 8])
def test_sphere_closed_forms(a, p):
    G = geo.shape_geometry(geo.ellipsoid_coef(a, a, a), p)
    assert abs(G["area"] - 4 * math.pi * a * a) < 1e-13 * a * a
    assert np.abs(G["tau"] - (8 * math.pi / 3) * a ** 4 * np.eye(3)).max() < 1e-12 * a ** 4
    assert np.abs(G["J"] - a * a).max() < 1e-13 * a * a
    assert np.abs(G["xc"]).max() < 1e-14 * a
    # outward unit normal equals x/a on a sphere
    assert np.abs(G["n"] - G["x"] / a).max() < 1e-14
    vol = np.sum(G["w"] * np.sum(G["x"] * G["n"], axis=0)) / 3.0
    assert abs(vol - 4 * math.pi * a ** 3 / 3) < 1e-12 * a ** 3


def _ellipsoid_area(a, b, c):
    # a >= b >= c; Legendre's form with incomplete elliptic integrals
    phi = math.acos(c / a)
    k2 = a * a * (b * b - c * c) / (b * b * (a * a - c * c))
    E, F = sps.ellipeinc(phi, k2), sps.ellipkinc(phi, k2)
    s = math.sin(phi)
    return 2 * math.pi * c * c + 2 * math.pi * a * b / s * (E * s * s + F * math.cos(phi) ** 2)


def test_ellipsoid_volume_and_area_converge():
    a, b, c = 1.0, 0.8, 0.6
    exact_area = _ellipsoid_area(a, b, c)
    errs = []
    for p in (4, 8, 16):
        G = geo.shape_geometry(geo.ellipsoid_coef(a, b, c), p)
        vol = np.sum(G["w"] * np.sum(G["x"] * G["n"], axis=0)) / 3.0
        assert abs(vol - 4 * math.pi * a * b * c / 3) < 1e-12
        errs.append(abs(G["area"] - exact_area))
        # symmetric body: centroid at the origin, tau diagonal
        assert np.abs(G["xc"]).max() < 1e-14
        assert np.abs(G["tau"] - np.diag(np.diag(G["tau"]))).max() < 1e-13
    assert errs[-1] < 1e-10
    assert errs[0] > errs[1] > errs[2]


def test_radial_conversion_reproduces_radius():
    rng = np.random.default_rng(5)
    rc = np.zeros(25)
    rc[0] = math.sqrt(4 * math.pi)
    rc[1:] = 0.03 * rng.standard_normal(24)
    p = 8
    coef = geo.radial_to_coef(rc, p)
    th = rng.uniform(0, math.pi, 40)
    ph = rng.uniform(0, 2 * math.pi, 40)
    from oracle import sphharm as sh
    Y, _, _ = sh.real_sh(4, th, ph)
    r = rc @ Y
    x, _, _ = geo.eval_surface(coef, th, ph)
    s = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    assert np.abs(x - r * s).max() < 1e-13
