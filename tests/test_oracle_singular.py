"""Pins of the oracle's weakly singular self operators (§3, §3.1)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import geometry as geo
from oracle import singular as sg
from oracle import sphharm as sh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _comp_major(v):
    """(3, M) field -> vector with index c*M + a."""
    return np.asarray(v).reshape(-1)


@pytest.mark.parametrize("a", [1.0, 1.7])
@pytest.mark.parametrize("p,ps", [(4, 5), (6, 12), (8, 16)])
def test_sphere_rigid_modes_exact(a, p, ps):
    # translating / rotating sphere (drag laws of a sphere of radius a):
    #   S[c] = (2a/3) c,  K[c] = -c/2,  S[Om x n] = (a/3)(Om x n)... written as (1/3) Om x x
    #   K[Om x n] = -(1/2) Om x n     (exact: circle averages are low-degree polynomials)
    coef = geo.ellipsoid_coef(a, a, a)
    ops = sg.singular_operators(coef, p, ps)
    G = geo.shape_geometry(coef, p)
    M = G["grid"]["M"]
    c = np.array([0.3, -1.2, 0.7])
    v = np.repeat(c, M)
    assert np.abs(ops["S"] @ v - (2 * a / 3) * v).max() < 2e-13 * a
    assert np.abs(ops["K"] @ v + 0.5 * v).max() < 2e-13
    Om = np.array([0.4, 0.1, -0.9])
    rot_n = np.cross(Om[:, None], G["n"], axis=0)
    rot_x = np.cross(Om[:, None], G["x"], axis=0)
    assert np.abs(ops["S"] @ _comp_major(rot_n) - _comp_major(rot_x) / 3.0).max() < 2e-13 * a
    assert np.abs(ops["K"] @ _comp_major(rot_n) + 0.5 * _comp_major(rot_n)).max() < 2e-13


def _perturbed(p, seed=2, sig=0.05):
    rng = np.random.default_rng(seed)
    rc = np.zeros(16)
    rc[0] = math.sqrt(4 * math.pi)
    rc[1:] = sig * rng.standard_normal(15)
    return geo.radial_to_coef(rc, p)


def test_normal_identities_converge_on_perturbed_body():
    # S[n] = 0 (the Stokeslet is divergence free) and K[n] = n/2 for any closed surface
    errS, errK = [], []
    for p in (5, 8, 12):
        coef = _perturbed(p)
        ops = sg.singular_operators(coef, p)
        n = _comp_major(geo.shape_geometry(coef, p)["n"])
        errS.append(np.abs(ops["S"] @ n).max())
        errK.append(np.abs(ops["K"] @ n - 0.5 * n).max())
    assert errS[0] > errS[-1] and errK[0] > errK[-1]
    assert errS[-1] < 1e-6 and errK[-1] < 1e-6
    assert errS[1] < 0.2 * errS[0] and errK[1] < 0.2 * errK[0]


def test_rule_matches_adaptive_bruteforce():
    with open(os.path.join(GOLDEN, "singular_bruteforce.json")) as f:
        gold = json.load(f)
    p = gold["case"]["p"]
    coef = geo.radial_to_coef(np.array(gold["radial_coef"]), p)
    cb = np.array(gold["band_coef"])
    g = sh.grid(p)
    mug = cb @ sh.synthesis_matrix(p, g["theta_a"], g["phi_a"])
    targets = [int(t) for t in gold["values"]]
    errs = {}
    for ps in (2 * p, 6 * p):
        rows = sg.singular_rows(coef, p, ps, targets)
        e = 0.0
        for i, t in enumerate(targets):
            for kind in "SK":
                ref = np.array(gold["values"][str(t)][kind])
                val = np.einsum("ijA,jA->i", rows[kind][i], mug)
                e = max(e, np.abs(val - ref).max() / np.abs(ref).max())
        errs[ps] = e
    # geometric convergence in p_s; tolerance stated at p_s = 2p
    assert errs[2 * p] < 2e-4
    assert errs[6 * p] < 1e-11


def test_rotation_covariance_grid_symmetry():
    # rotating the body by R_z(pi/p) permutes the grid: A' = P (R (x) I) A (R^T (x) I) P^T
    p = 6
    coef = _perturbed(p, seed=4, sig=0.06)
    g = sh.grid(p)
    M = g["M"]
    R = sg.rot_z(math.pi / p)
    x, _, _ = geo.eval_surface(coef, g["theta_a"], g["phi_a"])
    # x'(node (j,k)) = R x(node (j,k-1))
    src = g["j_a"] * 2 * p + (g["k_a"] - 1) % (2 * p)
    xr = R @ x[:, src]
    coef_r = np.zeros_like(coef)
    coef_r[:, sh.band_indices(p)] = xr @ sh.forward_matrix(p).T
    A = sg.singular_operators(coef, p)
    Ar = sg.singular_operators(coef_r, p)
    for kind in "SK":
        A4 = A[kind].reshape(3, M, 3, M)
        pred = np.einsum("ce,eafb,gf->cagb", R, A4[:, src][:, :, :, src], R).reshape(3 * M, 3 * M)
        assert np.abs(Ar[kind] - pred).max() < 1e-12 * np.abs(pred).max()
