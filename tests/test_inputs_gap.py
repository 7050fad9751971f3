"""The dense configurations (4000 perturbed spheres at 20 %, and their 512-body sibling)
are placed with a true surface gap of 0.1: every pair of surfaces is at least 0.1 apart
and near-contact pairs exist.  The surfaces here come from the oracle's own geometry (the
coordinate functions of the radial shapes and the area centroid of the discrete grid),
not from the generator's placement clouds.  For each pair of bodies within reach, each
surface is sampled on a cap of directions facing the other body, and the closest pair of
samples is refined three times on patches of shrinking size around it."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import geometry as geo
from oracle import sphharm as sh
from oracle import system as sy
from paper_1606_07428_amd import inputs


def _surfaces(w):
    """Per body: coordinate coefficients (3, 36) and the area centroid (oracle, p = 12)."""
    coefs, xcs = [], []
    for kind, d in w["shapes"]:
        coef = geo.radial_to_coef(np.asarray(d, dtype=np.float64), w["p"])
        g = geo.shape_geometry(coef, w["p"])
        coefs.append(coef[:, :36])      # x = r(s) s has degree <= 5
        xcs.append(g["xc"])
    return np.array(coefs), np.array(xcs)


def _points(coefs, xcs, c, R, body, dirs):
    """Lab points of bodies `body` (k,) at unit body-frame directions dirs (k, m, 3)."""
    k, m, _ = dirs.shape
    th = np.arccos(np.clip(dirs[..., 2], -1, 1)).ravel()
    ph = np.arctan2(dirs[..., 1], dirs[..., 0]).ravel()
    Y, _, _ = sh.real_sh(5, th, ph)                      # (36, k m)
    Y = Y.reshape(36, k, m)
    x = np.einsum("kcl,lkm->kmc", coefs[body], Y) - xcs[body][:, None, :]
    return c[body][:, None, :] + np.einsum("kcd,kmd->kmc", R[body], x)


def _cap(axis, half_angle, n):
    """n x n directions on a square patch of the given half-angle about the unit axes (k, 3)."""
    a = np.linspace(-half_angle, half_angle, n)
    A, B = np.meshgrid(a, a, indexing="ij")
    k = len(axis)
    e1 = np.cross(axis, np.where(np.abs(axis[:, :1]) < 0.9, [[1.0, 0, 0]], [[0, 1.0, 0]]))
    e1 /= np.linalg.norm(e1, axis=1)[:, None]
    e2 = np.cross(axis, e1)
    v = axis[:, None, :] + A.reshape(1, -1, 1) * e1[:, None, :] + B.reshape(1, -1, 1) * e2[:, None, :]
    return v / np.linalg.norm(v, axis=2)[..., None]


def _true_gaps(w, reach=0.3, chunk=200):
    """Refined surface distances of the body pairs whose centres are within the sum of
    their largest radii plus `reach`."""
    coefs, xcs = _surfaces(w)
    c = np.asarray(w["centres"], dtype=np.float64)
    R = np.array([sy.quat_to_rot(q) for q in w["quats"]])
    rmax = np.array([np.linalg.norm(geo.shape_geometry(cf, 12)["x"]
                                    - xc[:, None], axis=0).max() for cf, xc in zip(coefs, xcs)]) + 0.02
    pairs = np.array(sorted(cKDTree(c).query_pairs(2 * rmax.max() + reach)))
    D = np.linalg.norm(c[pairs[:, 0]] - c[pairs[:, 1]], axis=1)
    pairs = pairs[D < rmax[pairs[:, 0]] + rmax[pairs[:, 1]] + reach]
    gaps = np.empty(len(pairs))
    for s in range(0, len(pairs), chunk):
        I, J = pairs[s:s + chunk, 0], pairs[s:s + chunk, 1]
        k = len(I)
        u = c[J] - c[I]
        u /= np.linalg.norm(u, axis=1)[:, None]
        # body-frame axes of the caps facing the other body
        ai = np.einsum("kdc,kd->kc", R[I], u)
        aj = np.einsum("kdc,kd->kc", R[J], -u)
        half, n = 0.6, 17
        for _ in range(4):
            di, dj = _cap(ai, half, n), _cap(aj, half, n)
            Pi = _points(coefs, xcs, c, R, I, di)
            Pj = _points(coefs, xcs, c, R, J, dj)
            d2 = np.sum((Pi[:, :, None, :] - Pj[:, None, :, :]) ** 2, axis=3)
            best = d2.reshape(k, -1).argmin(axis=1)
            bi, bj = best // (n * n), best % (n * n)
            gaps[s:s + k] = np.sqrt(d2.reshape(k, -1)[np.arange(k), best])
            ai = di[np.arange(k), bi]
            aj = dj[np.arange(k), bj]
            half *= 0.2
    return gaps


@pytest.mark.parametrize("name", ["dense512", "dense4000"])
def test_true_surface_gap_is_the_stated_one(name):
    w = inputs.workload(name)
    gaps = _true_gaps(w)
    print(f"{name}: {len(gaps)} close pairs, minimum true gap {gaps.min():.4f}, "
          f"pairs under 0.15: {(gaps < 0.15).sum()}, under 0.2: {(gaps < 0.2).sum()}")
    # no pair closer than the stated gap (up to the placement clouds' discreteness) ...
    assert gaps.min() >= 0.1 - 3e-3
    # ... and the near-contact pairs the configuration states do occur
    assert gaps.min() <= 0.105
    assert (gaps < 0.15).sum() >= len(w["shapes"]) // 50


def test_bounding_gap_configurations_use_tight_radii():
    """random64 (gap 0.5 between bounding spheres): the bounding radius is within 0.01 of
    the largest centroid-to-node distance of the oracle's geometry at a fine grid, and the
    closest pair of bounding spheres is 0.5 apart (not inflated by a loose bound)."""
    w = inputs.workload("random64")
    coefs, xcs = _surfaces(w)
    rb = []
    for cf, xc, (kind, d) in zip(coefs, xcs, w["shapes"]):
        g = geo.shape_geometry(cf, 48)
        r_true = np.linalg.norm(g["x"] - xc[:, None], axis=0).max()
        r_gen = inputs.tight_radius(kind, d)
        assert r_true - 1e-3 <= r_gen <= r_true + 0.01
        rb.append(r_gen)
    rb = np.array(rb)
    c = np.asarray(w["centres"])
    D = np.linalg.norm(c[:, None] - c[None], axis=2) - rb[:, None] - rb[None]
    np.fill_diagonal(D, np.inf)
    assert 0.5 <= D.min() < 0.6
