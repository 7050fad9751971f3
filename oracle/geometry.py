"""Surface geometry of one genus-zero body, FP64 oracle (§2.2 and §3).

Test infrastructure only (see ``oracle/__init__``).

A shape is given by the real-SH coefficients a[3, (L+1)^2] of its coordinate
functions x(theta, phi) (the truncated expansion of §3), L <= p - 1.  At the grid of
``sphharm.grid`` it yields the points, the outward normal, the Jacobian
J = |x_theta x (x_phi / sin theta)| = W / sin(theta) with W the area element of §3,
the smooth quadrature weights w = (pi/p) lam_j J (the §3 rule with 2p azimuths),
the area |Gamma|, the area centroid x^c and the moment-of-inertia tensor tau of
§2.2.  The centroid is read as the area centroid (the zero-torque claims of §2.2
need the first area moment about x^c to vanish).
"""
import math

import numpy as np

from . import sphharm as sh


def eval_surface(coef, theta, phi):
    """x, x_theta, x_phi/sin(theta) at the points (theta, phi); coef (3, nc)."""
    L = int(round(math.sqrt(coef.shape[1]))) - 1
    Y, Yt, Yps = sh.real_sh(L, theta, phi)
    x = np.tensordot(coef, Y, axes=(1, 0))
    xt = np.tensordot(coef, Yt, axes=(1, 0))
    xps = np.tensordot(coef, Yps, axes=(1, 0))
    return x, xt, xps


def surface_frame(coef, theta, phi):
    """Points x, unit outward normal n and Jacobian J = W / sin(theta)."""
    x, xt, xps = eval_surface(coef, theta, phi)
    c = np.cross(xt, xps, axis=0)
    J = np.sqrt(np.sum(c * c, axis=0))
    return x, c / J, J


def radial_to_coef(rc, p):
    """Coordinate coefficients of x = r(s) s, r(s) = sum rc_lm Y_lm(s), s the unit
    vector.  Computed by the exact forward transform of the grid values; exact when
    the degree of x (deg r + 1) is below p.  Returns (3, (p+1)^2)."""
    Lr = int(round(math.sqrt(len(rc)))) - 1
    if Lr + 1 >= p:
        raise ValueError("radial degree + 1 must be below p")
    g = sh.grid(p)
    Y, _, _ = sh.real_sh(Lr, g["theta_a"], g["phi_a"])
    r = rc @ Y
    st, ct = np.sin(g["theta_a"]), np.cos(g["theta_a"])
    s = np.stack([st * np.cos(g["phi_a"]), st * np.sin(g["phi_a"]), ct])
    xg = r[None, :] * s
    F = sh.forward_matrix(p)
    cB = xg @ F.T
    coef = np.zeros((3, sh.n_modes(p)))
    coef[:, sh.band_indices(p)] = cB
    return coef


def ellipsoid_coef(a, b, c):
    """Coordinate coefficients of x = (a sin t cos f, b sin t sin f, c cos t).

    sin t cos f = sqrt(4 pi / 3) Y_11, sin t sin f = sqrt(4 pi/3) Y_1-1 and
    cos t = sqrt(4 pi / 3) Y_10 in the real basis of ``sphharm``."""
    k = math.sqrt(4.0 * math.pi / 3.0)
    coef = np.zeros((3, 4))
    coef[0, sh.sh_index(1, 1)] = a * k
    coef[1, sh.sh_index(1, -1)] = b * k
    coef[2, sh.sh_index(1, 0)] = c * k
    return coef


def shape_geometry(coef, p):
    """All per-shape grid quantities (body frame, before recentring is applied to
    the points: ``r`` holds x - x^c).

    Returns dict: x (3,M), n (3,M), J (M), w (M), area, xc (3), r (3,M), tau (3,3).
    """
    g = sh.grid(p)
    x, n, J = surface_frame(coef, g["theta_a"], g["phi_a"])
    w = (math.pi / p) * g["lam_a"] * J
    area = float(np.sum(w))
    xc = (x * w[None, :]).sum(axis=1) / area
    r = x - xc[:, None]
    rr = np.sum(r * r, axis=0)
    tau = np.eye(3) * np.sum(w * rr) - (r * w[None, :]) @ r.T
    return {"x": x, "n": n, "J": J, "w": w, "area": area, "xc": xc, "r": r,
            "tau": tau, "grid": g, "coef": coef, "p": p}
