"""Weakly singular self-interaction operators by spherical-grid rotation, FP64 oracle.

Test infrastructure only (see ``oracle/__init__``).

§3 computes the diagonal blocks S_ii and K_ii with the rotation-based quadrature
of Gimbutas and Veerapaneni (their Theorem 1): the spherical grid is rotated so that
the target becomes the pole, where the integrand divided by the kernel singularity
is smooth.  The rule itself is not printed in the paper; the reading used here:

  For target node t with unit-sphere point s_t take Q_t = R_z(phi_t) R_y(theta_t)
  (so Q_t e_z = s_t) and the rotated nodes s_jk = Q_t s'_jk, s'_jk the
  GL(p_s+1) x trapezoid(2 p_s) grid.  Since 1/|e_z - s'| = 1/sqrt(2(1-t'))
  = sum_nu P_nu(t') (Legendre generating function at h = 1), a circle-averaged
  integrand of degree <= p_s in t' is integrated exactly by

     int k(x_t, y) mu(y) dS_y  ~=  sum_jk W_jk  k(x_t, x(s_jk)) J(s_jk) mu~(s_jk),
     W_jk = (pi/p_s) lam'_j  [sum_{nu=0}^{p_s} P_nu(t'_j)]  sqrt(2 (1 - t'_j)),

  where mu~ is the band-limited interpolant sum_{b in B_p} (F mu)_b Y_b of the
  grid density and J = W/sin(theta) maps the unit sphere onto the surface.

The traction kernel n_t . T is O(1/r) on a smooth surface (r . n_t = O(r^2)), so
K_ii is an ordinary weakly singular integral, evaluated by the same rule; no
principal value treatment is needed.

Operators are returned in the body frame, component-major within the body:
row / column index c*M + a for component c of node a.  Lab-frame blocks follow
from the rotation covariance of §3.1: A_lab = (R (x) I_M) A (R^T (x) I_M).
"""
import math

import numpy as np

from . import geometry as geo
from . import sphharm as sh


def rot_y(t):
    c, s = math.cos(t), math.sin(t)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def rot_z(f):
    c, s = math.cos(f), math.sin(f)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def rotated_rule(ps):
    """Unit-sphere nodes s' (3, M_s) of the GL(ps+1) x trapezoid(2ps) grid and the
    singular weights W (without the Jacobian)."""
    t, lam = sh.gauss_legendre(ps + 1)
    # sum_{nu=0}^{ps} P_nu(t) by the Legendre three-term recurrence
    Pm1, P0 = np.zeros_like(t), np.ones_like(t)
    S = P0.copy()
    for nu in range(1, ps + 1):
        Pn = ((2 * nu - 1) * t * P0 - (nu - 1) * Pm1) / nu
        Pm1, P0 = P0, Pn
        S += Pn
    nphi = 2 * ps
    phi = math.pi * np.arange(nphi) / ps
    tt = np.repeat(t, nphi)
    ff = np.tile(phi, ps + 1)
    st = np.sqrt(1.0 - tt * tt)
    nodes = np.stack([st * np.cos(ff), st * np.sin(ff), tt])
    W = (math.pi / ps) * np.repeat(lam * S * np.sqrt(2.0 * (1.0 - t)), nphi)
    return nodes, W


def kernel_stokeslet(r, eta):
    """G(r)/eta with G the Stokeslet of §2.1; r (3, m) -> (3, 3, m)."""
    d2 = np.sum(r * r, axis=0)
    d = np.sqrt(d2)
    k = np.einsum("im,jm->ijm", r, r) / (d2 * d)[None, None, :]
    k[0, 0] += 1.0 / d
    k[1, 1] += 1.0 / d
    k[2, 2] += 1.0 / d
    return k / (8.0 * math.pi * eta)


def kernel_traction(r, nt):
    """n_t . T with T_ijk = -(3/4pi) r_i r_j r_k / |r|^5 (§2.1): the 3x3 matrix
    acting on the density, -(3/4pi) (r . n_t) r r^T / |r|^5; r (3, m) -> (3, 3, m)."""
    d2 = np.sum(r * r, axis=0)
    rn = nt @ r
    fac = -(3.0 / (4.0 * math.pi)) * rn / (d2 * d2 * np.sqrt(d2))
    return np.einsum("im,jm->ijm", r, r) * fac[None, None, :]


def singular_rows(coef, p, ps, targets, eta=1.0, which=("S", "K")):
    """Rows of the self operators for the listed target nodes.

    Returns dict kind -> array (len(targets), 3, 3, M): entry [i, c, c', a] is the
    weight of component c' of node a in component c of the integral at target i.
    """
    g = sh.grid(p)
    M = g["M"]
    F = sh.forward_matrix(p)
    B = sh.band_indices(p)
    xg, ng, _ = geo.surface_frame(coef, g["theta_a"], g["phi_a"])
    nodes, W = rotated_rule(ps)
    out = {k: np.zeros((len(targets), 3, 3, M)) for k in which}
    for i, t in enumerate(targets):
        Q = rot_z(g["phi_a"][t]) @ rot_y(g["theta_a"][t])
        s = Q @ nodes
        th = np.arccos(np.clip(s[2], -1.0, 1.0))
        ph = np.arctan2(s[1], s[0])
        Yall, Yt, Yps = sh.real_sh(p, th, ph)
        L = int(round(math.sqrt(coef.shape[1]))) - 1
        x = np.tensordot(coef, Yall[: sh.n_modes(L)], axes=(1, 0))
        xt = np.tensordot(coef, Yt[: sh.n_modes(L)], axes=(1, 0))
        xps = np.tensordot(coef, Yps[: sh.n_modes(L)], axes=(1, 0))
        J = np.linalg.norm(np.cross(xt, xps, axis=0), axis=0)
        r = xg[:, t][:, None] - x
        wq = W * J
        YB = Yall[B]
        for kind in which:
            if kind == "S":
                kmat = kernel_stokeslet(r, eta)
            else:
                kmat = kernel_traction(r, ng[:, t])
            C = np.einsum("ijq,q,bq->ijb", kmat, wq, YB)
            out[kind][i] = C @ F
    return out


def singular_operators(coef, p, ps=None, eta=1.0, which=("S", "K")):
    """Dense body-frame self operators S0, K0 (3M x 3M, index c*M + a)."""
    ps = 2 * p if ps is None else ps
    M = (p + 1) * 2 * p
    rows = singular_rows(coef, p, ps, range(M), eta, which)
    ops = {}
    for kind, R in rows.items():
        # R[t, c, c', a] -> A[c*M + t, c'*M + a]
        ops[kind] = np.transpose(R, (1, 0, 2, 3)).reshape(3 * M, 3 * M)
    return ops


def L_operator(geom):
    """Body-frame matrix of L_i of §2.3 on the discrete grid:
    L[mu](x_a) = sum_b w_b mu_b + (sum_b w_b r_b x mu_b) x r_a,
    i.e. block (a, b) = w_b (I - [r_a]x [r_b]x)."""
    r, w = geom["r"], geom["w"]
    M = r.shape[1]

    def cross_mat(v):
        z = np.zeros(v.shape[1])
        return np.array([[z, -v[2], v[1]], [v[2], z, -v[0]], [-v[1], v[0], z]])

    Cr = cross_mat(r)                      # (3,3,M)
    blk = np.einsum("ija,jkb->ikab", Cr, Cr)  # [r_a]x [r_b]x as (3,3,M,M)
    eye = np.eye(3)[:, :, None, None]
    Lb = (eye - blk) * w[None, None, None, :]
    return np.transpose(Lb, (0, 2, 1, 3)).reshape(3 * M, 3 * M)


def rotate_operator(A, R):
    """Lab-frame block (R (x) I_M) A (R^T (x) I_M) for body-frame A (3M x 3M)."""
    M = A.shape[0] // 3
    A4 = A.reshape(3, M, 3, M)
    return np.einsum("ce,eafb,gf->cagb", R, A4, R).reshape(3 * M, 3 * M)
