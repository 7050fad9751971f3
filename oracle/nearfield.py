"""Near-singular evaluation by upsampling (§3), FP64 oracle.

Test infrastructure only (see ``oracle/__init__``).

§3 evaluates the layer potentials between different bodies with the smooth rule
and, for targets close to another body, upsamples the boundary data.  The paper
gives neither the closeness criterion nor the upsampled order.  Reading used here:

  * body j is near body i (i != j) when |c_i - c_j| < R_i + R_j + kappa h_j, where
    R is the largest distance from a shape's area centroid to a node of its fine
    grid and h_j = sqrt(|Gamma_j| / M) is the mean node spacing of j's grid;
  * every target of body i then integrates over Gamma_j with the smooth rule of
    order p_u, on the (p_u + 1) x 2 p_u grid: the geometry is evaluated exactly from
    the shape's SH coefficients at the fine nodes, the weights are
    (pi / p_u) lam'_j J', and the density is replaced by its band-limited
    interpolant sum_{B_p} (F mu)_lm Y_lm at the fine nodes (the interpolant the
    singular rule of §3 uses).  Pairs that are not near keep the plain rule.

The fine nodes are recentred with the coarse grid's area centroid, so that a body
sits at the same lab position on both grids.
"""
import math

import numpy as np

from . import geometry as geo
from . import sphharm as sh


def fine_geometry(coef, xc, p_u):
    """Body-frame fine nodes r' = x' - xc, weights w' and the bounding radius."""
    g = geo.shape_geometry(np.asarray(coef, dtype=np.float64), p_u)
    r = g["x"] - np.asarray(xc)[:, None]
    return {"r": r, "w": g["w"], "M": g["grid"]["M"],
            "R": float(np.sqrt(np.max(np.sum(r * r, axis=0))))}


def interp_matrix(p, p_u):
    """Grid values at order p -> band-limited interpolant at the nodes of order p_u:
    U = Y_B(fine nodes)^T F, a (M_u x M) matrix."""
    gu = sh.grid(p_u)
    return sh.synthesis_matrix(p, gu["theta_a"], gu["phi_a"]).T @ sh.forward_matrix(p)


def near_matrix(centres, R, h, shape_id, kappa):
    """near[i, j] for the reading above (i != j); R and h are per shape."""
    c = np.asarray(centres, dtype=np.float64)
    sid = np.asarray(shape_id)
    n = len(sid)
    near = np.zeros((n, n), dtype=bool)
    for i in range(n):
        for j in range(n):
            if i != j:
                dist = math.sqrt(float(np.sum((c[i] - c[j]) ** 2)))
                near[i, j] = dist < R[sid[i]] + R[sid[j]] + kappa * h[sid[j]]
    return near


def traction_block(Xt, Nt, Xs, q):
    """-(3/(4 pi)) sum_b d (d.N_a)(d.q_b)/|d|^5 for every target a (no exclusions)."""
    d = Xt[:, None, :] - Xs[None, :, :]
    r2 = np.sum(d * d, axis=2)
    dn = np.einsum("abk,ak->ab", d, Nt)
    dq = np.einsum("abk,bk->ab", d, q)
    f = dn * dq / (r2 * r2 * np.sqrt(r2))
    return -(3.0 / (4.0 * math.pi)) * np.einsum("ab,abk->ak", f, d)


def stokeslet_block(Xt, Xs, q, eta):
    """(1/(8 pi eta)) sum_b [q_b/|d| + d (d.q_b)/|d|^3] for every target a."""
    d = Xt[:, None, :] - Xs[None, :, :]
    r2 = np.sum(d * d, axis=2)
    r = np.sqrt(r2)
    dq = np.einsum("abk,bk->ab", d, q)
    u = np.einsum("ab,bk->ak", 1.0 / r, q) + np.einsum("ab,abk->ak", dq / (r2 * r), d)
    return u / (8.0 * math.pi * eta)


def traction_matrix_block(Xt, Nt, Xs, w):
    """Matrix of traction_block in the density: (Mt, 3, Ms, 3), q_b = w_b mu_b."""
    d = Xt[:, None, :] - Xs[None, :, :]
    r2 = np.sum(d * d, axis=2)
    dn = np.einsum("abk,ak->ab", d, Nt)
    fac = -(3.0 / (4.0 * math.pi)) * dn / (r2 * r2 * np.sqrt(r2)) * w[None, :]
    return np.einsum("ab,abi,abj->aibj", fac, d, d)
