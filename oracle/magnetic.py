"""Magnetostatic forces on permeable bodies (§4, magnetorheological flows), FP64 oracle.

Test infrastructure only (see ``oracle/__init__``).

Bodies of permeability mu in a fluid of permeability mu0 and a uniform applied field
H0: the potential phi = -H0 . x + S^L[q](x), with S^L the Laplace single layer
(G = 1/(4 pi |x - y|)), satisfies the transmission conditions when q solves the
second-kind equation of §4

    (1/2 I + eta K^L) q = eta H0 . n,        eta = (mu - mu0) / (mu + mu0),

K^L the normal derivative of S^L at the surface (principal value).  The incident force
density of each body (§4) is the Maxwell traction of the fluid side,

    rho = mu0 [ (H . n) H - 1/2 |H|^2 n ],   H = -grad phi (exterior limit),

the input of the mobility problem in place of F/|Gamma| + tau^{-1} T x r.

Discretization, as for the Stokes operators: self interactions by the singular rule of
``singular`` (rotated grid, band-limited interpolant) with the kernels
1/(4 pi r) and -(r . n_t)/(4 pi r^3), r = x_t - y; other bodies by the smooth rule.
Readings (the paper states the equations only): the exterior field on the surface is
H = -(grad_s phi + n d phi/dn), with the tangential gradient of the band-limited
interpolant of phi on the grid (spectral differentiation, as for the geometry in §3)
and the exterior normal derivative from the jump relation
d phi/dn = -H0 . n - q/2 + K^L q.
"""
import math

import numpy as np

from . import geometry as geo
from . import singular as sg
from . import sphharm as sh


def laplace_rows(coef, p, ps, targets):
    """Rows of the body-frame Laplace self operators S^L, K^L for the listed nodes:
    dict kind -> (len(targets), M)."""
    g = sh.grid(p)
    F = sh.forward_matrix(p)
    B = sh.band_indices(p)
    xg, ng, _ = geo.surface_frame(coef, g["theta_a"], g["phi_a"])
    nodes, W = sg.rotated_rule(ps)
    L = int(round(math.sqrt(coef.shape[1]))) - 1
    out = {"S": np.zeros((len(targets), g["M"])), "K": np.zeros((len(targets), g["M"]))}
    for i, t in enumerate(targets):
        Q = sg.rot_z(g["phi_a"][t]) @ sg.rot_y(g["theta_a"][t])
        s = Q @ nodes
        th = np.arccos(np.clip(s[2], -1.0, 1.0))
        ph = np.arctan2(s[1], s[0])
        Yall, Yt, Yps = sh.real_sh(p, th, ph)
        x = np.tensordot(coef, Yall[: sh.n_modes(L)], axes=(1, 0))
        xt = np.tensordot(coef, Yt[: sh.n_modes(L)], axes=(1, 0))
        xps = np.tensordot(coef, Yps[: sh.n_modes(L)], axes=(1, 0))
        J = np.linalg.norm(np.cross(xt, xps, axis=0), axis=0)
        r = xg[:, t][:, None] - x
        d = np.sqrt(np.sum(r * r, axis=0))
        wq = W * J
        kS = 1.0 / (4.0 * math.pi * d)
        kK = -(ng[:, t] @ r) / (4.0 * math.pi * d**3)
        YB = Yall[B]
        out["S"][i] = ((kS * wq) @ YB.T) @ F
        out["K"][i] = ((kK * wq) @ YB.T) @ F
    return out


def laplace_operators(coef, p, ps=None):
    ps = 2 * p if ps is None else ps
    M = (p + 1) * 2 * p
    return laplace_rows(coef, p, ps, range(M))


def derivative_matrices(p):
    """Grid values -> theta derivative and (phi derivative)/sin(theta) of the band-limited
    interpolant at the grid nodes: (D_t, D_p), each M x M."""
    g = sh.grid(p)
    _, Yt, Yps = sh.real_sh(p, g["theta_a"], g["phi_a"])
    B = sh.band_indices(p)
    F = sh.forward_matrix(p)
    return Yt[B].T @ F, Yps[B].T @ F


class Magnetic:
    """Magnetostatics on an oracle ``system.Problem`` (no upsampling)."""

    def __init__(self, prob, mu_ratio, H0, mu0=1.0):
        self.prob = prob
        self.eta = (mu_ratio - 1.0) / (mu_ratio + 1.0)
        self.H0 = np.asarray(H0, dtype=np.float64)
        self.mu0 = mu0
        p = prob.shapes[0].p
        self.ops = [laplace_operators(s.coef, p, s.ps) for s in prob.shapes]
        self.Dt, self.Dp = derivative_matrices(p)
        g = sh.grid(p)
        # body-frame tangent vectors x_theta, x_phi / sin(theta) per shape
        self.tan = []
        for s in prob.shapes:
            _, xt, xps = geo.eval_surface(s.coef, g["theta_a"], g["phi_a"])
            self.tan.append((xt, xps))

    # -- operators on scalar node vectors (length N) ----------------------------------
    def _far(self, q, kind):
        P = self.prob
        out = np.zeros(P.N)
        for a in range(P.N):
            keep = P.body != P.body[a]
            d = P.X[a][None, :] - P.X[keep]
            r = np.sqrt(np.sum(d * d, axis=1))
            wq = P.w[keep] * q[keep]
            if kind == "S":
                out[a] = np.sum(wq / r) / (4.0 * math.pi)
            else:
                out[a] = -np.sum((d @ P.Nn[a]) * wq / r**3) / (4.0 * math.pi)
        return out

    def _self(self, q, kind):
        P = self.prob
        out = np.zeros(P.N)
        for i in range(P.n):
            out[P.sl(i)] = self.ops[P.shape_id[i]][kind] @ q[P.sl(i)]
        return out

    def KL(self, q):
        return self._self(q, "K") + self._far(q, "K")

    def SL(self, q):
        return self._self(q, "S") + self._far(q, "S")

    def matrix(self):
        """(1/2 I + eta K^L) as a dense N x N matrix."""
        P = self.prob
        d = P.X[:, None, :] - P.X[None, :, :]
        r2 = np.sum(d * d, axis=2)
        other = P.body[:, None] != P.body[None, :]
        r2[~other] = 1.0
        dn = np.einsum("abk,ak->ab", d, P.Nn)
        K = -dn / (4.0 * math.pi * r2 * np.sqrt(r2)) * P.w[None, :]
        K[~other] = 0.0
        for i in range(P.n):
            K[P.sl(i), P.sl(i)] = self.ops[P.shape_id[i]]["K"]
        return 0.5 * np.eye(P.N) + self.eta * K

    def density(self):
        """q solving (1/2 I + eta K^L) q = eta H0 . n (dense LU)."""
        P = self.prob
        return np.linalg.solve(self.matrix(), self.eta * (P.Nn @ self.H0))

    def field(self, q):
        """Exterior field H (N, 3) on every node."""
        P = self.prob
        phi = -(P.X @ self.H0) + self.SL(q)
        dn = -(P.Nn @ self.H0) - 0.5 * q + self.KL(q)
        H = np.zeros((P.N, 3))
        for i in range(P.n):
            sl = P.sl(i)
            xt, xps = self.tan[P.shape_id[i]]
            a = (P.R[i] @ xt).T                      # lab-frame tangents (M, 3)
            b = (P.R[i] @ xps).T
            ft, fp = self.Dt @ phi[sl], self.Dp @ phi[sl]
            aa, bb, ab = np.sum(a * a, 1), np.sum(b * b, 1), np.sum(a * b, 1)
            det = aa * bb - ab * ab
            grad = (((bb * ft - ab * fp) / det)[:, None] * a + ((aa * fp - ab * ft) / det)[:, None] * b)
            H[sl] = -(grad + dn[sl][:, None] * P.Nn[sl])
        return H

    def traction(self, H):
        """Maxwell traction of the fluid side, mu0 [(H.n) H - |H|^2 n / 2], (N, 3)."""
        n = self.prob.Nn
        Hn = np.sum(H * n, axis=1)
        return self.mu0 * (Hn[:, None] * H - 0.5 * np.sum(H * H, axis=1)[:, None] * n)

    def forces(self, rho):
        """Net force and torque (about the centroid) per body, (n, 6)."""
        P = self.prob
        out = np.zeros((P.n, 6))
        for i in range(P.n):
            sl = P.sl(i)
            wi = P.w[sl][:, None]
            out[i, :3] = np.sum(wi * rho[sl], axis=0)
            out[i, 3:] = np.sum(wi * np.cross(P.X[sl] - P.c[i], rho[sl]), axis=0)
        return out
