"""Off-body layer-potential sums with the smooth quadrature rule, FP64 oracle.

Test infrastructure only (see ``oracle/__init__``).

The paper evaluates interactions between different bodies with the smooth rule of
§3 accelerated by a Stokes FMM (§3.1); the oracle is the exact direct sum that such
an FMM approximates.  Sources are point forces q_b = w_b sigma_b.  Pairs whose
target and source lie on the same body are excluded (they belong to the singular
self blocks).  No near-singular upsampling is applied.

  Stokeslet (§2.1):     u_a = sum_b (1/(8 pi eta)) [q_b/|d| + d (d . q_b)/|d|^3]
  traction  (§2.1):     y_a = sum_b -(3/(4 pi)) d (d . N_a)(d . q_b) / |d|^5
  pressure  (Stokeslet pressure): p_a = sum_b (1/(4 pi)) (d . q_b)/|d|^3
with d = X_a - X_b.  Points are (N, 3) arrays here.
"""
import math

import numpy as np


def stokeslet_sum(Xt, Xs, q, body_t, body_s, eta=1.0):
    out = np.zeros((Xt.shape[0], 3))
    for a in range(Xt.shape[0]):
        keep = body_s != body_t[a]
        d = Xt[a][None, :] - Xs[keep]
        r2 = np.sum(d * d, axis=1)
        r = np.sqrt(r2)
        dq = np.sum(d * q[keep], axis=1)
        out[a] = np.sum(q[keep] / r[:, None] + d * (dq / (r2 * r))[:, None], axis=0)
    return out / (8.0 * math.pi * eta)


def traction_sum(Xt, Nt, Xs, q, body_t, body_s):
    out = np.zeros((Xt.shape[0], 3))
    for a in range(Xt.shape[0]):
        keep = body_s != body_t[a]
        d = Xt[a][None, :] - Xs[keep]
        r2 = np.sum(d * d, axis=1)
        dn = d @ Nt[a]
        dq = np.sum(d * q[keep], axis=1)
        out[a] = np.sum(d * (dn * dq / (r2 * r2 * np.sqrt(r2)))[:, None], axis=0)
    return -(3.0 / (4.0 * math.pi)) * out


def pressure_sum(Xt, Xs, q, body_t, body_s):
    out = np.zeros(Xt.shape[0])
    for a in range(Xt.shape[0]):
        keep = body_s != body_t[a]
        d = Xt[a][None, :] - Xs[keep]
        r2 = np.sum(d * d, axis=1)
        dq = np.sum(d * q[keep], axis=1)
        out[a] = np.sum(dq / (r2 * np.sqrt(r2)))
    return out / (4.0 * math.pi)
