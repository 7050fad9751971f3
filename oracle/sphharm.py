"""Spherical-harmonic machinery of §3 (discretization), FP64 oracle.

Test infrastructure only (see ``oracle/__init__``).

Conventions (the paper writes complex Y_n^m with P_n^{|m|} and no phase, §3):
  * real orthonormal basis, index l*l + l + m,
      Y_l0  = N_l0 P_l(cos t)
      Y_lm  = sqrt(2) N_lm P_l^m(cos t) cos(m phi)      m > 0
      Y_l-m = sqrt(2) N_lm P_l^m(cos t) sin(m phi)      m > 0
    with N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and P_l^m WITHOUT the
    Condon-Shortley phase;
  * grid: p+1 Gauss-Legendre nodes t_j in cos(theta) times 2p equispaced
    azimuths phi_k = pi k / p (the paper's node count N = 6p(p+1)n of §3.1 and the
    N column of its Table 1 fix 2p azimuths), node index a = j*2p + k;
  * the band B_p is every (l, m) with l <= p except (p, -p), whose sin(p phi)
    vanishes on the 2p-point azimuthal grid.
"""
import math

import numpy as np


def sh_index(l, m):
    return l * l + l + m


def n_modes(L):
    return (L + 1) * (L + 1)


def gauss_legendre(n):
    """n-point Gauss-Legendre nodes (ascending) and weights on [-1, 1]."""
    t, w = np.polynomial.legendre.leggauss(n)
    return t, w


def grid(p):
    """Parametric grid of §3 (nodes theta_j = arccos t_j, phi_k), read with 2p azimuths.

    Returns dict with t, lam (GL weights), theta, phi (1-D), and per node arrays
    (length M = (p+1)*2p) theta_a, phi_a, j_a (the GL index of node a).
    """
    t, lam = gauss_legendre(p + 1)
    nphi = 2 * p
    phi = math.pi * np.arange(nphi) / p
    theta = np.arccos(t)
    j_a = np.repeat(np.arange(p + 1), nphi)
    k_a = np.tile(np.arange(nphi), p + 1)
    return {
        "p": p, "t": t, "lam": lam, "theta": theta, "phi": phi,
        "theta_a": theta[j_a], "phi_a": phi[k_a], "t_a": t[j_a], "lam_a": lam[j_a],
        "j_a": j_a, "k_a": k_a, "M": (p + 1) * nphi,
    }


def legendre_normalized(L, x):
    """N_lm P_l^m(x) (no Condon-Shortley phase) for 0 <= m <= l <= L, the same
    divided by sin(theta) (m >= 1; pole regular), and d/dtheta of it.

    x = cos(theta) with theta in [0, pi] so that sin(theta) = sqrt(1 - x^2) >= 0.
    Returns three arrays of shape (L+1, L+2) + x.shape; entries with m > l are 0.
    Uses the standard three-term recurrences of the normalized functions:
      P_mm = sqrt((2m+1)/(2m)) s P_{m-1,m-1},   P_{m+1,m} = sqrt(2m+3) x P_mm,
      P_lm = a_lm (x P_{l-1,m} - b_lm P_{l-2,m}),
        a_lm = sqrt((4l^2-1)/(l^2-m^2)),  b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)),
    and  dP_lm/dtheta = m cos(theta) (P_lm/s) - sqrt((l-m)(l+m+1)) P_{l,m+1},
    which follows from P_l^m = s^m d^m P_l/dx^m.
    """
    x = np.asarray(x, dtype=np.float64)
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    P = np.zeros((L + 1, L + 2) + x.shape)
    Q = np.zeros((L + 1, L + 2) + x.shape)   # P / sin(theta), m >= 1
    P[0, 0] = 1.0 / math.sqrt(4.0 * math.pi)
    for m in range(1, L + 1):
        c = math.sqrt((2.0 * m + 1.0) / (2.0 * m))
        Q[m, m] = c * P[m - 1, m - 1]
        P[m, m] = c * s * P[m - 1, m - 1]
    for m in range(0, L):
        c = math.sqrt(2.0 * m + 3.0)
        P[m + 1, m] = c * x * P[m, m]
        Q[m + 1, m] = c * x * Q[m, m]
    for m in range(0, L + 1):
        for l in range(m + 2, L + 1):
            a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
            P[l, m] = a * (x * P[l - 1, m] - b * P[l - 2, m])
            Q[l, m] = a * (x * Q[l - 1, m] - b * Q[l - 2, m])
    D = np.zeros_like(P)
    for l in range(L + 1):
        for m in range(0, l + 1):
            up = math.sqrt((l - m) * (l + m + 1.0)) * P[l, m + 1] if m + 1 <= l else 0.0
            D[l, m] = m * x * Q[l, m] - up
    return P, Q, D


def real_sh(L, theta, phi):
    """Real orthonormal Y_lm(theta, phi), dY/dtheta and (dY/dphi)/sin(theta).

    Returns three arrays of shape ((L+1)^2,) + theta.shape.  The last one is pole
    regular (it is what the area element needs, §3 eq. for W).
    """
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    P, Q, D = legendre_normalized(L, np.cos(theta))
    nm = n_modes(L)
    Y = np.zeros((nm,) + theta.shape)
    Yt = np.zeros_like(Y)
    Yps = np.zeros_like(Y)
    r2 = math.sqrt(2.0)
    for l in range(L + 1):
        Y[sh_index(l, 0)] = P[l, 0]
        Yt[sh_index(l, 0)] = D[l, 0]
        for m in range(1, l + 1):
            cm, sm = np.cos(m * phi), np.sin(m * phi)
            Y[sh_index(l, m)] = r2 * P[l, m] * cm
            Yt[sh_index(l, m)] = r2 * D[l, m] * cm
            Yps[sh_index(l, m)] = -r2 * m * Q[l, m] * sm
            Y[sh_index(l, -m)] = r2 * P[l, m] * sm
            Yt[sh_index(l, -m)] = r2 * D[l, m] * sm
            Yps[sh_index(l, -m)] = r2 * m * Q[l, m] * cm
    return Y, Yt, Yps


def band_indices(p):
    """Indices (into the (p+1)^2 list) of the band B_p: all modes but (p, -p)."""
    drop = sh_index(p, -p)
    return np.array([i for i in range(n_modes(p)) if i != drop], dtype=np.int64)


def forward_matrix(p):
    """Grid -> band coefficients, F (|B_p| x M), the exact left inverse of synthesis
    on B_p: c_b = sum_a (pi/p) lam_j(a) Y_b(node a) f_a * nu_b, with nu = 1/2 for the
    cos(p phi) mode (l = p, m = p), whose square the 2p-point trapezoid rule counts
    twice, and nu = 1 otherwise (GL(p+1) x trapezoid(2p) quadrature of §3)."""
    g = grid(p)
    Y, _, _ = real_sh(p, g["theta_a"], g["phi_a"])
    B = band_indices(p)
    w = (math.pi / p) * g["lam_a"]
    F = Y[B] * w[None, :]
    nyq = np.where(B == sh_index(p, p))[0]
    F[nyq] *= 0.5
    return F


def synthesis_matrix(p, theta, phi):
    """Band coefficients -> values at arbitrary points: Y_B(points) (|B_p| x npts)."""
    Y, _, _ = real_sh(p, theta, phi)
    return Y[band_indices(p)]
