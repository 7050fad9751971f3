"""Pins of the oracle's off-body sums (§2.1, §3.1)."""
import math

import numpy as np

from oracle import farfield as ff


def _pts(seed, n):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-2, 2, (n, 3))
    q = rng.standard_normal((n, 3))
    return X, q


def test_against_pure_python_double_loop():
    X, q = _pts(0, 12)
    Nn = np.random.default_rng(1).standard_normal((12, 3))
    body = np.arange(12) // 3
    ref_u = np.zeros((12, 3))
    ref_t = np.zeros((12, 3))
    for a in range(12):
        for b in range(12):
            if body[a] == body[b]:
                continue
            d = [X[a][k] - X[b][k] for k in range(3)]
            r = math.sqrt(sum(v * v for v in d))
            dq = sum(d[k] * q[b][k] for k in range(3))
            dn = sum(d[k] * Nn[a][k] for k in range(3))
            for i in range(3):
                ref_u[a][i] += (q[b][i] / r + d[i] * dq / r ** 3) / (8 * math.pi)
                ref_t[a][i] += -3.0 / (4 * math.pi) * d[i] * dn * dq / r ** 5
    assert np.abs(ff.stokeslet_sum(X, X, q, body, body) - ref_u).max() < 1e-13
    assert np.abs(ff.traction_sum(X, Nn, X, q, body, body) - ref_t).max() < 1e-12


def test_traction_equals_stress_of_stokeslet_field():
    # K rho = [-p I + grad u + grad u^T] n for the Stokeslet sum (§3.1), by central
    # differences of the velocity sum and the Stokeslet pressure
    Xs, q = _pts(2, 30)
    rng = np.random.default_rng(3)
    Xt = rng.uniform(3, 4, (5, 3))
    Nt = rng.standard_normal((5, 3))
    Nt /= np.linalg.norm(Nt, axis=1)[:, None]
    bt = np.full(5, -1)
    bs = np.zeros(30, dtype=int)
    h = 1e-4
    grad = np.zeros((5, 3, 3))   # grad[a, i, j] = d u_i / d x_j
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        up = ff.stokeslet_sum(Xt + e, Xs, q, bt, bs)
        um = ff.stokeslet_sum(Xt - e, Xs, q, bt, bs)
        grad[:, :, j] = (up - um) / (2 * h)
    pr = ff.pressure_sum(Xt, Xs, q, bt, bs)
    sigma = -pr[:, None, None] * np.eye(3)[None] + grad + np.transpose(grad, (0, 2, 1))
    ref = np.einsum("aij,aj->ai", sigma, Nt)
    got = ff.traction_sum(Xt, Nt, Xs, q, bt, bs)
    assert np.abs(got - ref).max() < 1e-8 * np.abs(ref).max()


def test_stokeslet_pressure_satisfies_stokes_equations():
    # -Lap u + grad p = 0 and div u = 0 away from the sources
    Xs, q = _pts(4, 10)
    Xt = np.array([[5.0, 0.3, -0.2]])
    bt, bs = np.full(1, -1), np.zeros(10, dtype=int)
    h = 1e-3
    lap = np.zeros(3)
    div = 0.0
    gp = np.zeros(3)
    u0 = ff.stokeslet_sum(Xt, Xs, q, bt, bs)[0]
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        up = ff.stokeslet_sum(Xt + e, Xs, q, bt, bs)[0]
        um = ff.stokeslet_sum(Xt - e, Xs, q, bt, bs)[0]
        lap += (up - 2 * u0 + um) / h ** 2
        div += (up[j] - um[j]) / (2 * h)
        gp[j] = (ff.pressure_sum(Xt + e, Xs, q, bt, bs)[0] - ff.pressure_sum(Xt - e, Xs, q, bt, bs)[0]) / (2 * h)
    scale = np.abs(gp).max()
    assert np.abs(-lap + gp).max() < 1e-5 * scale
    assert abs(div) < 1e-7 * np.abs(u0).max()
