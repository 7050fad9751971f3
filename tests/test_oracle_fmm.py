"""Pins of the oracle's fast multipole approximation of the off-body traction sum (the
O(N) far field of §3.1): the solid-harmonic identities it rests on (closed forms, the
addition theorem against 1/|x - y|, translations, derivatives by finite differences), the
translation operators on single charges, and the FMM against the direct sum: exact when
nothing is far, converging geometrically in the order P otherwise."""
import itertools
import math

import numpy as np
import pytest

from oracle import farfield as ff
from oracle import fmm


def _i(n, m):
    return n * n + n + m


def test_low_degree_closed_forms():
    x = np.array([0.3, -0.7, 1.1])
    R, I = fmm.solid_harmonics(x, 3)
    R, I = R[0], I[0]
    r = np.linalg.norm(x)
    w = complex(x[0], x[1])
    assert abs(R[_i(0, 0)] - 1) < 1e-15
    assert abs(R[_i(1, 0)] - x[2]) < 1e-15
    assert abs(R[_i(1, 1)] - w / 2) < 1e-15
    assert abs(R[_i(2, 0)] - (3 * x[2] ** 2 - r * r) / 4) < 1e-14
    for m in range(4):                       # R_m^m = (x + iy)^m / (2^m m!)
        assert abs(R[_i(m, m)] - w ** m / (2 ** m * math.factorial(m))) < 1e-14
    assert abs(I[_i(0, 0)] - 1 / r) < 1e-15
    assert abs(I[_i(1, 0)] - x[2] / r ** 3) < 1e-15
    assert abs(I[_i(1, 1)] - w / r ** 3) < 1e-15
    assert abs(R[_i(2, -1)] - (-1) * np.conj(R[_i(2, 1)])) < 1e-15


def test_addition_theorem_and_translations():
    rng = np.random.default_rng(0)
    x = np.array([4.0, -2.5, 3.0])
    y = rng.uniform(-0.6, 0.6, 3)
    Q = 40
    Ry = fmm.solid_harmonics(y, Q)[0][0]
    Ix = fmm.solid_harmonics(x, Q)[1][0]
    assert abs(np.sum(np.conj(Ry) * Ix) - 1 / np.linalg.norm(x - y)) < 1e-15
    # R_n^m(x + y) = sum R_k^l(x) R_{n-k}^{m-l}(y)
    P = 7
    a, b = rng.standard_normal(3), rng.standard_normal(3)
    Ra, Rb, Rab = (fmm.solid_harmonics(v, P)[0][0] for v in (a, b, a + b))
    for n in range(P + 1):
        for m in range(-n, n + 1):
            s = sum(Ra[_i(k, l)] * Rb[_i(n - k, m - l)] for k in range(n + 1) for l in range(-k, k + 1)
                    if abs(m - l) <= n - k)
            assert abs(s - Rab[_i(n, m)]) < 1e-13 * max(1.0, abs(Rab[_i(n, m)]))
    # I_n^m(a + b) = sum (-1)^k conj(R_k^l(b)) I_{n+k}^{m+l}(a), |b| < |a|
    a = np.array([3.0, 2.0, -4.0])
    b = 0.4 * rng.standard_normal(3)
    Q = 45
    Ia = fmm.solid_harmonics(a, P + Q)[1][0]
    Rb = fmm.solid_harmonics(b, Q)[0][0]
    Iab = fmm.solid_harmonics(a + b, P)[1][0]
    for n in range(P + 1):
        for m in range(-n, n + 1):
            s = sum((-1) ** k * np.conj(Rb[_i(k, l)]) * Ia[_i(n + k, m + l)]
                    for k in range(Q + 1) for l in range(-k, k + 1))
            assert abs(s - Iab[_i(n, m)]) < 1e-12 * abs(Iab[_i(n, m)])


def test_derivative_identities_by_finite_differences():
    P, h = 6, 1e-5
    x = np.array([0.4, -0.3, 0.6])
    R = lambda v: fmm.solid_harmonics(v, P)[0][0]
    d = [(R(x + h * e) - R(x - h * e)) / (2 * h) for e in np.eye(3)]
    R0 = R(x)
    for n in range(1, P + 1):
        for m in range(-n, n + 1):
            lower = lambda mm: R0[_i(n - 1, mm)] if abs(mm) <= n - 1 else 0.0
            assert abs(d[2][_i(n, m)] - lower(m)) < 1e-9
            assert abs(d[0][_i(n, m)] + 1j * d[1][_i(n, m)] + lower(m + 1)) < 1e-9
            assert abs(d[0][_i(n, m)] - 1j * d[1][_i(n, m)] - lower(m - 1)) < 1e-9


def test_translation_operators_on_one_charge_converge():
    rng = np.random.default_rng(1)
    c1 = np.zeros(3)
    y = rng.uniform(-0.5, 0.5, 3)
    c2 = np.array([0.5, 0.5, -0.5])              # parent centre
    ct = np.array([4.0, 0.0, 2.0])               # target box centre, width 1
    x = ct + np.array([0.3, -0.4, 0.2])
    exact = 1.0 / np.linalg.norm(x - y)
    errs = []
    for P in (4, 8, 12, 16):
        M = np.conj(fmm.solid_harmonics(y - c1, P)[0][0])
        M2 = fmm.m2m_matrix(c1 - c2, P) @ M
        Lt = fmm.m2l_matrix(ct - c2, P) @ M2
        c3 = ct + np.array([0.25, -0.25, 0.25])
        L3 = fmm.l2l_matrix(c3 - ct, P) @ Lt
        v = L3 @ np.conj(fmm.solid_harmonics(x - c3, P)[0][0])
        errs.append(abs(v - exact) / exact)
        # multipole evaluated directly and M2M are exact up to truncation only
        assert abs(M2 @ fmm.solid_harmonics(x - c2, P)[1][0] - exact) / exact < 2 * 0.3 ** (P + 1)
    assert errs[-1] < 1e-8 and all(b < a / 10 for a, b in zip(errs, errs[1:]))


def _spheres(side, spacing, npts, seed):
    rng = np.random.default_rng(seed)
    k = np.arange(npts) + 0.5
    th = np.arccos(1 - 2 * k / npts)
    ph = math.pi * (1 + 5 ** 0.5) * k
    u = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)
    X, Nn, body = [], [], []
    for b, c in enumerate(itertools.product(range(side), repeat=3)):
        X.append(np.array(c) * spacing + rng.uniform(-0.2, 0.2, 3) + u)
        Nn.append(u)
        body.append(np.full(npts, b))
    X, Nn, body = np.concatenate(X), np.concatenate(Nn), np.concatenate(body)
    q = rng.standard_normal(X.shape)
    return X, Nn, q, body


def test_plan_keeps_every_body_in_adjacent_leaves():
    X, _, _, body = _spheres(4, 3.0, 40, 2)
    lo, D, L = fmm.plan(X, 2.0)
    assert L >= 2 and D / 2 ** L >= 2.0 and D / 2 ** (L + 1) < 2.0
    w = D / 2 ** L
    ijk = np.minimum(np.floor((X - lo) / w).astype(int), 2 ** L - 1)
    for b in np.unique(body):
        g = ijk[body == b]
        assert (g.max(axis=0) - g.min(axis=0)).max() <= 1


def test_fmm_is_the_direct_sum_when_nothing_is_far():
    X, Nn, q, body = _spheres(2, 3.0, 30, 3)
    y, (_, _, L) = fmm.traction(X, Nn, q, body, 6, 2.0)
    assert L < 2
    ref = ff.traction_sum(X, Nn, X, q, body, body)
    assert np.abs(y - ref).max() < 1e-13 * np.abs(ref).max()


def test_fmm_converges_to_the_direct_sum():
    X, Nn, q, body = _spheres(4, 3.0, 40, 4)
    ref = ff.traction_sum(X, Nn, X, q, body, body)
    errs = []
    for P in (4, 8, 12):
        y, (_, _, L) = fmm.traction(X, Nn, q, body, P, 2.0)
        assert L == 2
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    assert errs[2] < 2e-3 and errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3


@pytest.mark.parametrize("bad", ["direction", "parity"])
def test_convergence_pin_catches_planted_mistakes(bad, monkeypatch):
    """An M2L built for the reversed displacement, or without its (-1)^k factor, is caught
    by the convergence pin."""
    X, Nn, q, body = _spheres(4, 3.0, 40, 4)
    ref = ff.traction_sum(X, Nn, X, q, body, body)
    orig = fmm.m2l_matrix
    if bad == "direction":
        monkeypatch.setattr(fmm, "m2l_matrix", lambda a, P: orig(-a, P))
    else:
        def dropped(a, P):
            k = np.concatenate([[n] * (2 * n + 1) for n in range(P + 1)])
            return orig(a, P) * ((-1.0) ** k)[:, None]
        monkeypatch.setattr(fmm, "m2l_matrix", dropped)
    y, _ = fmm.traction(X, Nn, q, body, 12, 2.0)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) > 1e-2


def test_fmm_converges_with_three_levels():
    """Leaf level 3: multipoles move up (M2M) and locals down (L2L) between levels."""
    X, Nn, q, body = _spheres(6, 3.0, 16, 5)
    ref = ff.traction_sum(X, Nn, X, q, body, body)
    errs = []
    for P in (4, 8):
        y, (_, _, L) = fmm.traction(X, Nn, q, body, P, 2.0)
        assert L == 3
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    assert errs[1] < 1e-2 and errs[1] < errs[0] / 3
