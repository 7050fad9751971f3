"""Fast multipole approximation of the off-body traction sum, FP64 oracle.

Test infrastructure only (see ``oracle/__init__``).

§3.1 evaluates the sums between bodies with a Stokes FMM (linear cost, an
approximation of the direct sum of ``farfield``).  This module is the reference for
the GPU's O(N) equivalent.  The paper leaves the FMM to a library and fixes nothing
about it, so everything below is a reading, listed here.

Stokes through four harmonic potentials.  With d = x - y, the traction sum
y(x) = sum_b -(3/4pi) d (d.N)(d.q_b)/|d|^5 is the traction [-pI + grad u + grad u^T] N
of the Stokeslet field of the point forces q_b (§2.1).  Let
phi_j(x) = sum_b q_bj / |x - y_b| for j = 1..3, and let psi_c(x) = sum_b ((y_b - c).q_b) / |x - y_b|
for a fixed point c.  Then, with s = x - c,

    p = -(1/4pi) div phi,    grad u + grad u^T = (1/4pi) [H(psi_c) - s_j H(phi_j)],
    y(x) = (1/4pi) [ (div phi) N + (H(psi_c) - s_j H(phi_j)) N ],

where H is the Hessian at x.  Taking c = the centre of the leaf box that holds x keeps
the cancellation between the two Hessian terms small.

Expansions use complex solid harmonics normalised with factorials.  P_n^m is the
associated Legendre function without the Condon-Shortley phase.
    R_n^m(x) = r^n P_n^m(cos t) e^{i m p} / (n + m)!,   I_n^m(x) = (n - m)! P_n^m(cos t) e^{i m p} / r^{n+1},
    R_n^{-m} = (-1)^m conj(R_n^m),  I_n^{-m} = (-1)^m conj(I_n^m).
They satisfy
    1/|x - y| = sum_{n,m} conj(R_n^m(y)) I_n^m(x)                      (|y| < |x|),
    R_n^m(x + y) = sum_{k,l} R_k^l(x) R_{n-k}^{m-l}(y),
    I_n^m(a + b) = sum_{k,l} (-1)^k conj(R_k^l(b)) I_{n+k}^{m+l}(a)     (|b| < |a|),
    d/dz R_n^m = R_{n-1}^m,  (d/dx + i d/dy) R_n^m = -R_{n-1}^{m+1},  (d/dx - i d/dy) R_n^m = R_{n-1}^{m-1}.
The pins in ``tests/test_oracle_fmm.py`` check each of these numerically.

Multipole about c:       phi(x) = sum M_n^m I_n^m(x - c),           M_n^m = sum_b q_b conj(R_n^m(y_b - c)).
Local about c:           phi(x) = sum L_k^l conj(R_k^l(x - c)).
M2M (child c1 to parent c2):  M'_n^m = sum_{k,l} M_k^l conj(R_{n-k}^{m-l}(c1 - c2)).
M2L (source c_s to target c_t, a = c_t - c_s):  L_k^l = (-1)^k sum_{n,m} M_n^m I_{n+k}^{m+l}(a).
L2L (parent c to child c'):   L'_j^i = sum_{k,l} L_k^l conj(R_{k-j}^{l-i}(c' - c)).
Every expansion is truncated at degree P.  Moving the psi density from centre c to c'
adds (c - c').q to each charge, so before a translation its coefficients gain
(c - c')_j times those of phi_j.

Tree.  lo is the componentwise minimum of the points.  The root cube has side
D = e (1 + 2^-20), where e is the largest extent.  The leaf level L is the finest
level whose box width D / 2^L is at least d_max, the largest body diameter, capped at
L_max.  As a result two nodes of one body always lie in the same or adjacent leaves.
Leaf of a point: floor((x - lo) / w) per coordinate, clamped to [0, 2^L - 1].  Box id
(k 2^l + j) 2^l + i, x fastest.
Near field (direct, other bodies only): the 27 adjacent leaves, the leaf itself included.
Interaction list at levels 2..L: the boxes that are not adjacent but whose parents
are adjacent (at most 189).
With L < 2 nothing is far, and the sum is direct.
"""
import itertools
import math

import numpy as np
from scipy.special import lpmv


def _idx(n, m):
    return n * n + n + m


def _legendre_all(P, t):
    """P_n^m(t) for 0 <= m <= n <= P without the Condon-Shortley phase: dict (n, m) -> array."""
    out = {}
    for n in range(P + 1):
        for m in range(n + 1):
            out[(n, m)] = lpmv(m, n, t) * (-1.0) ** m
    return out


def solid_harmonics(x, P):
    """(R, I): complex (npts, (P+1)^2) arrays of R_n^m(x) and I_n^m(x), index n^2 + n + m."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    r = np.sqrt(np.sum(x * x, axis=1))
    rs = np.where(r > 0, r, 1.0)
    t = np.clip(x[:, 2] / rs, -1.0, 1.0)
    ph = np.arctan2(x[:, 1], x[:, 0])
    Pl = _legendre_all(P, t)
    R = np.zeros((len(r), (P + 1) ** 2), complex)
    I = np.zeros((len(r), (P + 1) ** 2), complex)
    for n in range(P + 1):
        for m in range(n + 1):
            e = np.exp(1j * m * ph)
            vr = r ** n * Pl[(n, m)] * e / math.factorial(n + m)
            vi = math.factorial(n - m) * Pl[(n, m)] * e / rs ** (n + 1)
            R[:, _idx(n, m)] = vr
            I[:, _idx(n, m)] = vi
            if m > 0:
                R[:, _idx(n, -m)] = (-1) ** m * np.conj(vr)
                I[:, _idx(n, -m)] = (-1) ** m * np.conj(vi)
    return R, I


def _pairs(P):
    return [(n, m) for n in range(P + 1) for m in range(-n, n + 1)]


_MAPS = {}


def _maps(P):
    """Index maps of the three translation operators at order P (built once per P):
    (rows, cols, table index[, sign]) of the nonzero entries."""
    if P not in _MAPS:
        m2m, m2l, l2l = ([], [], []), ([], [], [], []), ([], [], [])
        for n, m in _pairs(P):
            for k, l in _pairs(n):
                if abs(m - l) <= n - k:
                    for lst, v in zip(m2m, (_idx(n, m), _idx(k, l), _idx(n - k, m - l))):
                        lst.append(v)
        for k, l in _pairs(P):
            for n, m in _pairs(P):
                for lst, v in zip(m2l, (_idx(k, l), _idx(n, m), _idx(n + k, m + l), (-1) ** k)):
                    lst.append(v)
        for j, i in _pairs(P):
            for k, l in _pairs(P):
                if k >= j and abs(l - i) <= k - j:
                    for lst, v in zip(l2l, (_idx(j, i), _idx(k, l), _idx(k - j, l - i))):
                        lst.append(v)
        _MAPS[P] = tuple(tuple(np.array(a) for a in t) for t in (m2m, m2l, l2l))
    return _MAPS[P]


def m2m_matrix(t, P):
    """Operator on multipole coefficients for the shift c1 -> c2, t = c1 - c2:
    entry ((n, m), (k, l)) = conj(R_{n-k}^{m-l}(t))."""
    r, c, i = _maps(P)[0]
    A = np.zeros(((P + 1) ** 2, (P + 1) ** 2), complex)
    A[r, c] = np.conj(solid_harmonics(t, P)[0][0])[i]
    return A


def m2l_matrix(a, P):
    """Operator from multipole (about c_s) to local (about c_t) coefficients, a = c_t - c_s:
    entry ((k, l), (n, m)) = (-1)^k I_{n+k}^{m+l}(a)."""
    r, c, i, sg = _maps(P)[1]
    B = np.zeros(((P + 1) ** 2, (P + 1) ** 2), complex)
    B[r, c] = sg * solid_harmonics(a, 2 * P)[1][0][i]
    return B


def l2l_matrix(t, P):
    """Operator on local coefficients for the shift c -> c', t = c' - c:
    entry ((j, i), (k, l)) = conj(R_{k-j}^{l-i}(t)) for k >= j."""
    r, c, i = _maps(P)[2]
    C = np.zeros(((P + 1) ** 2, (P + 1) ** 2), complex)
    C[r, c] = np.conj(solid_harmonics(t, P)[0][0])[i]
    return C


def derivative_coefficients(Lc, P, dk, dl, sign=1.0):
    """Coefficients of a derivative of a local expansion: out_k^l = sign L_{k+dk}^{l+dl}, k <= P - dk
    (dz: (1, 0); d/dx + i d/dy: (1, 1); d/dx - i d/dy: (1, -1) with sign -1)."""
    out = np.zeros(Lc.shape[:-1] + ((P + 1 - dk) ** 2,), complex)
    for k, l in _pairs(P - dk):
        if abs(l + dl) <= k + dk:
            out[..., _idx(k, l)] = sign * Lc[..., _idx(k + dk, l + dl)]
    return out


def plan(X, d_max, L_max=6):
    """(lo, D, L) of the tree over the points X (N, 3)."""
    lo = X.min(axis=0)
    e = float((X.max(axis=0) - lo).max())
    D = e * (1.0 + 2.0 ** -20) if e > 0 else 1.0
    L = 0
    while L < L_max and D / 2.0 ** (L + 1) >= d_max:
        L += 1
    return lo, D, L


def _box_ids(ijk, n):
    return (ijk[..., 2] * n + ijk[..., 1]) * n + ijk[..., 0]


def _centres(lo, D, level):
    n = 2 ** level
    g = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)
    ids = _box_ids(g, n)
    c = np.zeros((n ** 3, 3))
    c[ids] = lo + (g + 0.5) * (D / n)
    return c


def _ijk(ids, n):
    return np.stack([ids % n, (ids // n) % n, ids // (n * n)], -1)


def traction(X, Nn, q, body, P, d_max, L_max=6):
    """FMM approximation of ``farfield.traction_sum`` at every point (targets = sources)."""
    X, Nn, q = (np.asarray(a, dtype=np.float64) for a in (X, Nn, q))
    body = np.asarray(body)
    N = len(X)
    lo, D, L = plan(X, d_max, L_max)
    nb = 2 ** L
    w = D / nb
    ijk = np.minimum(np.floor((X - lo) / w).astype(np.int64), nb - 1)
    leaf = _box_ids(ijk, nb)
    K = (P + 1) ** 2
    far = np.zeros((N, 3))
    if L >= 2:
        cen = {lev: _centres(lo, D, lev) for lev in range(2, L + 1)}
        cl = cen[L][leaf]
        s = X - cl
        Rs = solid_harmonics(s, P)[0]
        charges = np.concatenate([q, np.sum(s * q, axis=1)[:, None]], axis=1)      # (N, 4)
        M = {L: np.zeros((nb ** 3, 4, K), complex)}
        np.add.at(M[L], leaf, charges[:, :, None] * np.conj(Rs)[:, None, :])
        # upward pass
        for lev in range(L, 2, -1):
            n = 2 ** lev
            ids = np.arange(n ** 3)
            g = _ijk(ids, n)
            par = _box_ids(g // 2, n // 2)
            Mp = np.zeros(((n // 2) ** 3, 4, K), complex)
            for o in itertools.product([0, 1], repeat=3):
                sel = np.all(g % 2 == np.array(o), axis=1)
                t = cen[lev][ids[sel][0]] - cen[lev - 1][par[sel][0]]          # c1 - c2
                A = m2m_matrix(t, P)
                Mc = M[lev][sel].copy()
                Mc[:, 3] += np.einsum("j,bjk->bk", t, Mc[:, :3])                # psi: c1 -> c2
                np.add.at(Mp, par[sel], Mc @ A.T)
            M[lev - 1] = Mp
        # downward pass
        Lx = {}
        for lev in range(2, L + 1):
            n = 2 ** lev
            ids = np.arange(n ** 3)
            g = _ijk(ids, n)
            Lx[lev] = np.zeros((n ** 3, 4, K), complex)
            if lev > 2:
                par = _box_ids(g // 2, n // 2)
                for o in itertools.product([0, 1], repeat=3):
                    sel = np.all(g % 2 == np.array(o), axis=1)
                    t = cen[lev][ids[sel][0]] - cen[lev - 1][par[sel][0]]      # c' - c
                    C = l2l_matrix(t, P)
                    Lp = Lx[lev - 1][par[sel]].copy()
                    Lp[:, 3] -= np.einsum("j,bjk->bk", t, Lp[:, :3])           # psi: c -> c'
                    Lx[lev][sel] += Lp @ C.T
            for v in itertools.product(range(-3, 4), repeat=3):
                v = np.array(v)
                if np.abs(v).max() <= 1:
                    continue
                src = g - v
                ok = np.all((src >= 0) & (src < n), axis=1) & np.all(np.abs(src // 2 - g // 2) <= 1, axis=1)
                if not ok.any():
                    continue
                a = v * (D / n)                                                  # c_t - c_s
                B = m2l_matrix(a, P)
                Ms = M[lev][_box_ids(src[ok], n)].copy()
                Ms[:, 3] -= np.einsum("j,bjk->bk", a, Ms[:, :3])                # psi: c_s -> c_t
                Lx[lev][ids[ok]] += Ms @ B.T
        # evaluation at the targets
        Lt = Lx[L][leaf]
        Rc = np.conj(Rs)

        def ev(dk, dl, sign=1.0):
            Kd = (P + 1 - dk) ** 2
            return np.einsum("nck,nk->nc", derivative_coefficients(Lt, P, dk, dl, sign), Rc[:, :Kd])

        gp = ev(1, 1)                         # (d/dx + i d/dy) of each density
        gz = ev(1, 0)
        A2 = ev(2, 2)                         # (d/dx + i d/dy)^2
        B2 = ev(2, 1)                         # d/dz (d/dx + i d/dy)
        C2 = ev(2, 0)                         # d^2/dz^2
        H = np.zeros((N, 4, 3, 3))
        H[:, :, 0, 0] = 0.5 * (A2.real - C2.real)
        H[:, :, 1, 1] = 0.5 * (-A2.real - C2.real)
        H[:, :, 0, 1] = H[:, :, 1, 0] = 0.5 * A2.imag
        H[:, :, 0, 2] = H[:, :, 2, 0] = B2.real
        H[:, :, 1, 2] = H[:, :, 2, 1] = B2.imag
        H[:, :, 2, 2] = C2.real
        div = gp[:, 0].real + gp[:, 1].imag + gz[:, 2].real
        Hs = H[:, 3] - np.einsum("nj,njik->nik", s, H[:, :3])
        far = (div[:, None] * Nn + np.einsum("nik,nk->ni", Hs, Nn)) / (4.0 * math.pi)
    # near field: adjacent leaves, other bodies
    near = np.zeros((N, 3))
    order = np.argsort(leaf, kind="stable")
    starts = np.searchsorted(leaf[order], np.arange(nb ** 3 + 1))
    for t in np.unique(leaf):
        tgt = order[starts[t]:starts[t + 1]]
        ti = _ijk(np.array([t]), nb)[0]
        src = []
        for dv in itertools.product([-1, 0, 1], repeat=3):
            sj = ti + np.array(dv)
            if np.all((sj >= 0) & (sj < nb)):
                sb = _box_ids(sj, nb)
                src.append(order[starts[sb]:starts[sb + 1]])
        src = np.concatenate(src)
        d = X[tgt][:, None, :] - X[src][None, :, :]
        other = body[tgt][:, None] != body[src][None, :]
        r2 = np.where(other, np.sum(d * d, axis=2), 1.0)
        f = np.where(other, np.einsum("tsk,tk->ts", d, Nn[tgt]) * np.einsum("tsk,sk->ts", d, q[src])
                     / (r2 * r2 * np.sqrt(r2)), 0.0)
        near[tgt] = -3.0 / (4.0 * math.pi) * np.einsum("ts,tsk->tk", f, d)
    return far + near, (lo, D, L)
