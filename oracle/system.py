"""The discrete mobility problem, FP64 oracle (§2.2, §2.3, §3, §3.2, §3.3).

Test infrastructure only (see ``oracle/__init__``).

Given body shapes, poses and loads (F_i, T_i):
  1. incident density rho_i = F_i/|Gamma_i| + tau_i^{-1} T_i x (x - x^c_i)   (§2.2)
  2. solve the augmented second-kind system (§2.3)
        (1/2 I + K + L) mu = -(1/2 I + K) rho,
     K = K_self (singular rule, body blocks) + K_far (smooth rule, other bodies;
     optionally upsampled for near body pairs, see ``nearfield``);
  3. u = S[rho + mu] on every node; v_i = (1/|Gamma_i|) int u,
     omega_i = tau_i^{-1} int (y - x^c_i) x u                               (§3.3)

Vectors are (N, 3) arrays over the global nodes, bodies contiguous, node a of body
i at global index i*M + a.  Poses: R_i = R(q_i), q = (w, x, y, z) maps the body
frame to the lab frame; lab node X = c_i + R_i (x - x^c) where c_i is the lab area
centroid.  The sign convention of the loads: F_i is the force the body exerts on
the fluid (its surface traction integrates to -F_i, §2 force/torque conditions), so
an isolated sphere moves with v = F/(6 pi eta a).
"""
import math

import numpy as np

from . import farfield as ff
from . import geometry as geo
from . import nearfield as nf
from . import singular as sg


def quat_to_rot(q):
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


class _LazyR:
    """Per-shape fine-grid bounding radii, computed when indexed."""

    def __init__(self, prob):
        self.prob = prob

    def __getitem__(self, s):
        return self.prob.fine(int(s))["R"]


class Shape:
    """One body shape: geometry at the grid plus its singular self operators."""

    def __init__(self, coef, p, ps=None, eta=1.0, with_ops=True):
        self.p = p
        self.ps = 2 * p if ps is None else ps
        self.eta = eta
        self.coef = np.asarray(coef, dtype=np.float64)
        self.geom = geo.shape_geometry(self.coef, p)
        self.M = self.geom["grid"]["M"]
        self.ops = None
        if with_ops:
            self.ops = sg.singular_operators(self.coef, p, self.ps, eta)


class Problem:
    """The discrete problem; ``upsample = (p_u, kappa)`` switches on the near-singular
    rule of ``nearfield`` for body pairs that are near (None: plain smooth rule)."""

    def __init__(self, shapes, shape_id, centres, quats, eta=1.0, upsample=None):
        self.shapes = shapes
        self.shape_id = np.asarray(shape_id, dtype=np.int64)
        self.n = len(self.shape_id)
        self.M = shapes[0].M
        self.N = self.n * self.M
        self.eta = eta
        self.c = np.asarray(centres, dtype=np.float64).reshape(self.n, 3)
        self.R = np.array([quat_to_rot(q) for q in np.asarray(quats).reshape(self.n, 4)])
        X, Nn, w, body = [], [], [], []
        for i in range(self.n):
            g = shapes[self.shape_id[i]].geom
            X.append((self.c[i][:, None] + self.R[i] @ g["r"]).T)
            Nn.append((self.R[i] @ g["n"]).T)
            w.append(g["w"])
            body.append(np.full(self.M, i))
        self.X = np.concatenate(X)
        self.Nn = np.concatenate(Nn)
        self.w = np.concatenate(w)
        self.body = np.concatenate(body)
        # lab-frame area and tau recomputed from the lab points (§2.2)
        self.area = np.zeros(self.n)
        self.tau = np.zeros((self.n, 3, 3))
        for i in range(self.n):
            sl = self.sl(i)
            rr = self.X[sl] - self.c[i]
            wi = self.w[sl]
            self.area[i] = wi.sum()
            self.tau[i] = np.eye(3) * np.sum(wi * np.sum(rr * rr, axis=1)) - (rr * wi[:, None]).T @ rr
        self.upsample = upsample
        self._near = None if upsample is not None else np.zeros((self.n, self.n), dtype=bool)
        self._near_rows = {}
        if upsample is not None:
            p_u, kappa = upsample
            p = shapes[0].p
            self._fine = [None] * len(shapes)
            self.U = nf.interp_matrix(p, p_u)
            self._h = [math.sqrt(s.geom["area"] / s.M) for s in shapes]

    # The fine geometry of a shape and the near test of a body are evaluated on first use
    # (large suspensions need them only for a few bodies); the values are those of
    # ``nearfield.fine_geometry`` and ``nearfield.near_matrix``.
    def fine(self, s):
        if self._fine[s] is None:
            sh_ = self.shapes[s]
            self._fine[s] = nf.fine_geometry(sh_.coef, sh_.geom["xc"], self.upsample[0])
        return self._fine[s]

    @property
    def near(self):
        """near[i, j]: body j is near body i (all bodies)."""
        if self._near is None:
            R = [self.fine(s)["R"] for s in range(len(self.shapes))]
            self._near = nf.near_matrix(self.c, R, self._h, self.shape_id, self.upsample[1])
        return self._near

    def near_row(self, i):
        """Row i of ``near``, computed from the bodies that can possibly be near i: a fine
        grid's bounding radius is within a factor 2 of the coarse grid's."""
        if self._near is not None:
            return self._near[i]
        if i not in self._near_rows:
            rc = [float(np.sqrt(np.max(np.sum(s_.geom["r"] ** 2, axis=0)))) for s_ in self.shapes]
            reach = 2.0 * rc[self.shape_id[i]] + 2.0 * max(rc) + self.upsample[1] * max(self._h)
            dist = np.sqrt(np.sum((self.c - self.c[i]) ** 2, axis=1))
            cand = np.where(dist < reach)[0]                # includes i itself
            sub = nf.near_matrix(self.c[cand], _LazyR(self), self._h, self.shape_id[cand], self.upsample[1])
            row = np.zeros(self.n, dtype=bool)
            row[cand] = sub[int(np.where(cand == i)[0][0])]
            self._near_rows[i] = row
        return self._near_rows[i]

    def fine_sources(self, j):
        """Lab-frame fine nodes X' of body j and their weights w'."""
        f = self.fine(self.shape_id[j])
        return (self.c[j][:, None] + self.R[j] @ f["r"]).T, f["w"]

    def _far_upsampled(self, kind, vec, idx):
        """Off-body sum at the targets idx with the plain rule for pairs that are not
        near and the upsampled rule for near ones."""
        out = np.zeros((len(idx), 3))
        tb = self.body[idx]
        for i in np.unique(tb):
            sel = np.where(tb == i)[0]
            Xt = self.X[idx[sel]]
            near_i = self.near_row(i)
            for j in range(self.n):
                if j == i:
                    continue
                if near_i[j]:
                    Xs, ws = self.fine_sources(j)
                    q = ws[:, None] * (self.U @ vec[self.sl(j)])
                else:
                    Xs, q = self.X[self.sl(j)], self.w[self.sl(j)][:, None] * vec[self.sl(j)]
                if kind == "K":
                    out[sel] += nf.traction_block(Xt, self.Nn[idx[sel]], Xs, q)
                else:
                    out[sel] += nf.stokeslet_block(Xt, Xs, q, self.eta)
        return out

    def sl(self, i):
        return slice(i * self.M, (i + 1) * self.M)

    # ---- body-block operators (lab frame) ---------------------------------------
    def _apply_body_op(self, kind, i, v):
        """Lab-frame block of the body-frame operator 'S' or 'K' applied to v (M,3)."""
        A0 = self.shapes[self.shape_id[i]].ops[kind]
        R = self.R[i]
        vb = (v @ R).T.reshape(-1)          # body-frame components, c*M + a
        yb = (A0 @ vb).reshape(3, self.M).T
        return yb @ R.T

    def K_self(self, mu):
        out = np.zeros_like(mu)
        for i in range(self.n):
            out[self.sl(i)] = self._apply_body_op("K", i, mu[self.sl(i)])
        return out

    def S_self(self, sig):
        out = np.zeros_like(sig)
        for i in range(self.n):
            out[self.sl(i)] = self._apply_body_op("S", i, sig[self.sl(i)])
        return out

    def L_apply(self, mu):
        """L_i[mu](x) = int mu + (int (y - x^c) x mu) x (x - x^c)   (§2.3)."""
        out = np.zeros_like(mu)
        for i in range(self.n):
            sl = self.sl(i)
            rr = self.X[sl] - self.c[i]
            wi = self.w[sl][:, None]
            Fm = np.sum(wi * mu[sl], axis=0)
            Tm = np.sum(wi * np.cross(rr, mu[sl]), axis=0)
            out[sl] = Fm[None, :] + np.cross(Tm[None, :], rr)
        return out

    def K_far(self, mu, targets=None):
        idx = np.arange(self.N) if targets is None else np.asarray(targets)
        if self.upsample is not None:
            return self._far_upsampled("K", mu, idx)
        q = self.w[:, None] * mu
        return ff.traction_sum(self.X[idx], self.Nn[idx], self.X, q, self.body[idx], self.body)

    def S_far(self, sig, targets=None):
        idx = np.arange(self.N) if targets is None else np.asarray(targets)
        if self.upsample is not None:
            return self._far_upsampled("S", sig, idx)
        q = self.w[:, None] * sig
        return ff.stokeslet_sum(self.X[idx], self.X, q, self.body[idx], self.body, self.eta)

    # ---- the method ----------------------------------------------------------
    def incident_density(self, FT):
        """rho of §2.2 (eq. for rho_i): F_i/|Gamma_i| + tau_i^{-1} T_i x (x - x^c_i)."""
        FT = np.asarray(FT, dtype=np.float64).reshape(self.n, 6)
        rho = np.zeros((self.N, 3))
        for i in range(self.n):
            sl = self.sl(i)
            rr = self.X[sl] - self.c[i]
            Om = np.linalg.solve(self.tau[i], FT[i, 3:])
            rho[sl] = FT[i, :3][None, :] / self.area[i] + np.cross(Om[None, :], rr)
        return rho

    def apply_A(self, mu):
        """(1/2 I + K + L) mu, the augmented operator of §2.3."""
        return 0.5 * mu + self.K_self(mu) + self.K_far(mu) + self.L_apply(mu)

    def rhs(self, rho):
        """-(1/2 I + K) rho."""
        return -(0.5 * rho + self.K_self(rho) + self.K_far(rho))

    def dense_matrix(self):
        """The augmented operator as a dense (3N x 3N) matrix acting on the flattened
        (N, 3) vector (index 3*g + c): 1/2 I + body blocks (lab K_self + L) + the
        smooth-rule traction matrix between different bodies."""
        N, M = self.N, self.M
        A = 0.5 * np.eye(3 * N)
        for i in range(self.n):
            R = self.R[i]
            K0 = self.shapes[self.shape_id[i]].ops["K"].reshape(3, M, 3, M)
            Kl = np.einsum("ce,eafb,gf->acbg", R, K0, R).reshape(3 * M, 3 * M)
            rr = self.X[self.sl(i)] - self.c[i]
            wi = self.w[self.sl(i)]
            cx = np.zeros((M, 3, 3))
            cx[:, 0, 1], cx[:, 0, 2], cx[:, 1, 2] = -rr[:, 2], rr[:, 1], -rr[:, 0]
            cx[:, 1, 0], cx[:, 2, 0], cx[:, 2, 1] = rr[:, 2], -rr[:, 1], rr[:, 0]
            Lb = (np.eye(3)[None, None] - np.einsum("aij,bjk->abik", cx, cx)) * wi[None, :, None, None]
            Ll = np.transpose(Lb, (0, 2, 1, 3)).reshape(3 * M, 3 * M)
            s3 = slice(3 * i * M, 3 * (i + 1) * M)
            A[s3, s3] += Kl + Ll
        d = self.X[:, None, :] - self.X[None, :, :]
        r2 = np.sum(d * d, axis=2)
        other = self.body[:, None] != self.body[None, :]
        r2[~other] = 1.0
        dn = np.einsum("abk,ak->ab", d, self.Nn)
        fac = -(3.0 / (4.0 * math.pi)) * dn / (r2 * r2 * np.sqrt(r2)) * self.w[None, :]
        fac[~other] = 0.0
        Kf = np.einsum("ab,abi,abj->aibj", fac, d, d)
        for i, j in zip(*np.nonzero(self.near)):
            Xs, ws = self.fine_sources(j)
            Bf = nf.traction_matrix_block(self.X[self.sl(i)], self.Nn[self.sl(i)], Xs, ws)
            Kf[self.sl(i), :, self.sl(j), :] = np.einsum("aibj,bc->aicj", Bf, self.U)
        return A + Kf.reshape(3 * N, 3 * N)

    def velocities(self, rho, mu):
        """(v_i, omega_i) from u = S[rho + mu] (§3.3)."""
        sig = rho + mu
        u = self.S_self(sig) + self.S_far(sig)
        return self.project_rigid(u)

    def project_rigid(self, u):
        VW = np.zeros((self.n, 6))
        for i in range(self.n):
            sl = self.sl(i)
            rr = self.X[sl] - self.c[i]
            wi = self.w[sl][:, None]
            VW[i, :3] = np.sum(wi * u[sl], axis=0) / self.area[i]
            VW[i, 3:] = np.linalg.solve(self.tau[i], np.sum(wi * np.cross(rr, u[sl]), axis=0))
        return VW


def solve_dense(prob, FT):
    """Exact discrete solution by LU with partial pivoting (small problems)."""
    rho = prob.incident_density(FT)
    b = prob.rhs(rho).reshape(-1)
    if np.linalg.norm(b) == 0.0:
        mu = np.zeros_like(rho)
    else:
        mu = np.linalg.solve(prob.dense_matrix(), b).reshape(prob.N, 3)
    return rho, mu, prob.velocities(rho, mu)


def solve_dense_density(prob, rho):
    """As ``solve_dense`` for a given incident density rho (N, 3) (e.g. a Maxwell traction,
    §4) in place of F/|Gamma| + tau^{-1} T x (x - x^c)."""
    rho = np.asarray(rho, dtype=np.float64).reshape(prob.N, 3)
    b = prob.rhs(rho).reshape(-1)
    mu = np.zeros_like(rho) if np.linalg.norm(b) == 0.0 else \
        np.linalg.solve(prob.dense_matrix(), b).reshape(prob.N, 3)
    return mu, prob.velocities(rho, mu)


def gmres(apply, b, tol, maxit=500, x0=None):
    """Unrestarted GMRES with modified Gram-Schmidt Arnoldi and Givens rotations;
    stops when the true residual ||b - A x|| <= tol ||b||.  Returns x, iterations."""
    n = b.size
    x = np.zeros(n) if x0 is None else x0.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros(n), 0
    r = b - apply(x)
    beta = np.linalg.norm(r)
    if beta <= tol * bn:
        return x, 0
    V = np.zeros((maxit + 1, n))
    H = np.zeros((maxit + 1, maxit))
    cs, sn = np.zeros(maxit), np.zeros(maxit)
    g = np.zeros(maxit + 1)
    V[0] = r / beta
    g[0] = beta
    k = 0
    for k in range(maxit):
        w = apply(V[k])
        for j in range(k + 1):
            H[j, k] = V[j] @ w
            w = w - H[j, k] * V[j]
        H[k + 1, k] = np.linalg.norm(w)
        if H[k + 1, k] > 0:
            V[k + 1] = w / H[k + 1, k]
        for j in range(k):
            t = cs[j] * H[j, k] + sn[j] * H[j + 1, k]
            H[j + 1, k] = -sn[j] * H[j, k] + cs[j] * H[j + 1, k]
            H[j, k] = t
        den = math.hypot(H[k, k], H[k + 1, k])
        cs[k], sn[k] = H[k, k] / den, H[k + 1, k] / den
        H[k, k] = den
        H[k + 1, k] = 0.0
        g[k + 1] = -sn[k] * g[k]
        g[k] = cs[k] * g[k]
        if abs(g[k + 1]) <= tol * bn:
            break
    m = k + 1
    y = np.linalg.solve(np.triu(H[:m, :m]), g[:m])
    x = x + V[:m].T @ y
    return x, m


def solve_gmres(prob, FT, tol=1e-12, maxit=500):
    rho = prob.incident_density(FT)
    b = prob.rhs(rho).reshape(-1)
    x, its = gmres(lambda v: prob.apply_A(v.reshape(prob.N, 3)).reshape(-1), b, tol, maxit)
    mu = x.reshape(prob.N, 3)
    return rho, mu, prob.velocities(rho, mu), its


def mobility_matrix(prob):
    """6n x 6n mobility matrix M with V = M F (§1), from 6n unit-load dense solves."""
    n6 = 6 * prob.n
    A = prob.dense_matrix()
    Mm = np.zeros((n6, n6))
    for j in range(n6):
        FT = np.zeros(n6)
        FT[j] = 1.0
        rho = prob.incident_density(FT)
        b = prob.rhs(rho).reshape(-1)
        mu = np.zeros_like(rho) if np.linalg.norm(b) == 0 else np.linalg.solve(A, b).reshape(prob.N, 3)
        Mm[:, j] = prob.velocities(rho, mu).reshape(-1)
    return Mm
