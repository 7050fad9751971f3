"""Learned GMRES warm start: features, targets and the per-body MLP, FP64 oracle.

Test infrastructure only (see ``oracle/__init__``).

This part is not in the paper; it is defined by the build's specification of the
warm start.  For body i, in its own frame (R_i^T applied to every lab vector):
  * own load R^T F_i, R^T T_i;
  * its shape descriptor (the first S radial SH coefficients, zero padded);
  * for each of its k nearest neighbours j (centre distance, ties to the lower
    index, zero rows when fewer exist): e = R^T d/|d|^2 with d = c_j - c_i, the
    first two columns of R_i^T R_j, R^T F_j and R^T T_j.
Output: the body-frame band coefficients (§3 forward transform F) of the density
correction mu* - mu_BD, mu_BD = P^{-1} b the block-diagonal (isolated-particle)
guess; layout [component][band index].  Network: dense layers with SiLU between
them, MSE loss, Adam.  With ``bf16=True`` every GEMM operand is rounded to
bfloat16 (round to nearest even) as the GPU's MFMA path does, the products and
sums staying in float64.
"""
import numpy as np

from . import sphharm as sh


def bf16_round(x):
    """Round float64 values to the nearest bfloat16 (ties to even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(c, R, FT, shape_desc, k):
    """Feature matrix (n, 6 + S + 15 k); c (n,3), R (n,3,3), FT (n,6), shape_desc (n,S)."""
    n = len(c)
    S = shape_desc.shape[1]
    X = np.zeros((n, 6 + S + 15 * k))
    for i in range(n):
        Rt = R[i].T
        X[i, 0:3] = Rt @ FT[i, :3]
        X[i, 3:6] = Rt @ FT[i, 3:]
        X[i, 6:6 + S] = shape_desc[i]
        d2 = np.sum((c - c[i]) ** 2, axis=1)
        d2[i] = np.inf
        order = np.lexsort((np.arange(n), d2))[: min(k, n - 1)]
        for slot, j in enumerate(order):
            off = 6 + S + 15 * slot
            d = c[j] - c[i]
            X[i, off:off + 3] = Rt @ d / (d @ d)
            Q = Rt @ R[j]
            X[i, off + 3:off + 6] = Q[:, 0]
            X[i, off + 6:off + 9] = Q[:, 1]
            X[i, off + 9:off + 12] = Rt @ FT[j, :3]
            X[i, off + 12:off + 15] = Rt @ FT[j, 3:]
    return X


def band_targets(dmu, R, p):
    """Body-frame band coefficients of a lab density dmu (N, 3): (n, 3 |B_p|)."""
    F = sh.forward_matrix(p)
    n = len(R)
    M = dmu.shape[0] // n
    out = np.zeros((n, 3 * F.shape[0]))
    for i in range(n):
        body = dmu[i * M:(i + 1) * M] @ R[i]          # (M, 3) body-frame components
        out[i] = (F @ body).T.reshape(-1)
    return out


def synthesize(coef, R, p):
    """Lab density (N, 3) from body-frame band coefficients (n, 3 |B_p|)."""
    g = sh.grid(p)
    Y = sh.synthesis_matrix(p, g["theta_a"], g["phi_a"])   # (|B|, M)
    nB = Y.shape[0]
    out = []
    for i in range(len(R)):
        cb = coef[i].reshape(3, nB)
        body = (cb @ Y).T                                    # (M, 3)
        out.append(body @ R[i].T)
    return np.concatenate(out)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, X, bf16=False):
    """params: list of (W (in, out), b (out,)).  Returns output and cache."""
    rnd = bf16_round if bf16 else (lambda a: a)
    A = X
    cache = []
    for li, (W, b) in enumerate(params):
        Z = rnd(A) @ rnd(W) + b
        cache.append((A, Z))
        A = silu(Z) if li < len(params) - 1 else Z
    return A, cache


def loss_and_grads(params, X, T, bf16=False):
    """MSE = mean over rows and outputs of (Y - T)^2, and its parameter gradients."""
    rnd = bf16_round if bf16 else (lambda a: a)
    Y, cache = forward(params, X, bf16)
    R, O = Y.shape
    loss = np.mean((Y - T) ** 2)
    dZ = 2.0 * (Y - T) / (R * O)
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        A, Z = cache[li]
        W, _ = params[li]
        if li < len(params) - 1:
            dZ = dZ * dsilu(Z)
        grads[li] = (rnd(A).T @ rnd(dZ), dZ.sum(axis=0))
        dA = rnd(dZ) @ rnd(W).T
        dZ = dA
    return loss, grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); state = dict(t, m, v) updated in place."""
    state["t"] += 1
    t = state["t"]
    new = []
    for li, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        out = []
        for k, (P, G) in enumerate(((W, gW), (b, gb))):
            m = state["m"][li][k] = beta1 * state["m"][li][k] + (1 - beta1) * G
            v = state["v"][li][k] = beta2 * state["v"][li][k] + (1 - beta2) * G * G
            mh = m / (1 - beta1 ** t)
            vh = v / (1 - beta2 ** t)
            out.append(P - lr * mh / (np.sqrt(vh) + eps))
        new.append(tuple(out))
    return new
