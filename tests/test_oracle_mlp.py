"""Pins of the oracle's learned-warm-start pieces: bf16 rounding against torch,
gradients against finite differences, Adam's first step, invariances of the
features, analysis as the left inverse of synthesis."""
import numpy as np
import pytest
import torch

from oracle import mlp
from oracle import system as sy
from oracle import timestep as ts


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(2000) * 10 ** rng.uniform(-6, 6, 2000),
                        [1 + 2 ** -8, 1 + 3 * 2 ** -9, -1 - 2 ** -8, 0.0, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)


def _net(rng, dims):
    return [(rng.standard_normal((a, b)) / np.sqrt(a), 0.1 * rng.standard_normal(b))
            for a, b in zip(dims[:-1], dims[1:])]


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    params = _net(rng, [7, 11, 9, 5])
    X = rng.standard_normal((13, 7))
    T = rng.standard_normal((13, 5))
    loss, grads = mlp.loss_and_grads(params, X, T)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for k, P in enumerate((W, b)):
            idx = tuple(rng.integers(0, s) for s in P.shape)
            Pp = [list(t) for t in params]
            Q = P.copy()
            Q[idx] += h
            Pp[li][k] = Q
            lp = mlp.loss_and_grads([tuple(t) for t in Pp], X, T)[0]
            Q = P.copy()
            Q[idx] -= h
            Pp[li][k] = Q
            lm = mlp.loss_and_grads([tuple(t) for t in Pp], X, T)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[li][k][idx]) <= 1e-7 * max(1.0, abs(fd))


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(2)
    params = _net(rng, [3, 4])
    grads = [(rng.standard_normal((3, 4)), rng.standard_normal(4))]
    state = {"t": 0, "m": [[np.zeros((3, 4)), np.zeros(4)]], "v": [[np.zeros((3, 4)), np.zeros(4)]]}
    new = mlp.adam_step(params, grads, state, lr=0.01, eps=0.0)
    assert np.allclose(params[0][0] - new[0][0], 0.01 * np.sign(grads[0][0]), atol=1e-15)


def _config(rng, n):
    c = rng.uniform(-5, 5, (n, 3))
    q = ts.normalize(rng.standard_normal((n, 4)))
    R = np.array([sy.quat_to_rot(x) for x in q])
    FT = rng.standard_normal((n, 6))
    return c, R, FT


def test_features_are_rigid_motion_and_permutation_invariant():
    rng = np.random.default_rng(3)
    n, k = 12, 5
    c, R, FT = _config(rng, n)
    desc = rng.standard_normal((n, 4))
    X = mlp.features(c, R, FT, desc, k)
    assert X.shape == (n, 6 + 4 + 15 * k)
    Q = sy.quat_to_rot(ts.normalize(rng.standard_normal(4)))
    c2 = c @ Q.T + np.array([3.0, -1.0, 2.0])
    R2 = np.einsum("ab,ibc->iac", Q, R)
    FT2 = np.concatenate([FT[:, :3] @ Q.T, FT[:, 3:] @ Q.T], axis=1)
    assert np.abs(mlp.features(c2, R2, FT2, desc, k) - X).max() < 1e-12
    perm = rng.permutation(n)
    assert np.abs(mlp.features(c[perm], R[perm], FT[perm], desc[perm], k) - X[perm]).max() < 1e-12


def test_features_pad_when_few_neighbours():
    rng = np.random.default_rng(4)
    c, R, FT = _config(rng, 3)
    X = mlp.features(c, R, FT, np.zeros((3, 0)), 4)
    assert np.all(X[:, 6 + 15 * 2:] == 0.0)
    assert np.all(np.abs(X[:, 6:6 + 15 * 2]).sum(axis=1) > 0)


@pytest.mark.parametrize("p", [4, 7])
def test_analysis_is_left_inverse_of_synthesis(p):
    rng = np.random.default_rng(p)
    n = 3
    R = np.array([sy.quat_to_rot(ts.normalize(rng.standard_normal(4))) for _ in range(n)])
    coef = rng.standard_normal((n, 3 * (p * p + 2 * p)))
    dmu = mlp.synthesize(coef, R, p)
    assert np.abs(mlp.band_targets(dmu, R, p) - coef).max() < 1e-12
