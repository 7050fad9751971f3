"""Learned warm start on the GPU against the oracle: features, network forward and
gradients (bf16 MFMA vs float64 with bf16-rounded operands), captured targets,
synthesis of the guess, and the effect of training and of a corrupted network."""
import math

import numpy as np
import pytest

from paper_1606_07428_amd import inputs, rbm
from oracle import mlp
from oracle import system as sy
from tests.helpers import oracle_problem, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _desc(w):
    L = max(len(d) for _, d in w["shapes"])
    D = np.zeros((len(w["shapes"]), L))
    for i, (_, d) in enumerate(w["shapes"]):
        D[i, :len(d)] = d
    return D[w["shape_id"]]


def _flat(params):
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in params]).astype(np.float32)


def test_features_match_oracle():
    _case("features n=9 p=6 k=4")
    w = inputs.tiny(9, 6, seed=41)
    s = rbm.solver_for(w)
    info = s.learned_bind(k_nbr=4, hidden=16, n_hidden=1, capacity=64, batch_max=32)
    FT = torch.as_tensor(np.asarray(w["FT"]), device="cuda")
    X = torch.zeros((s.n, info["F"]), dtype=torch.float32, device="cuda")
    s.learned_features(FT, X)
    prob = oracle_problem(w, with_ops=False)
    Xo = mlp.features(prob.c, prob.R, np.asarray(w["FT"]), _desc(w), 4)
    assert Xo.shape == tuple(X.shape)
    assert np.abs(X.cpu().numpy() - Xo).max() < 2e-6 * np.abs(Xo).max()
    s.close()


@pytest.mark.parametrize("side,jitter,k", [(6, 0.0, 16), (5, 0.3, 8)])
def test_features_match_oracle_beyond_one_wave(side, jitter, k):
    """More bodies than lanes in a wave; on the unjittered lattice many neighbours are at
    exactly equal distances, where both sides order by body index."""
    _case(f"features lattice side={side} jitter={jitter} k={k}")
    w = inputs.mhd_lattice(side=side, p=2, spacing=3.0, jitter=jitter, seed=3)
    rng = np.random.default_rng(side)
    q = rng.standard_normal((len(w["centres"]), 4))
    w["quats"] = q / np.linalg.norm(q, axis=1, keepdims=True)
    w["FT"] = rng.standard_normal((len(w["centres"]), 6))
    s = rbm.solver_for(w)
    info = s.learned_bind(k_nbr=k, hidden=16, n_hidden=1, capacity=64, batch_max=32)
    FT = torch.as_tensor(np.asarray(w["FT"]), device="cuda")
    X = torch.zeros((s.n, info["F"]), dtype=torch.float32, device="cuda")
    s.learned_features(FT, X)
    prob = oracle_problem(w, with_ops=False)
    Xo = mlp.features(prob.c, prob.R, np.asarray(w["FT"]), _desc(w), k)
    assert np.abs(X.cpu().numpy() - Xo).max() < 2e-6 * np.abs(Xo).max()
    s.close()


def test_forward_and_gradients_match_oracle():
    _case("mlp forward/backward vs oracle bf16")
    w = inputs.tiny(3, 5, seed=42)
    s = rbm.solver_for(w)
    info = s.learned_bind(k_nbr=2, hidden=48, n_hidden=2, capacity=64, batch_max=128)
    F, O = info["F"], info["O"]
    rng = np.random.default_rng(0)
    dims = [F, 48, 48, O]
    params = [((rng.standard_normal((a, b)) / math.sqrt(a)).astype(np.float32).astype(np.float64),
               (0.1 * rng.standard_normal(b)).astype(np.float32).astype(np.float64))
              for a, b in zip(dims[:-1], dims[1:])]
    flat = np.concatenate([_flat(params), np.zeros(F, np.float32), np.ones(F, np.float32),
                           np.ones(2, np.float32)])
    s.learned_set_params(flat)
    rows = 77
    X = rng.standard_normal((rows, F)).astype(np.float32)
    T = rng.standard_normal((rows, O)).astype(np.float32)
    Xd = torch.as_tensor(X, device="cuda")
    Td = torch.as_tensor(T, device="cuda")
    Yd = torch.zeros((rows, O), dtype=torch.float32, device="cuda")
    s.learned_forward(Xd, Yd)
    Yo, _ = mlp.forward(params, X.astype(np.float64), bf16=True)
    Y = Yd.cpu().numpy()
    assert np.linalg.norm(Y - Yo) / np.linalg.norm(Yo) < 3e-3
    G = torch.zeros(info["n_params"], dtype=torch.float32, device="cuda")
    loss = s.learned_loss_grad(Xd, Td, G)
    lo, go = mlp.loss_and_grads(params, X.astype(np.float64), T.astype(np.float64), bf16=True)
    assert abs(loss - lo) < 1e-3 * lo
    g = G.cpu().numpy().astype(np.float64)
    off = 0
    for (gW, gb) in go:
        for ref in (gW.reshape(-1), gb):
            got = g[off:off + ref.size]
            off += ref.size
            cos = got @ ref / (np.linalg.norm(got) * np.linalg.norm(ref))
            assert cos > 0.999, cos
            assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 2e-2
    s.close()


def _mu_bd_oracle(prob, b):
    out = np.zeros_like(b)
    for i in range(prob.n):
        sh = prob.shapes[prob.shape_id[i]]
        A0 = 0.5 * np.eye(3 * prob.M) + sh.ops["K"] + __import__("oracle.singular", fromlist=["x"]).L_operator(sh.geom)
        R = prob.R[i]
        bb = (b[prob.sl(i)] @ R).T.reshape(-1)
        out[prob.sl(i)] = np.linalg.solve(A0, bb).reshape(3, prob.M).T @ R.T
    return out


def test_captured_targets_and_guess_synthesis_match_oracle():
    _case("capture + guess synthesis n=4 p=6")
    w = inputs.tiny(4, 6, seed=43)
    s = rbm.solver_for(w, tol=1e-13)
    info = s.learned_bind(k_nbr=3, hidden=16, n_hidden=1, capacity=64, batch_max=32)
    F, O = info["F"], info["O"]
    FT = torch.as_tensor(np.asarray(w["FT"]), device="cuda")
    VW = torch.zeros_like(FT)
    s.solve_dev(FT, VW)
    s.learned_capture(FT)
    assert s.learned_info()["samples"] == s.n
    mu_g, _ = s.density()
    prob = oracle_problem(w)
    rho = prob.incident_density(w["FT"])
    mu_bd = _mu_bd_oracle(prob, prob.rhs(rho))
    T_ref = mlp.band_targets(mu_g.T - mu_bd, prob.R, w["p"])
    T_gpu = s.read("learned_T", s.n * O, dtype=np.float32).reshape(s.n, O)
    assert np.abs(T_gpu - T_ref).max() < 1e-5 * np.abs(T_ref).max()
    X_gpu = s.read("learned_X", s.n * F, dtype=np.float32).reshape(s.n, F)
    X_ref = mlp.features(prob.c, prob.R, np.asarray(w["FT"]), _desc(w), 3)
    assert np.abs(X_gpu - X_ref).max() < 2e-6 * np.abs(X_ref).max()
    # a network that outputs a fixed coefficient vector (zero weights, last bias = c)
    n_par = info["n_params"]
    rng = np.random.default_rng(1)
    cvec = (0.01 * rng.standard_normal(O)).astype(np.float32)
    flat = np.zeros(n_par + 2 * F + 2, np.float32)
    flat[n_par - O:n_par] = cvec
    flat[n_par + F:n_par + 2 * F] = 1.0
    flat[n_par + 2 * F:] = [2.0, 0.5]
    s.learned_set_params(flat)
    mu0 = torch.zeros((3, s.N), dtype=torch.float64, device="cuda")
    s.learned_guess(FT, mu0)
    ref = mu_bd + mlp.synthesize(np.tile(2.0 * cvec.astype(np.float64), (s.n, 1)), prob.R, w["p"])
    assert rel_err(mu0.cpu().numpy().T, ref) < 1e-10
    s.close()


def test_training_on_time_stepping_reduces_iterations_and_fallback_on_garbage():
    _case("train on RK4 solves, 16 bodies p=6")
    w = inputs.workload_perturbed(16, 6, 0.10, 0.5, np.random.default_rng(44), lmax=3)
    w["FT"][:, :3] = [0.0, 0.0, -1.0]
    w["FT"][:, 3:] = math.sqrt(0.1) * np.random.default_rng(45).standard_normal((16, 3))
    s = rbm.solver_for(w, tol=1e-10, guess=rbm.GUESS_BLOCKDIAG)
    s.learned_bind(k_nbr=8, hidden=128, n_hidden=2, capacity=4096, batch_max=256, seed=5)
    FT = torch.as_tensor(np.asarray(w["FT"]), device="cuda")
    s.learned_set_capture(True)
    for _ in range(12):
        s.step_rk4(0.5, FT)
    s.learned_set_capture(False)
    assert s.learned_info()["samples"] == 12 * 4 * 16
    l0 = s.learned_train(1, 64, 1e-3)
    l1 = s.learned_train(150, 64, 1e-3)
    print(f"loss {l0:.3e} -> {l1:.3e}", flush=True)
    assert l1 < 0.3 * l0
    VW = torch.zeros_like(FT)
    its = {"bd": [], "learned": []}
    res = {"bd": [], "learned": []}
    for _ in range(3):
        s.step_rk4(0.5, FT)
        for name, g in (("bd", rbm.GUESS_BLOCKDIAG), ("learned", rbm.GUESS_LEARNED)):
            s.set_guess_mode(g)
            info = s.solve_dev(FT, VW)
            its[name].append(info["iters"])
            res[name].append(info["init_rel_residual"])
            assert info["rel_residual"] < 1e-10
    print(its, res, flush=True)
    assert np.mean(res["learned"]) < 0.7 * np.mean(res["bd"])
    assert sum(its["learned"]) <= sum(its["bd"])
    # a corrupted network is rejected for the block-diagonal guess
    p = s.learned_params()
    p[: len(p) // 2] = 50.0
    s.learned_set_params(p)
    s.set_guess_mode(rbm.GUESS_LEARNED)
    info = s.solve_dev(FT, VW)
    assert info["fallback_used"] == 1 and info["rel_residual"] < 1e-10
    s.close()


def test_capture_buffer_is_a_ring():
    """Capacity of two solves' bodies, three captures: the third overwrites the first."""
    _case("capture ring buffer: capacity 2n, three captures, n=4 p=6")
    w = inputs.tiny(4, 6, seed=44)
    s = rbm.solver_for(w, tol=1e-12)
    info = s.learned_bind(k_nbr=3, hidden=16, n_hidden=1, capacity=2 * 4, batch_max=8)
    F = info["F"]
    prob = oracle_problem(w)
    rng = np.random.default_rng(3)
    FTs = [rng.standard_normal((4, 6)) for _ in range(3)]
    for k, FTk in enumerate(FTs):
        FT = torch.as_tensor(FTk, device="cuda")
        VW = torch.zeros_like(FT)
        s.solve_dev(FT, VW)
        s.learned_capture(FT)
        assert s.learned_info()["samples"] == min(2, k + 1) * 4
    X = s.read("learned_X", 8 * F, dtype=np.float32).reshape(8, F)
    for rows, FTk in ((slice(0, 4), FTs[2]), (slice(4, 8), FTs[1])):
        ref = mlp.features(prob.c, prob.R, FTk, _desc(w), 3)
        assert np.abs(X[rows] - ref).max() < 2e-6 * np.abs(ref).max()
    assert np.isfinite(s.learned_train(2, 8, 1e-3))
    s.close()


def _unflat(flat, dims):
    out, off = [], 0
    for a, b in zip(dims[:-1], dims[1:]):
        W = flat[off:off + a * b].reshape(a, b).astype(np.float64)
        off += a * b
        out.append((W, flat[off:off + b].astype(np.float64)))
        off += b
    return out


def test_training_step_matches_oracle_standardisation_gradients_and_adam():
    """One rbm_learned_train epoch whose single batch holds every captured sample: the
    feature standardisation and target scale fixed from the buffer, the bf16 gradients and
    the Adam update (moments, bias-corrected step) against the oracle's statistics,
    loss_and_grads and adam_step on the same samples and initial weights."""
    _case("training step vs oracle: 12 samples, layers F-32-32-O")
    w = inputs.tiny(4, 6, seed=46)
    s = rbm.solver_for(w, tol=1e-12)
    info = s.learned_bind(k_nbr=3, hidden=32, n_hidden=2, capacity=12, batch_max=16, seed=9)
    F, O, npar = info["F"], info["O"], info["n_params"]
    rng = np.random.default_rng(12)
    for _ in range(3):
        FT = torch.as_tensor(rng.standard_normal((4, 6)), device="cuda")
        VW = torch.zeros_like(FT)
        s.solve_dev(FT, VW)
        s.learned_capture(FT)
    assert s.learned_info()["samples"] == 12
    P0 = s.learned_params()[:npar]
    X = s.read("learned_X", 12 * F, dtype=np.float32).reshape(12, F).astype(np.float64)
    T = s.read("learned_T", 12 * O, dtype=np.float32).reshape(12, O).astype(np.float64)
    lr = 1e-3
    loss = s.learned_train(1, 12, lr)
    after = s.learned_params()
    P1, mean, istd, tsc = after[:npar], after[npar:npar + F], after[npar + F:npar + 2 * F], after[-2:]
    m_g = s.read("learned_m", npar, dtype=np.float32).astype(np.float64)
    v_g = s.read("learned_v", npar, dtype=np.float32).astype(np.float64)
    # standardisation and target scale
    mean_o = X.mean(axis=0)
    var_o = X.var(axis=0)
    istd_o = np.where(var_o > 1e-20, 1.0 / np.sqrt(np.maximum(var_o, 1e-300)), 0.0)
    rms_o = math.sqrt(np.mean(T * T))
    assert np.abs(mean - mean_o).max() <= 1e-6 * max(np.abs(mean_o).max(), 1.0)
    assert np.abs(istd - istd_o).max() <= 1e-6 * np.abs(istd_o).max()
    assert abs(tsc[0] - rms_o) <= 1e-6 * rms_o and abs(tsc[1] - 1.0 / rms_o) <= 1e-6 / rms_o
    # gradients and Adam on the oracle
    dims = [F, 32, 32, O]
    params0 = _unflat(P0, dims)
    Xs = (X - mean_o) * istd_o
    loss_o, grads = mlp.loss_and_grads(params0, Xs, T / rms_o, bf16=True)
    state = {"t": 0, "m": [[np.zeros_like(W), np.zeros_like(b)] for W, b in params0],
             "v": [[np.zeros_like(W), np.zeros_like(b)] for W, b in params0]}
    params1 = mlp.adam_step(params0, grads, state, lr)
    assert abs(loss - loss_o) < 1e-2 * loss_o
    flat = lambda lst: np.concatenate([np.concatenate([a.reshape(-1), b]) for a, b in lst])  # noqa: E731
    m_o, v_o, g_o, P1_o = flat(state["m"]), flat(state["v"]), flat(grads), flat(params1)
    off = 0
    for a, b in zip(dims[:-1], dims[1:]):
        for size in (a * b, b):
            sl = slice(off, off + size)
            off += size
            for got, ref in ((m_g[sl], m_o[sl]), (v_g[sl], v_o[sl])):
                nr = np.linalg.norm(ref)
                if nr == 0.0:
                    assert np.abs(got).max() == 0.0
                    continue
                assert got @ ref / (np.linalg.norm(got) * nr) > 0.999
                assert np.linalg.norm(got - ref) / nr < 6e-2
            # Adam's first step moves each parameter by lr g / (|g| + eps): the two sides agree
            # except where bf16 rounding flips the sign of a gradient that is small next to
            # the tensor's largest
            d = np.abs(P1[sl] - P1_o[sl])
            big = np.abs(g_o[sl]) > 0.05 * np.abs(g_o[sl]).max()
            assert d[big].max(initial=0.0) < 1e-3 * lr + 1e-7 * np.abs(P1_o[sl]).max()
            assert np.mean(d > 1e-3 * lr + 1e-7 * np.abs(P1_o[sl]).max()) < 0.03
    s.close()
