"""rbm_far_traction_static (the no-allocation variant of rbm_far_traction) through the C ABI:
two calls in a row, the second on a smaller input, each against rbm_far_traction of a
context (same kernels and split, so bitwise equal) and the float64 one against the oracle's
direct sum at sampled targets."""
import math

import numpy as np
import pytest

from paper_1606_07428_amd import rbm
from oracle import farfield as ff
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _ctx(n_points, M):
    p = 2
    while 2 * p * (p + 1) < M:
        p += 1
    nb = -(-n_points // (2 * p * (p + 1)))
    w = {"p": p, "shapes": [("radial", [math.sqrt(4 * math.pi)])], "shape_id": np.zeros(nb, np.int32),
         "centres": np.arange(nb)[:, None] * np.array([[3.0, 0, 0]]), "quats": np.tile([1.0, 0, 0, 0], (nb, 1))}
    return rbm.solver_for(w)


@pytest.mark.parametrize("prec", [0, 1])
def test_static_scratch_sum_equals_the_context_sum(prec):
    M = 312
    s = _ctx(20000, M)
    for k, n_points in enumerate((20000, 5003)):
        print(f"\n[case] static far traction n={n_points} precision={prec} call {k + 1}", flush=True)
        rng = np.random.default_rng(n_points + prec)
        X = rng.uniform(-6, 6, (n_points, 3))
        Nn = rng.standard_normal((n_points, 3))
        Nn /= np.linalg.norm(Nn, axis=1)[:, None]
        q = rng.standard_normal((n_points, 3))
        add = rng.standard_normal((n_points, 3))
        Xd, Nd, qd, ad = _dev(X.T), _dev(Nn.T), _dev(q.T), _dev(add.T)
        y_static = rbm.far_traction_static(Xd, Nd, qd, M, add=ad, precision=prec)
        y_ctx = s.far_traction(Xd, Nd, qd, M, add=ad, precision=prec)
        torch.cuda.synchronize()
        a, b = y_static.cpu().numpy(), y_ctx.cpu().numpy()
        assert np.array_equal(a, b)
        if prec == 0:
            idx = rng.choice(n_points, 64, replace=False)
            body = np.arange(n_points) // M
            ref = add[idx] + ff.traction_sum(X[idx], Nn[idx], X, q, body[idx], body)
            assert rel_err(a.T[idx], ref) < 1e-12
    s.close()


def test_static_scratch_rejects_inputs_beyond_its_size():
    print("\n[case] static far traction: 900,000 points refused (no kernel runs)", flush=True)
    lib = rbm.load()
    dummy = torch.zeros(3, dtype=torch.float64, device="cuda")
    p = torch.cuda.current_stream().cuda_stream
    import ctypes
    st = lib.rbm_far_traction_static(900_000, 312, ctypes.c_void_p(dummy.data_ptr()), ctypes.c_void_p(dummy.data_ptr()),
                                     ctypes.c_void_p(dummy.data_ptr()), None, ctypes.c_void_p(dummy.data_ptr()), 0,
                                     ctypes.c_void_p(p))
    assert st == rbm.RBM_E_NOMEM
    assert b"static scratch" in lib.rbm_last_error()
