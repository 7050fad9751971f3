"""Failure handling through the C ABI, forced from the host (no kernel is made to
fault): non-convergence reports RBM_E_NOCONV with outputs written, call-order and
argument errors are rejected before any device work."""
import ctypes

import numpy as np
import pytest

from paper_1606_07428_amd import inputs, rbm

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_nonconvergence_writes_outputs_and_reports():
    print("\n[case] max_iter=1, max_restart=0, tol=1e-14", flush=True)
    w = inputs.tiny(4, 6, seed=51)
    s = rbm.solver_for(w, tol=1e-14, max_iter=1, max_restart=0)
    VW, info = s.solve(w["FT"])
    assert s.last_status == rbm.RBM_E_NOCONV
    assert info["iters"] == 1 and info["rel_residual"] > 1e-14
    assert np.all(np.isfinite(VW)) and np.abs(VW).max() > 0
    s.close()


def test_user_guess_requires_a_guess_and_is_used():
    print("\n[case] RBM_GUESS_USER", flush=True)
    w = inputs.tiny(3, 6, seed=52)
    s = rbm.solver_for(w, tol=1e-12, guess=rbm.GUESS_USER)
    with pytest.raises(rbm.RbmError) as e:
        s.solve(w["FT"])
    assert e.value.status == rbm.RBM_E_STATE
    ref = rbm.solver_for(w, tol=1e-13)
    VW_ref, _ = ref.solve(w["FT"])
    mu, _ = ref.density()
    s.set_guess_dev(torch.as_tensor(mu, device="cuda"))
    VW, info = s.solve(w["FT"])
    assert info["iters"] <= 1 and info["init_rel_residual"] < 1e-12
    assert np.abs(VW - VW_ref).max() < 1e-11 * np.abs(VW_ref).max()
    s.close()
    ref.close()


def test_argument_and_order_errors():
    print("\n[case] argument / order errors", flush=True)
    w = inputs.tiny(3, 5, seed=53)
    s = rbm.solver_for(w)
    lib = rbm.load()
    FT = torch.as_tensor(np.asarray(w["FT"]), device="cuda")
    assert lib.rbm_step_rk4(s.ctx, -1.0, ctypes.c_void_p(FT.data_ptr()), None) == rbm.RBM_E_INVAL
    assert lib.rbm_set_guess(s.ctx, 9) == rbm.RBM_E_INVAL
    # more bodies than the bound workspace holds
    n = s.n + 5
    sid = np.zeros(n, np.int32)
    cen = np.arange(3 * n, dtype=np.float64).reshape(n, 3) * 5
    q = np.tile([1.0, 0, 0, 0], (n, 1))
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    assert lib.rbm_set_bodies(s.ctx, n, P(sid), P(cen), P(q)) == rbm.RBM_E_NOMEM
    # NaN loads are rejected before the device is touched
    bad = np.asarray(w["FT"], dtype=np.float64).copy()
    bad[0, 0] = np.nan
    with pytest.raises(rbm.RbmError) as e:
        s.solve(bad)
    assert e.value.status == rbm.RBM_E_INVAL
    # learned calls before the learned workspace is bound
    loss = ctypes.c_double()
    assert lib.rbm_learned_train(s.ctx, 1, 8, 1e-3, ctypes.byref(loss)) == rbm.RBM_E_STATE
    # the context still solves correctly afterwards
    VW, info = s.solve(w["FT"])
    assert info["rel_residual"] < 1e-12
    s.close()
