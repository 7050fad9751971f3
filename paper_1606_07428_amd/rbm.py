"""Thin ctypes binding of librbm.so (C ABI in include/rbm.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides the device workspace and the stream.  ``load()`` raises if the
library has not been built; nothing here falls back to a CPU path.
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbm.so")

RBM_OK, RBM_E_INVAL, RBM_E_NOMEM, RBM_E_DEVICE, RBM_E_NOCONV, RBM_E_OVERLAP, RBM_E_STATE = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED_FP32, MIXED_BF16 = 0, 1, 2
GUESS_ZERO, GUESS_BLOCKDIAG, GUESS_USER, GUESS_LEARNED = 0, 1, 2, 3

EXPORTED = [
    "rbm_default_options", "rbm_create", "rbm_destroy", "rbm_set_shapes", "rbm_set_shapes_radial",
    "rbm_set_bodies", "rbm_workspace_size", "rbm_bind_workspace", "rbm_setup", "rbm_solve",
    "rbm_solve_dev", "rbm_set_guess_dev", "rbm_get_density", "rbm_debug_ptr", "rbm_debug_read",
    "rbm_far_traction", "rbm_far_stokeslet", "rbm_last_error", "rbm_step_rk4", "rbm_get_bodies",
    "rbm_learned_default_config", "rbm_learned_workspace_size", "rbm_learned_bind",
    "rbm_learned_capture", "rbm_learned_set_capture", "rbm_learned_train", "rbm_learned_info",
    "rbm_learned_get_params", "rbm_learned_set_params", "rbm_learned_forward_dev",
    "rbm_learned_loss_grad_dev", "rbm_learned_features_dev", "rbm_learned_guess_dev", "rbm_set_guess",
    "rbm_apply_dev", "rbm_find_contacts", "rbm_solve_contacts", "rbm_magnetic_traction_dev",
    "rbm_solve_density_dev", "rbm_step_rk4_magnetic", "rbm_far_traction_fmm", "rbm_mobility_matrix",
    "rbm_get_state", "rbm_set_state", "rbm_far_traction_static",
]


class Options(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("p_sing", ctypes.c_int), ("eta", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("max_restart", ctypes.c_int),
                ("precision", ctypes.c_int), ("guess", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("stream", ctypes.c_void_p), ("p_up", ctypes.c_int), ("near_factor", ctypes.c_double),
                ("contact_delta", ctypes.c_double), ("magnetic", ctypes.c_int),
                ("fmm_order", ctypes.c_int), ("fmm_max_level", ctypes.c_int),
                ("gmres_lookahead", ctypes.c_int), ("ir_stall", ctypes.c_double),
                ("velocity_fusion", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("matvecs", ctypes.c_int), ("refinements", ctypes.c_int),
                ("cycles", ctypes.c_int), ("rel_residual", ctypes.c_double), ("bnorm", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("ms_far", ctypes.c_double), ("ms_self", ctypes.c_double),
                ("far_pairs", ctypes.c_double), ("n_traction", ctypes.c_int),
                ("n_stokeslet", ctypes.c_int), ("ms_traction", ctypes.c_double),
                ("ms_stokeslet", ctypes.c_double), ("pairs_per_launch", ctypes.c_double),
                ("guess_used", ctypes.c_int), ("fallback_used", ctypes.c_int),
                ("init_rel_residual", ctypes.c_double), ("near_pairs", ctypes.c_int),
                ("ms_near", ctypes.c_double), ("fmm_level", ctypes.c_int),
                ("fmm_applies", ctypes.c_int), ("n_traction32", ctypes.c_int),
                ("ms_traction32", ctypes.c_double), ("fp64_cycles", ctypes.c_int),
                ("n_fused", ctypes.c_int), ("fused_used", ctypes.c_int), ("ms_fused", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LearnedConfig(ctypes.Structure):
    _fields_ = [("k_nbr", ctypes.c_int), ("hidden", ctypes.c_int), ("n_hidden", ctypes.c_int),
                ("capacity", ctypes.c_int), ("batch_max", ctypes.c_int), ("seed", ctypes.c_ulonglong)]


_LIB = None


def load():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    sig = {
        "rbm_default_options": (None, [P]),
        "rbm_create": (I, [P, P]),
        "rbm_destroy": (None, [P]),
        "rbm_set_shapes": (I, [P, I, I, P]),
        "rbm_set_shapes_radial": (I, [P, I, I, P]),
        "rbm_set_bodies": (I, [P, I, P, P, P]),
        "rbm_workspace_size": (I, [P, I, P]),
        "rbm_bind_workspace": (I, [P, P, S]),
        "rbm_setup": (I, [P]),
        "rbm_solve": (I, [P, P, P, P]),
        "rbm_solve_dev": (I, [P, P, P, P]),
        "rbm_set_guess_dev": (I, [P, P]),
        "rbm_get_density": (I, [P, P, P]),
        "rbm_debug_ptr": (P, [P, ctypes.c_char_p]),
        "rbm_debug_read": (I, [P, ctypes.c_char_p, S, S, P]),
        "rbm_far_traction": (I, [P, I, I, P, P, P, P, P, I]),
        "rbm_far_stokeslet": (I, [P, I, I, P, P, P, I]),
        "rbm_last_error": (ctypes.c_char_p, []),
        "rbm_step_rk4": (I, [P, D, P, P]),
        "rbm_get_bodies": (I, [P, P, P]),
        "rbm_learned_default_config": (None, [P]),
        "rbm_learned_workspace_size": (I, [P, P, P]),
        "rbm_learned_bind": (I, [P, P, P, S]),
        "rbm_learned_capture": (I, [P, P]),
        "rbm_learned_set_capture": (I, [P, I]),
        "rbm_learned_train": (I, [P, I, I, D, P]),
        "rbm_learned_info": (I, [P, P, P, P, P]),
        "rbm_learned_get_params": (I, [P, P, S]),
        "rbm_learned_set_params": (I, [P, P, S]),
        "rbm_learned_forward_dev": (I, [P, P, I, P]),
        "rbm_learned_loss_grad_dev": (I, [P, P, P, I, P, P]),
        "rbm_learned_features_dev": (I, [P, P, P]),
        "rbm_learned_guess_dev": (I, [P, P, P]),
        "rbm_set_guess": (I, [P, I]),
        "rbm_apply_dev": (I, [P, P, P]),
        "rbm_find_contacts": (I, [P, D, I, P, P, P]),
        "rbm_solve_contacts": (I, [P, P, I, P, P, P, P, P]),
        "rbm_magnetic_traction_dev": (I, [P, P, D, D, D, P, P, P]),
        "rbm_solve_density_dev": (I, [P, P, P, P]),
        "rbm_step_rk4_magnetic": (I, [P, D, P, D, D, D, P]),
        "rbm_far_traction_fmm": (I, [P, I, I, P, P, P, D, P, I, P]),
        "rbm_mobility_matrix": (I, [P, P, P]),
        "rbm_get_state": (I, [P, P, P]),
        "rbm_set_state": (I, [P, P, S]),
        "rbm_far_traction_static": (I, [I, I, P, P, P, P, P, I, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


class RbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"rbm status {status}: {msg}")
        self.status = status


def _check(status, allow=()):
    if status != RBM_OK and status not in allow:
        raise RbmError(status, load().rbm_last_error().decode())
    return status


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Solver:
    """One library context: shapes, bodies, a PyTorch-owned workspace and a stream."""

    def __init__(self, p, shapes, shape_id, centres, quats, eta=1.0, p_sing=0, tol=1e-12,
                 max_iter=100, max_restart=4, precision=FP64, guess=GUESS_BLOCKDIAG,
                 inner_tol=1e-4, n_max=None, stream=None, device="cuda", p_up=0, near_factor=5.0,
                 contact_delta=0.0, magnetic=0, fmm_order=0, fmm_max_level=5,
                 gmres_lookahead=1, ir_stall=0.5, velocity_fusion=1):
        import torch
        lib = load()
        self.torch = torch
        self.device = torch.device(device)
        opt = Options()
        lib.rbm_default_options(ctypes.byref(opt))
        opt.p, opt.p_sing, opt.eta, opt.tol = p, p_sing, eta, tol
        opt.max_iter, opt.max_restart, opt.precision, opt.guess = max_iter, max_restart, precision, guess
        opt.inner_tol = inner_tol
        opt.p_up, opt.near_factor, opt.contact_delta = p_up, near_factor, contact_delta
        opt.magnetic = magnetic
        opt.fmm_order, opt.fmm_max_level = fmm_order, fmm_max_level
        opt.gmres_lookahead = gmres_lookahead
        opt.ir_stall = ir_stall
        opt.velocity_fusion = velocity_fusion
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        opt.stream = ctypes.c_void_p(self.stream.cuda_stream)
        self.opt = opt
        ctx = ctypes.c_void_p()
        _check(lib.rbm_create(ctypes.byref(opt), ctypes.byref(ctx)))
        self.ctx = ctx
        self.p = p
        self.M = 2 * p * (p + 1)
        self.set_shapes(shapes)
        self.set_bodies(shape_id, centres, quats)
        n_max = self.n if n_max is None else n_max
        nbytes = ctypes.c_size_t()
        _check(lib.rbm_workspace_size(self.ctx, int(n_max), ctypes.byref(nbytes)))
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        _check(lib.rbm_bind_workspace(self.ctx, ctypes.c_void_p(self.ws.data_ptr()), nbytes.value))
        self.workspace_bytes = nbytes.value
        _check(lib.rbm_setup(self.ctx))

    # -- inputs -------------------------------------------------------------------
    def set_shapes(self, shapes):
        lib = load()
        kinds = {k for k, _ in shapes}
        if len(kinds) != 1:
            raise ValueError("all shapes must use one encoding")
        kind = kinds.pop()
        if kind == "radial":
            L = max(int(round(math.sqrt(len(d)))) - 1 for _, d in shapes)
            arr = np.zeros((len(shapes), (L + 1) ** 2))
            for i, (_, d) in enumerate(shapes):
                arr[i, :len(d)] = d
            _check(lib.rbm_set_shapes_radial(self.ctx, len(shapes), L, _ptr(arr)))
        else:
            L = max(int(round(math.sqrt(np.asarray(d).shape[1]))) - 1 for _, d in shapes)
            arr = np.zeros((len(shapes), 3, (L + 1) ** 2))
            for i, (_, d) in enumerate(shapes):
                d = np.asarray(d)
                arr[i, :, :d.shape[1]] = d
            _check(lib.rbm_set_shapes(self.ctx, len(shapes), L, _ptr(arr)))
        self._shape_arr = arr
        self.n_shapes = len(shapes)

    def set_bodies(self, shape_id, centres, quats):
        lib = load()
        sid = np.ascontiguousarray(shape_id, dtype=np.int32)
        cen = _f64(centres, (-1, 3))
        q = _f64(quats, (-1, 4))
        _check(lib.rbm_set_bodies(self.ctx, len(sid), _ptr(sid), _ptr(cen), _ptr(q)))
        self.n = len(sid)
        self.N = self.n * self.M

    # -- solves -------------------------------------------------------------------
    def solve(self, FT):
        lib = load()
        FT = _f64(FT, (self.n, 6))
        VW = np.zeros((self.n, 6))
        info = SolveInfo()
        st = _check(lib.rbm_solve(self.ctx, _ptr(FT), _ptr(VW), ctypes.byref(info)), allow=(RBM_E_NOCONV,))
        self.last_status = st
        return VW, info.as_dict()

    def solve_dev(self, FT_dev, VW_dev):
        """FT_dev, VW_dev: float64 (n, 6) CUDA tensors."""
        lib = load()
        info = SolveInfo()
        st = _check(lib.rbm_solve_dev(self.ctx, ctypes.c_void_p(FT_dev.data_ptr()),
                                      ctypes.c_void_p(VW_dev.data_ptr()), ctypes.byref(info)),
                    allow=(RBM_E_NOCONV,))
        self.last_status = st
        return info.as_dict()

    def mobility_matrix(self):
        """(6n, 6n) mobility matrix at the current poses and the summed solve info."""
        m = 6 * self.n
        Mm = np.zeros((m, m))
        info = SolveInfo()
        st = _check(load().rbm_mobility_matrix(self.ctx, _ptr(Mm), ctypes.byref(info)), allow=(RBM_E_NOCONV,))
        self.last_status = st
        return Mm, info.as_dict()

    def get_state(self):
        """The run state as a bytes object."""
        nb = ctypes.c_size_t()
        _check(load().rbm_get_state(self.ctx, None, ctypes.byref(nb)))
        buf = ctypes.create_string_buffer(nb.value)
        _check(load().rbm_get_state(self.ctx, buf, ctypes.byref(nb)))
        return buf.raw[:nb.value]

    def set_state(self, state):
        buf = ctypes.create_string_buffer(bytes(state), len(state))
        _check(load().rbm_set_state(self.ctx, buf, len(state)))

    def apply_dev(self, mu_dev):
        """y = A mu at the current poses; mu_dev: float64 (3, N) CUDA tensor."""
        y = self.torch.empty_like(mu_dev)
        _check(load().rbm_apply_dev(self.ctx, ctypes.c_void_p(mu_dev.data_ptr()),
                                    ctypes.c_void_p(y.data_ptr())))
        return y

    def magnetic_traction(self, H0, mu_ratio, mu0=1.0, tol=1e-12):
        """Maxwell traction (3, N) CUDA tensor, net loads (n, 6) CUDA tensor, GMRES iterations."""
        rho = self.torch.empty((3, self.N), dtype=self.torch.float64, device=self.device)
        FT = self.torch.empty((self.n, 6), dtype=self.torch.float64, device=self.device)
        h = _f64(H0, (3,))
        it = ctypes.c_int()
        _check(load().rbm_magnetic_traction_dev(self.ctx, _ptr(h), float(mu_ratio), float(mu0), float(tol),
                                                ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(FT.data_ptr()),
                                                ctypes.byref(it)))
        return rho, FT, it.value

    def solve_density_dev(self, rho_dev, VW_dev):
        """Mobility solve with incident density rho_dev (3, N) CUDA tensor into VW_dev (n, 6)."""
        info = SolveInfo()
        st = _check(load().rbm_solve_density_dev(self.ctx, ctypes.c_void_p(rho_dev.data_ptr()),
                                                 ctypes.c_void_p(VW_dev.data_ptr()), ctypes.byref(info)),
                    allow=(RBM_E_NOCONV,))
        self.last_status = st
        return info.as_dict()

    def find_contacts(self, delta, max_contacts=4096):
        """Body pairs whose closest nodes are within delta: (pairs (k, 2), points (k, 3))."""
        pairs = np.zeros((max_contacts, 2), dtype=np.int32)
        pts = np.zeros((max_contacts, 3))
        nf = ctypes.c_int()
        _check(load().rbm_find_contacts(self.ctx, float(delta), max_contacts, ctypes.byref(nf),
                                        _ptr(pairs), _ptr(pts)))
        k = min(nf.value, max_contacts)
        return pairs[:k].copy(), pts[:k].copy()

    def solve_contacts(self, FT, pairs, points):
        """Velocities with contact forces: (VW (n, 6), Fc (k, 3), info)."""
        FT = _f64(FT, (self.n, 6))
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        points = _f64(points, (-1, 3))
        VW = np.zeros((self.n, 6))
        Fc = np.zeros((max(len(pairs), 1), 3))
        info = SolveInfo()
        _check(load().rbm_solve_contacts(self.ctx, _ptr(FT), len(pairs), _ptr(pairs), _ptr(points),
                                         _ptr(VW), _ptr(Fc), ctypes.byref(info)))
        return VW, Fc[:len(pairs)], info.as_dict()

    def step_rk4(self, dt, FT_dev):
        """One RK4 step with loads FT_dev (float64 (n, 6) CUDA tensor); returns the
        four stage infos."""
        infos = (SolveInfo * 4)()
        st = _check(load().rbm_step_rk4(self.ctx, float(dt), ctypes.c_void_p(FT_dev.data_ptr()), infos),
                    allow=(RBM_E_NOCONV,))
        self.last_status = st
        return [i.as_dict() for i in infos]

    def step_rk4_magnetic(self, dt, H0, mu_ratio, mu0=1.0, tol_mag=1e-12):
        """One RK4 step driven by the Maxwell traction of the field H0 (§4); returns the
        four stage infos."""
        infos = (SolveInfo * 4)()
        h = _f64(H0, (3,))
        st = _check(load().rbm_step_rk4_magnetic(self.ctx, float(dt), _ptr(h), float(mu_ratio), float(mu0),
                                                 float(tol_mag), infos),
                    allow=(RBM_E_NOCONV,))
        self.last_status = st
        return [i.as_dict() for i in infos]

    def bodies(self):
        cen = np.zeros((self.n, 3))
        q = np.zeros((self.n, 4))
        _check(load().rbm_get_bodies(self.ctx, _ptr(cen), _ptr(q)))
        return cen, q

    # -- learned warm start -----------------------------------------------------------
    def learned_bind(self, k_nbr=8, hidden=256, n_hidden=3, capacity=65536, batch_max=1024, seed=1234):
        lib = load()
        cfg = LearnedConfig()
        lib.rbm_learned_default_config(ctypes.byref(cfg))
        cfg.k_nbr, cfg.hidden, cfg.n_hidden = k_nbr, hidden, n_hidden
        cfg.capacity, cfg.batch_max, cfg.seed = capacity, batch_max, seed
        nb = ctypes.c_size_t()
        _check(lib.rbm_learned_workspace_size(self.ctx, ctypes.byref(cfg), ctypes.byref(nb)))
        self.learned_ws = self.torch.empty(nb.value, dtype=self.torch.uint8, device=self.device)
        _check(lib.rbm_learned_bind(self.ctx, ctypes.byref(cfg), ctypes.c_void_p(self.learned_ws.data_ptr()),
                                    nb.value))
        self.learned_cfg = cfg
        return self.learned_info()

    def learned_info(self):
        a, b, c, d = (ctypes.c_int() for _ in range(4))
        _check(load().rbm_learned_info(self.ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                       ctypes.byref(d)))
        return {"samples": a.value, "F": b.value, "O": c.value, "n_params": d.value}

    def learned_capture(self, FT_dev):
        _check(load().rbm_learned_capture(self.ctx, ctypes.c_void_p(FT_dev.data_ptr())))

    def learned_set_capture(self, on):
        _check(load().rbm_learned_set_capture(self.ctx, int(bool(on))))

    def learned_train(self, epochs, batch, lr):
        loss = ctypes.c_double()
        _check(load().rbm_learned_train(self.ctx, int(epochs), int(batch), float(lr), ctypes.byref(loss)))
        return loss.value

    def learned_params(self):
        info = self.learned_info()
        out = np.zeros(info["n_params"] + 2 * info["F"] + 2, dtype=np.float32)
        _check(load().rbm_learned_get_params(self.ctx, _ptr(out), out.size))
        return out

    def learned_set_params(self, arr):
        arr = np.ascontiguousarray(arr, dtype=np.float32)
        _check(load().rbm_learned_set_params(self.ctx, _ptr(arr), arr.size))

    def learned_forward(self, X_dev, Y_dev):
        _check(load().rbm_learned_forward_dev(self.ctx, ctypes.c_void_p(X_dev.data_ptr()), X_dev.shape[0],
                                              ctypes.c_void_p(Y_dev.data_ptr())))

    def learned_loss_grad(self, X_dev, T_dev, G_dev):
        loss = ctypes.c_double()
        _check(load().rbm_learned_loss_grad_dev(self.ctx, ctypes.c_void_p(X_dev.data_ptr()),
                                                ctypes.c_void_p(T_dev.data_ptr()), X_dev.shape[0],
                                                ctypes.c_void_p(G_dev.data_ptr()), ctypes.byref(loss)))
        return loss.value

    def learned_features(self, FT_dev, X_dev):
        _check(load().rbm_learned_features_dev(self.ctx, ctypes.c_void_p(FT_dev.data_ptr()),
                                               ctypes.c_void_p(X_dev.data_ptr())))

    def learned_guess(self, FT_dev, mu_dev):
        _check(load().rbm_learned_guess_dev(self.ctx, ctypes.c_void_p(FT_dev.data_ptr()),
                                            ctypes.c_void_p(mu_dev.data_ptr())))

    def set_guess_mode(self, guess):
        _check(load().rbm_set_guess(self.ctx, int(guess)))
        self.opt.guess = guess

    def set_guess_dev(self, mu0_dev):
        _check(load().rbm_set_guess_dev(self.ctx, ctypes.c_void_p(mu0_dev.data_ptr())))

    def density(self):
        mu = np.zeros((3, self.N))
        rho = np.zeros((3, self.N))
        _check(load().rbm_get_density(self.ctx, _ptr(mu), _ptr(rho)))
        return mu, rho

    def read(self, name, count, dtype=np.float64, offset=0):
        out = np.zeros(count, dtype=dtype)
        _check(load().rbm_debug_read(self.ctx, name.encode(), offset, out.nbytes, _ptr(out)))
        return out

    # -- low-level sums -------------------------------------------------------------
    def far_traction(self, X, Nrm, q, M, add=None, precision=0):
        """X, Nrm, q, add: float64 (3, n) CUDA tensors; returns (3, n) tensor."""
        torch = self.torch
        n = X.shape[1]
        y = torch.empty_like(X)
        a = ctypes.c_void_p(add.data_ptr()) if add is not None else None
        _check(load().rbm_far_traction(self.ctx, n, M, ctypes.c_void_p(X.data_ptr()),
                                       ctypes.c_void_p(Nrm.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                                       a, ctypes.c_void_p(y.data_ptr()), precision))
        return y

    def far_traction_fmm(self, X, Nrm, q, M, d_max, precision=0):
        """Fast multipole approximation of far_traction (add = None): ((3, n) tensor, leaf level)."""
        n = X.shape[1]
        y = self.torch.empty_like(X)
        lev = ctypes.c_int()
        _check(load().rbm_far_traction_fmm(self.ctx, n, M, ctypes.c_void_p(X.data_ptr()),
                                           ctypes.c_void_p(Nrm.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                                           float(d_max), ctypes.c_void_p(y.data_ptr()), precision,
                                           ctypes.byref(lev)))
        return y, lev.value

    def far_stokeslet(self, X, q, M, precision=0):
        torch = self.torch
        n = X.shape[1]
        u = torch.empty_like(X)
        _check(load().rbm_far_stokeslet(self.ctx, n, M, ctypes.c_void_p(X.data_ptr()),
                                        ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                        precision))
        return u

    def close(self):
        if getattr(self, "ctx", None):
            load().rbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def far_traction_static(X, Nrm, q, M, add=None, precision=0, stream=None):
    """rbm_far_traction_static on float64 (3, n) CUDA tensors (no context, no allocation by the
    library); returns y (3, n), allocated here by PyTorch, on `stream` (default: current)."""
    import torch
    n = X.shape[1]
    y = torch.empty_like(X)
    st = stream if stream is not None else torch.cuda.current_stream(X.device)
    a = ctypes.c_void_p(add.data_ptr()) if add is not None else None
    _check(load().rbm_far_traction_static(n, M, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Nrm.data_ptr()),
                                          ctypes.c_void_p(q.data_ptr()), a, ctypes.c_void_p(y.data_ptr()),
                                          precision, ctypes.c_void_p(st.cuda_stream)))
    return y


def solver_for(workload, **kw):
    """Build a Solver from a ``paper_1606_07428_amd.inputs`` workload dict."""
    return Solver(workload["p"], workload["shapes"], workload["shape_id"], workload["centres"],
                  workload["quats"], eta=workload.get("eta", 1.0), **kw)
