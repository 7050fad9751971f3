"""The C-ABI library: it loads, exports every function include/rbm.h declares, and
rejects bad arguments on the host (no GPU needed for these calls)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1606_07428_amd import rbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rbm_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = rbm.load()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(rbm.EXPORTED)


def _opts(**kw):
    o = rbm.Options()
    rbm.load().rbm_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def test_default_options():
    o = _opts()
    assert (o.p, o.eta, o.tol, o.max_iter, o.precision, o.guess) == (8, 1.0, 1e-12, 100, 0, 1)
    assert (o.p_up, o.near_factor, o.contact_delta, o.magnetic, o.fmm_order, o.fmm_max_level,
            o.gmres_lookahead, o.ir_stall, o.velocity_fusion) == (0, 5.0, 0.0, 0, 0, 5, 1, 0.5, 1)


def test_fmm_level_bound_checked_only_with_an_order():
    lib = rbm.load()
    ctx = ctypes.c_void_p()
    o = _opts(fmm_order=8, fmm_max_level=7)
    assert lib.rbm_create(ctypes.byref(o), ctypes.byref(ctx)) == rbm.RBM_E_INVAL
    o = _opts(fmm_order=0, fmm_max_level=7)
    assert lib.rbm_create(ctypes.byref(o), ctypes.byref(ctx)) == rbm.RBM_OK
    lib.rbm_destroy(ctx)


@pytest.mark.parametrize("field,value", [("p", 1), ("p", 21), ("eta", 0.0), ("eta", float("nan")),
                                         ("tol", -1.0), ("max_iter", 0), ("precision", 7),
                                         ("guess", 9), ("p_sing", 3), ("p_up", 3),
                                         ("near_factor", -1.0), ("contact_delta", -0.5),
                                         ("fmm_order", 1), ("fmm_order", 17), ("ir_stall", 1.0),
                                         ("ir_stall", -0.1), ("velocity_fusion", 2),
                                         ("gmres_lookahead", -1), ("gmres_lookahead", 3)])
def test_create_rejects_bad_options(field, value):
    lib = rbm.load()
    o = _opts(**{field: value})
    ctx = ctypes.c_void_p()
    assert lib.rbm_create(ctypes.byref(o), ctypes.byref(ctx)) == rbm.RBM_E_INVAL
    assert lib.rbm_last_error()


def _ctx(p=6):
    lib = rbm.load()
    o = _opts(p=p)
    ctx = ctypes.c_void_p()
    assert lib.rbm_create(ctypes.byref(o), ctypes.byref(ctx)) == rbm.RBM_OK
    return lib, ctx


def test_host_side_validation_of_inputs():
    lib, ctx = _ctx(6)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    rc = np.array([[math.sqrt(4 * math.pi)]])
    # call order: bodies before shapes
    sid = np.zeros(1, np.int32)
    cen = np.zeros((1, 3))
    q = np.array([[1.0, 0, 0, 0]])
    assert lib.rbm_set_bodies(ctx, 1, P(sid), P(cen), P(q)) == rbm.RBM_E_STATE
    # radial degree too high for p, non-finite coefficients
    assert lib.rbm_set_shapes_radial(ctx, 1, 5, P(np.zeros((1, 36)))) == rbm.RBM_E_INVAL
    bad = rc.copy()
    bad[0, 0] = np.nan
    assert lib.rbm_set_shapes_radial(ctx, 1, 0, P(bad)) == rbm.RBM_E_INVAL
    assert lib.rbm_set_shapes_radial(ctx, 1, 0, P(rc)) == rbm.RBM_OK
    # unknown shape id, non-unit quaternion, NaN centre
    assert lib.rbm_set_bodies(ctx, 1, P(np.array([3], np.int32)), P(cen), P(q)) == rbm.RBM_E_INVAL
    assert lib.rbm_set_bodies(ctx, 1, P(sid), P(cen), P(2 * q)) == rbm.RBM_E_INVAL
    cnan = cen.copy()
    cnan[0, 1] = np.inf
    assert lib.rbm_set_bodies(ctx, 1, P(sid), P(cnan), P(q)) == rbm.RBM_E_INVAL
    assert lib.rbm_set_bodies(ctx, 1, P(sid), P(cen), P(q)) == rbm.RBM_OK
    # setup / solve before a workspace is bound
    assert lib.rbm_setup(ctx) == rbm.RBM_E_NOMEM
    FT = np.zeros((1, 6))
    VW = np.zeros((1, 6))
    assert lib.rbm_solve(ctx, P(FT), P(VW), None) == rbm.RBM_E_NOMEM
    nbytes = ctypes.c_size_t()
    assert lib.rbm_workspace_size(ctx, 4, ctypes.byref(nbytes)) == rbm.RBM_OK
    assert nbytes.value > 0
    lib.rbm_destroy(ctx)


def test_workspace_grows_with_bodies_and_order():
    sizes = []
    for p, n in [(6, 4), (6, 40), (8, 40)]:
        lib, ctx = _ctx(p)
        P = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        assert lib.rbm_set_shapes_radial(ctx, 1, 0, P(np.array([[math.sqrt(4 * math.pi)]]))) == 0
        nb = ctypes.c_size_t()
        assert lib.rbm_workspace_size(ctx, n, ctypes.byref(nb)) == 0
        sizes.append(nb.value)
        lib.rbm_destroy(ctx)
    assert sizes[0] < sizes[1] < sizes[2]


def test_binding_structures_match_header():
    # field order and size of the option / info / config structs of include/rbm.h
    src = open(os.path.join(ROOT, "include", "rbm.h")).read()
    for cls, tag in ((rbm.Options, "rbm_options"), (rbm.SolveInfo, "rbm_solve_info"),
                     (rbm.LearnedConfig, "rbm_learned_config")):
        body = src[:src.index("} " + tag + ";")]
        body = body[body.rindex("typedef struct {"):]
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = re.findall(r"(\w+)\s*;", body)
        names = [x for part in re.findall(r"(?:int|double|void\*|unsigned long long)\s+([\w ,]+);", body)
                 for x in re.split(r"\s*,\s*", part.strip())]
        assert [f for f, _ in cls._fields_] == names, (tag, names)
    info = rbm.SolveInfo()
    assert set(info.as_dict()) == {f for f, _ in rbm.SolveInfo._fields_}
