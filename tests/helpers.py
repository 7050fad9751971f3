"""Shared test helpers: build oracle problems from seeded workloads."""
import numpy as np

from oracle import geometry as geo
from oracle import system as sy


def shape_coef(shape, p):
    kind, d = shape
    d = np.asarray(d, dtype=np.float64)
    return geo.radial_to_coef(d, p) if kind == "radial" else d


def oracle_shapes(w, with_ops=True, ps=None):
    return [sy.Shape(shape_coef(s, w["p"]), w["p"], ps=ps, eta=w.get("eta", 1.0), with_ops=with_ops)
            for s in w["shapes"]]


def oracle_problem(w, with_ops=True, ps=None, upsample=None):
    shapes = oracle_shapes(w, with_ops, ps)
    q = np.asarray(w["quats"], dtype=np.float64)
    q = q / np.linalg.norm(q, axis=1)[:, None]
    return sy.Problem(shapes, w["shape_id"], w["centres"], q, eta=w.get("eta", 1.0), upsample=upsample)


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
