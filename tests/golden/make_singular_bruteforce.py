"""Writes singular_bruteforce.json: adaptive-quadrature values of the weakly
singular self integrals S[mu](x_t) and (n_t . T)[mu](x_t) on a small perturbed
sphere, for a random band-limited density.  Calls only the oracle's geometry and
spherical-harmonic evaluation plus scipy's adaptive Gauss-Kronrod quadrature; the
singular rule under test is not used.  The integral over the unit sphere is taken in
polar coordinates about the target (theta', phi'), where sin(theta') cancels the
1/r singularity, so the integrand is bounded.

Run:  python tests/golden/make_singular_bruteforce.py
"""
import json
import math
import os
import sys

import numpy as np
from scipy.integrate import quad

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle import geometry as geo  # noqa: E402
from oracle import singular as sg  # noqa: E402
from oracle import sphharm as sh  # noqa: E402

CASE = {"p": 4, "seed": 3, "radial_sigma": 0.08, "targets": [7, 21]}


def main():
    rng = np.random.default_rng(CASE["seed"])
    p = CASE["p"]
    rc = np.zeros(9)
    rc[0] = math.sqrt(4 * math.pi)
    rc[1:] = CASE["radial_sigma"] * rng.standard_normal(8)
    coef = geo.radial_to_coef(rc, p)
    g = sh.grid(p)
    B = sh.band_indices(p)
    cb = rng.standard_normal((3, len(B)))
    xg, ng, _ = geo.surface_frame(coef, g["theta_a"], g["phi_a"])
    out = {"case": CASE, "radial_coef": rc.tolist(), "band_coef": cb.tolist(), "values": {}}
    for t in CASE["targets"]:
        xt, nt = xg[:, t], ng[:, t]
        Q = sg.rot_z(g["phi_a"][t]) @ sg.rot_y(g["theta_a"][t])

        def integrand(tp, fp, kind, c):
            st = math.sin(tp)
            s = Q @ np.array([st * math.cos(fp), st * math.sin(fp), math.cos(tp)])
            th = math.acos(max(-1.0, min(1.0, s[2])))
            ph = math.atan2(s[1], s[0])
            x, _, J = geo.surface_frame(coef, np.array([th]), np.array([ph]))
            Yb = sh.synthesis_matrix(p, np.array([th]), np.array([ph]))[:, 0]
            mu = cb @ Yb
            r = (xt - x[:, 0])[:, None]
            if kind == "S":
                k = sg.kernel_stokeslet(r, 1.0)[:, :, 0]
            else:
                k = sg.kernel_traction(r, nt)[:, :, 0]
            return (k @ mu)[c] * J[0] * st

        vals = {}
        for kind in "SK":
            vals[kind] = [
                quad(lambda fp: quad(lambda tp: integrand(tp, fp, kind, c), 0, math.pi,
                                     epsabs=1e-13, epsrel=1e-13, limit=200)[0],
                     0, 2 * math.pi, epsabs=1e-13, epsrel=1e-13, limit=200)[0]
                for c in range(3)]
        out["values"][str(t)] = vals
        print(t, vals, flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "singular_bruteforce.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
