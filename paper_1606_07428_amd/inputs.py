"""Seeded synthetic workloads for the rigid-body mobility solve.

This module holds no arithmetic of the method: it only draws shapes, poses and
loads, and is the one module that both the HIP path and the FP64 oracle are fed
from.  Shapes are encoded in the library's input format (real orthonormal SH
without the Condon-Shortley phase, index l*l + l + m):

  * ``("radial", rc)``: r(s) = sum rc_lm Y_lm(s), body x = r(s) s;
  * ``("coef", a)``: coordinate-function coefficients a[3, (L+1)^2].

A unit sphere is ("radial", [sqrt(4 pi)]) since Y_00 = 1/sqrt(4 pi).  An ellipsoid
with semi-axes (a, b, c) is ("coef", ...) with a*sqrt(4pi/3) on (x, Y_11),
b*sqrt(4pi/3) on (y, Y_1-1) and c*sqrt(4pi/3) on (z, Y_10).

Placement is random sequential addition in a cube whose side L gives the stated
volume fraction phi with the nominal body volume; a conservative bounding radius
(from |Y_lm| <= sqrt((2l+1)/(4pi))) enforces the minimum gap.  Orientations are
uniform on SO(3) (normalised 4-D Gaussians, quaternion (w, x, y, z), body -> lab).
"""
import math

import numpy as np

BASE_SEED = 160607428


def _radial_perturbed(rng, lmax=4, amp=0.1):
    """Radius 1 plus an SH perturbation, coefficients N(0, (amp/(1+l)^2)^2), l<=lmax."""
    rc = np.zeros((lmax + 1) ** 2)
    for l in range(lmax + 1):
        sig = amp / (1.0 + l) ** 2
        for m in range(-l, l + 1):
            rc[l * l + l + m] = sig * rng.standard_normal()
    rc[0] += math.sqrt(4.0 * math.pi)
    return rc


def bounding_radius(kind, data):
    """Upper bound of the distance from the area centroid to the surface."""
    if kind == "radial":
        rc = np.asarray(data)
        base = abs(rc[0]) / math.sqrt(4 * math.pi)
        dev = 0.0
        lmax = int(round(math.sqrt(len(rc)))) - 1
        for l in range(1, lmax + 1):
            amp = math.sqrt((2 * l + 1) / (4 * math.pi))
            dev += amp * np.abs(rc[l * l:(l + 1) ** 2]).sum()
        return base + 2.0 * dev
    a = np.asarray(data)
    lmax = int(round(math.sqrt(a.shape[1]))) - 1
    tot = 0.0
    for l in range(lmax + 1):
        amp = math.sqrt((2 * l + 1) / (4 * math.pi))
        tot += amp * np.linalg.norm(a[:, l * l:(l + 1) ** 2], axis=0).sum()
    return 2.0 * tot


def _uniform_quats(rng, n):
    q = rng.standard_normal((n, 4))
    return q / np.linalg.norm(q, axis=1)[:, None]


def _rsa(rng, rb, side, gap, max_tries=20_000_000):
    """Random sequential addition: draw uniform centres in the cube, keep one if its
    bounding sphere clears every placed one by `gap`.  A cell list (cell size >= the
    largest exclusion distance) limits each test to the 27 neighbouring cells."""
    n = len(rb)
    pos = np.zeros((n, 3))
    placed = 0
    tries = 0
    order = np.argsort(-rb)
    cell = 2.0 * float(rb.max()) + gap
    nc = max(1, int(side // cell))
    h = side / nc
    cells = {}
    while placed < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not converge")
        i = order[placed]
        c = rng.uniform(0.0, side, 3)
        key = tuple(np.minimum((c // h).astype(int), nc - 1))
        near = []
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    near.extend(cells.get((key[0] + dx, key[1] + dy, key[2] + dz), ()))
        if near:
            near = np.asarray(near)
            d = np.linalg.norm(pos[near] - c, axis=1)
            if np.any(d < rb[near] + rb[i] + gap):
                continue
        pos[i] = c
        cells.setdefault(key, []).append(i)
        placed += 1
    return pos


def workload(name, seed=None):
    """Return a dict describing one synthetic configuration.

    Names: 'two_spheres' (2 unit spheres at (0,0,0), (3,0,0), p = 8),
    'single_sphere', 'random64' (64 SH-perturbed bodies, p = 12),
    'ellipsoids1000' (1000 ellipsoids (1, .8, .6), p = 16), 'sediment512'
    (512 perturbed spheres, F = (0,0,-1)), 'dense4000' (4000 perturbed spheres at
    volume fraction 20 %, gap 0.1), 'dense4000_train' (the same generator, another seed)
    and 'dense512' (a smaller, separately seeded sibling); ``tiny``, ``lattice`` and
    ``workload_perturbed`` build other configurations.
    """
    cfg_index = {"two_spheres": 0, "single_sphere": 0, "random64": 1, "ellipsoids1000": 2,
                 "sediment512": 3, "dense4000": 4, "dense512": 5, "dense4000_train": 6}
    if seed is None:
        seed = BASE_SEED + cfg_index.get(name, 99)
    rng = np.random.default_rng(seed)
    unit = ("radial", np.array([math.sqrt(4 * math.pi)]))
    if name == "two_spheres":
        return dict(name=name, p=8, eta=1.0, shapes=[unit], shape_id=np.zeros(2, np.int32),
                    centres=np.array([[0.0, 0, 0], [3.0, 0, 0]]),
                    quats=np.array([[1.0, 0, 0, 0]] * 2),
                    FT=np.array([[1.0, 0, 0, 0, 0, 1], [0.0, 0, 0, 0, 0, 0]]))
    if name == "single_sphere":
        return dict(name=name, p=8, eta=1.0, shapes=[unit], shape_id=np.zeros(1, np.int32),
                    centres=np.zeros((1, 3)), quats=np.array([[1.0, 0, 0, 0]]),
                    FT=np.array([[1.0, 0, 0, 0, 0, 1]]))
    if name == "random64":
        return workload_perturbed(64, 12, 0.10, 0.5, rng, name)
    if name == "sediment512":
        w = workload_perturbed(512, 12, 0.10, 0.5, rng, name)
        w["FT"][:, :3] = [0.0, 0.0, -1.0]
        w["FT"][:, 3:] = math.sqrt(0.1) * rng.standard_normal((512, 3))
        return w
    if name == "dense4000":
        return workload_perturbed(4000, 12, 0.20, 0.1, rng, name)
    if name == "dense4000_train":
        # the dense configuration's generator with another seed: time-stepped to train the
        # warm start that is then evaluated on dense4000
        return workload_perturbed(4000, 12, 0.20, 0.1, rng, name)
    if name == "dense512":
        # a smaller, separately seeded suspension with the dense configuration's statistics
        # (20 %, gap 0.1), used to train the warm start that is then applied to dense4000
        return workload_perturbed(512, 12, 0.20, 0.1, rng, name)
    if name == "ellipsoids1000":
        n = 1000
        k = math.sqrt(4 * math.pi / 3)
        a = np.zeros((3, 4))
        a[0, 3], a[1, 1], a[2, 2] = 1.0 * k, 0.8 * k, 0.6 * k
        vol = 4 * math.pi / 3 * 0.48
        side = (n * vol / 0.10) ** (1 / 3)
        pos = _rsa(rng, np.ones(n), side, 0.1)
        return dict(name=name, p=16, eta=1.0, shapes=[("coef", a)], shape_id=np.zeros(n, np.int32),
                    centres=pos, quats=_uniform_quats(rng, n), FT=rng.standard_normal((n, 6)))
    raise KeyError(name)


def lattice(n, p):
    """The paper's scaling workload (§4): a 2 x 2 x n/4 lattice of unit spheres with centre
    spacing 5, identity orientations, sedimenting under F = (0, 0, -1), T = 0."""
    if n % 4:
        raise ValueError("n must be a multiple of 4")
    nz = n // 4
    cen = np.array([[5.0 * i, 5.0 * j, 5.0 * k] for k in range(nz) for j in range(2) for i in range(2)])
    FT = np.zeros((n, 6))
    FT[:, 2] = -1.0
    return dict(name=f"lattice{n}_p{p}", p=p, eta=1.0, shapes=[("radial", np.array([math.sqrt(4 * math.pi)]))],
                shape_id=np.zeros(n, np.int32), centres=cen, quats=np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)), FT=FT)


def mhd_lattice(side=8, p=8, spacing=3.0, jitter=0.0, seed=0):
    """The magnetorheological workload of §4 (Fig. 1): side^3 unit spheres on a cubic lattice
    (centre spacing `spacing`, optionally jittered uniformly by +-jitter per coordinate),
    identity orientations, no external loads; the field is applied separately."""
    rng = np.random.default_rng(160607428 + 50 + seed)
    g = np.arange(side) * spacing
    cen = np.array([[x, y, z] for z in g for y in g for x in g])
    if jitter > 0:
        cen = cen + rng.uniform(-jitter, jitter, cen.shape)
    n = len(cen)
    return dict(name=f"mhd{n}_p{p}", p=p, eta=1.0, shapes=[("radial", np.array([math.sqrt(4 * math.pi)]))],
                shape_id=np.zeros(n, np.int32), centres=cen, quats=np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)),
                FT=np.zeros((n, 6)))


def workload_perturbed(n, p, phi, gap, rng, name="perturbed", lmax=4, amp=0.1):
    """n distinct SH-perturbed spheres (one shape each), volume fraction phi."""
    shapes = [("radial", _radial_perturbed(rng, lmax, amp)) for _ in range(n)]
    rb = np.array([bounding_radius(k, d) for k, d in shapes])
    side = (n * (4 * math.pi / 3) / phi) ** (1 / 3)
    pos = _rsa(rng, rb, side, gap)
    return dict(name=name, p=p, eta=1.0, shapes=shapes, shape_id=np.arange(n, dtype=np.int32),
                centres=pos, quats=_uniform_quats(rng, n), FT=rng.standard_normal((n, 6)))


def tiny(n=3, p=6, seed=7, amp=0.1, lmax=3, shared=False):
    """A few perturbed bodies on a line-ish cluster, for parity tests."""
    rng = np.random.default_rng(seed)
    ns = 1 if shared else n
    shapes = [("radial", _radial_perturbed(rng, lmax, amp)) for _ in range(ns)]
    rb = np.array([bounding_radius(*s) for s in shapes])
    side = max(2.0, (n * 4.19 / 0.08) ** (1 / 3))
    pos = _rsa(rng, rb[np.zeros(n, int) if shared else np.arange(n)], side, 0.4)
    return dict(name="tiny", p=p, eta=1.0, shapes=shapes,
                shape_id=np.zeros(n, np.int32) if shared else np.arange(n, dtype=np.int32),
                centres=pos, quats=_uniform_quats(rng, n), FT=rng.standard_normal((n, 6)))
