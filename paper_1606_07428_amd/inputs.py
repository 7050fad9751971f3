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

Placement is random sequential addition (RSA) in a cube whose side L gives the
stated volume fraction phi with the nominal body volume 4 pi / 3.  The centre the
library receives is the lab position of a body's area centroid, so placement works
with surfaces relative to that centroid.  Three gap rules:

  * ``"bounding"``: centre distance >= R_i + R_j + gap with R the largest
    centroid-to-surface distance (tight, from a dense point cloud of the surface);
  * ``"surface"``: the true distance between the two surfaces >= gap, taken as the
    smallest distance between dense point clouds of them (about 16,000 points per
    body, spacing ~0.03), tested only for bodies whose bounding spheres come within
    reach and decided early when inscribed spheres are already too close or a
    coarse cloud is already clear by twice its covering radius;
  * ``"loose"``: the bounding radius 1 + 2 sum_l sqrt((2l+1)/4pi) |rc_lm| about the
    radial origin (from |Y_lm| <= sqrt((2l+1)/(4pi))), which over-estimates the body
    radius by about 0.2; kept only for the small parity clusters of ``tiny``.

The surface point clouds and the area centroid used for placement are computed
here only to decide where bodies go (neither side reads them: the library and the
oracle each build their own geometry from the coefficients).  Orientations are
uniform on SO(3) (normalised 4-D Gaussians, quaternion (w, x, y, z), body -> lab).
"""
import copy
import functools
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
    """Loose upper bound of the distance from the radial origin (or the coordinate
    origin) to the surface, from |Y_lm| <= sqrt((2l+1)/(4 pi))."""
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


# ---------------------------------------------------------------------------------
# Surfaces of radial shapes for placement (the shape definition r(s) = sum rc Y,
# evaluated with scipy's associated Legendre functions)

def _real_sh(lmax, ct, phi):
    """Real orthonormal Y_lm at the directions (cos theta, phi), no Condon-Shortley
    phase: ((lmax+1)^2, K).  scipy's lpmv carries the (-1)^m phase, removed here."""
    from scipy.special import lpmv
    out = np.zeros(((lmax + 1) ** 2, len(ct)))
    for l in range(lmax + 1):
        for m in range(l + 1):
            nrm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            P = (-1.0) ** m * lpmv(m, l, ct)
            if m == 0:
                out[l * l + l] = nrm * P
            else:
                out[l * l + l + m] = math.sqrt(2.0) * nrm * P * np.cos(m * phi)
                out[l * l + l - m] = math.sqrt(2.0) * nrm * P * np.sin(m * phi)
    return out


def _fibonacci_dirs(K):
    """K nearly uniform unit directions (golden-angle spiral): (ct, phi, unit (K, 3))."""
    k = np.arange(K) + 0.5
    ct = 1.0 - 2.0 * k / K
    phi = np.mod(math.pi * (3.0 - math.sqrt(5.0)) * k, 2 * math.pi)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    return ct, phi, np.stack([st * np.cos(phi), st * np.sin(phi), ct], axis=1)


class _RadialFamily:
    """Direction sets shared by all radial shapes of one degree."""

    K_COARSE = 1200
    K_FINE = 16000

    def __init__(self, lmax):
        self.lmax = lmax
        ct, phi, self.u_coarse = _fibonacci_dirs(self.K_COARSE)
        self.Y_coarse = _real_sh(lmax, ct, phi)
        ct, phi, self.u_fine = _fibonacci_dirs(self.K_FINE)
        self.Y_fine = _real_sh(lmax, ct, phi)
        # quadrature for the area centroid: Gauss-Legendre in cos(theta) x trapezoid in phi
        # (the integrand r sqrt(r^2 + |grad r|^2) x is smooth; 48 x 96 points resolve it to
        # far below the placement tolerance); d/dtheta by central differences
        t, lam = np.polynomial.legendre.leggauss(48)
        ph = 2 * math.pi * np.arange(96) / 96
        T, Pz = np.meshgrid(np.arccos(t), ph, indexing="ij")
        self.q_w = (np.repeat(lam, 96) * (2 * math.pi / 96))
        th, phq = T.ravel(), Pz.ravel()
        h = 1e-6
        self.q_Y = _real_sh(lmax, np.cos(th), phq)
        self.q_Yt = (_real_sh(lmax, np.cos(th + h), phq) - _real_sh(lmax, np.cos(th - h), phq)) / (2 * h)
        self.q_Yp = (_real_sh(lmax, np.cos(th), phq + h) - _real_sh(lmax, np.cos(th), phq - h)) / (2 * h)
        self.q_sin = np.sin(th)
        self.q_u = np.stack([np.sin(th) * np.cos(phq), np.sin(th) * np.sin(phq), np.cos(th)], axis=1)

    def shape(self, rc):
        """Centroid offset, inscribed / circumscribed radii about the area centroid and
        the coarse cloud (body frame, relative to the centroid) of r = rc . Y."""
        r = rc @ self.q_Y
        rt = rc @ self.q_Yt
        rp = rc @ self.q_Yp
        dS = r * np.sqrt(r * r + rt * rt + (rp / self.q_sin) ** 2) * self.q_w
        xc = (dS[:, None] * r[:, None] * self.q_u).sum(axis=0) / dS.sum()
        rf = rc @ self.Y_fine
        cloud_f = rf[:, None] * self.u_fine - xc
        r_out = float(np.sqrt((cloud_f * cloud_f).sum(axis=1)).max()) + 0.005
        r_in = float(rf.min()) - float(np.linalg.norm(xc)) - 0.01
        cloud_c = (rc @ self.Y_coarse)[:, None] * self.u_coarse - xc
        return xc, r_in, r_out, cloud_c

    def fine_cloud(self, rc, xc):
        return (rc @ self.Y_fine)[:, None] * self.u_fine - xc


@functools.lru_cache(maxsize=4)
def _family(lmax):
    return _RadialFamily(lmax)


def _min_dist(P, Q):
    """Smallest distance between the point sets P (a, 3) and Q (b, 3)."""
    from scipy.spatial import cKDTree
    if len(P) == 0 or len(Q) == 0:
        return math.inf
    d, _ = cKDTree(Q).query(P, k=1)
    return float(d.min())


def _quat_to_rot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _uniform_quats(rng, n):
    q = rng.standard_normal((n, 4))
    return q / np.linalg.norm(q, axis=1)[:, None]


def _rsa(rng, rb, side, gap, max_tries=20_000_000):
    """Random sequential addition with bounding spheres: draw uniform centres in the
    cube, keep one if its bounding sphere clears every placed one by `gap`.  A cell list
    (cell size >= the largest exclusion distance) limits each test to the 27
    neighbouring cells."""
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


def _rsa_surface(rng, shapes, side, gap, max_tries=20_000_000):
    """Random sequential addition with a true surface gap for radial shapes: each trial
    draws a centre (uniform in the cube) and an orientation (uniform on SO(3)) and is
    kept when its surface clears every placed body's surface by `gap`.  Returns centres
    (of the area centroids) and quaternions."""
    n = len(shapes)
    lmax = max(int(round(math.sqrt(len(d)))) - 1 for _, d in shapes)
    fam = _family(lmax)
    rcs = []
    for _, d in shapes:
        rc = np.zeros((lmax + 1) ** 2)
        rc[:len(d)] = d
        rcs.append(rc)
    geo = [fam.shape(rc) for rc in rcs]
    xc = np.array([g[0] for g in geo])
    r_in = np.array([g[1] for g in geo])
    r_out = np.array([g[2] for g in geo])
    # covering radius of the coarse cloud on the surface (generous): a coarse distance
    # d_c bounds the true one within [d_c - 2 rho, d_c]
    rho = 1.2 * math.sqrt(4 * math.pi / fam.K_COARSE) * float(r_out.max())
    pos = np.zeros((n, 3))
    quat = np.zeros((n, 4))
    rot = np.zeros((n, 3, 3))
    cell = 2.0 * float(r_out.max()) + gap
    nc = max(1, int(side // cell))
    h = side / nc
    cells = {}
    placed = 0
    tries = 0
    order = np.argsort(-r_out)
    fine = {}

    def fine_lab(k, c, R):
        if k not in fine:
            fine[k] = fam.fine_cloud(rcs[k], xc[k])
        return c + fine[k] @ R.T

    while placed < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random sequential addition did not converge")
        i = order[placed]
        c = rng.uniform(0.0, side, 3)
        q = rng.standard_normal(4)
        q /= np.linalg.norm(q)
        key = tuple(np.minimum((c // h).astype(int), nc - 1))
        near = []
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    near.extend(cells.get((key[0] + dx, key[1] + dy, key[2] + dz), ()))
        ok = True
        R = None
        for j in near:
            D = float(np.linalg.norm(pos[j] - c))
            if D >= r_out[i] + r_out[j] + gap:
                continue
            if D < r_in[i] + r_in[j] + gap:
                ok = False
                break
            if R is None:
                R = _quat_to_rot(q)
            # the parts of each surface that can come within gap of the other body
            Pi = c + geo[i][3] @ R.T
            Pj = pos[j] + geo[j][3] @ rot[j].T
            Pi = Pi[np.linalg.norm(Pi - pos[j], axis=1) < r_out[j] + gap + 2 * rho]
            Pj = Pj[np.linalg.norm(Pj - c, axis=1) < r_out[i] + gap + 2 * rho]
            dc = _min_dist(Pi, Pj)
            if dc < gap:
                ok = False
                break
            if dc - 2 * rho >= gap:
                continue
            Fi = fine_lab(i, c, R)
            Fj = fine_lab(j, pos[j], rot[j])
            Fi = Fi[np.linalg.norm(Fi - pos[j], axis=1) < r_out[j] + gap]
            Fj = Fj[np.linalg.norm(Fj - c, axis=1) < r_out[i] + gap]
            if _min_dist(Fi, Fj) < gap:
                ok = False
                break
        if not ok:
            continue
        pos[i] = c
        quat[i] = q
        rot[i] = R if R is not None else _quat_to_rot(q)
        cells.setdefault(key, []).append(i)
        placed += 1
        fine.pop(i, None)
    return pos, quat


def tight_radius(kind, data):
    """Largest distance from the area centroid to the surface (from the dense point
    cloud, plus 0.005) for a radial shape; for coordinate shapes the loose bound."""
    if kind != "radial":
        return bounding_radius(kind, data)
    rc = np.asarray(data, dtype=np.float64)
    lmax = int(round(math.sqrt(len(rc)))) - 1
    return _family(lmax).shape(rc)[2]


def placement_geometry(kind, data):
    """(area-centroid offset from the radial origin, inscribed radius, circumscribed
    radius) of a radial shape as used for placement."""
    rc = np.asarray(data, dtype=np.float64)
    lmax = int(round(math.sqrt(len(rc)))) - 1
    xc, r_in, r_out, _ = _family(lmax).shape(rc)
    return xc, r_in, r_out


def workload(name, seed=None):
    """Return a dict describing one synthetic configuration.

    Names: 'two_spheres' (2 unit spheres at (0,0,0), (3,0,0), p = 8),
    'single_sphere', 'random64' (64 SH-perturbed bodies, p = 12, 10 %, bounding gap
    0.5), 'ellipsoids1000' (1000 ellipsoids (1, .8, .6), p = 16, 10 %, bounding gap
    0.1), 'sediment512' (512 perturbed spheres, 10 %, bounding gap 0.5, F = (0,0,-1)),
    'dense4000' (4000 perturbed spheres at volume fraction 20 %, true surface gap 0.1),
    'dense4000_train' (the same generator, another seed) and 'dense512' (a smaller,
    separately seeded sibling); ``tiny``, ``lattice`` and ``workload_perturbed`` build
    other configurations.  Generated workloads are cached per process; callers get a
    copy.
    """
    return copy.deepcopy(_workload_cached(name, seed))


@functools.lru_cache(maxsize=8)
def _workload_cached(name, seed):
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
    if name in ("dense4000", "dense4000_train"):
        # dense4000_train: the dense configuration's generator with another seed
        return workload_perturbed(4000, 12, 0.20, 0.1, rng, name, gap_rule="surface")
    if name == "dense512":
        # a smaller, separately seeded suspension with the dense configuration's statistics
        return workload_perturbed(512, 12, 0.20, 0.1, rng, name, gap_rule="surface")
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


def workload_perturbed(n, p, phi, gap, rng, name="perturbed", lmax=4, amp=0.1, gap_rule="bounding"):
    """n distinct SH-perturbed spheres (one shape each), volume fraction phi, minimum gap
    by the rule `gap_rule` ("bounding": tight bounding spheres; "surface": true surface
    distance)."""
    shapes = [("radial", _radial_perturbed(rng, lmax, amp)) for _ in range(n)]
    side = (n * (4 * math.pi / 3) / phi) ** (1 / 3)
    if gap_rule == "surface":
        pos, quats = _rsa_surface(rng, shapes, side, gap)
    else:
        rb = np.array([tight_radius(k, d) for k, d in shapes])
        pos = _rsa(rng, rb, side, gap)
        quats = _uniform_quats(rng, n)
    return dict(name=name, p=p, eta=1.0, shapes=shapes, shape_id=np.arange(n, dtype=np.int32),
                centres=pos, quats=quats, FT=rng.standard_normal((n, 6)), gap=gap, gap_rule=gap_rule)


def tiny(n=3, p=6, seed=7, amp=0.1, lmax=3, shared=False):
    """A few perturbed bodies on a line-ish cluster, for parity tests (loose bounding radius,
    so the clusters keep a generous gap)."""
    rng = np.random.default_rng(seed)
    ns = 1 if shared else n
    shapes = [("radial", _radial_perturbed(rng, lmax, amp)) for _ in range(ns)]
    rb = np.array([bounding_radius(*s) for s in shapes])
    side = max(2.0, (n * 4.19 / 0.08) ** (1 / 3))
    pos = _rsa(rng, rb[np.zeros(n, int) if shared else np.arange(n)], side, 0.4)
    return dict(name="tiny", p=p, eta=1.0, shapes=shapes,
                shape_id=np.zeros(n, np.int32) if shared else np.arange(n, dtype=np.int32),
                centres=pos, quats=_uniform_quats(rng, n), FT=rng.standard_normal((n, 6)))
