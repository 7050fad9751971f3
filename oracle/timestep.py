"""Rigid-body evolution of centroids and orientations, FP64 oracle (§3.3, Algorithm 1).

Test infrastructure only (see ``oracle/__init__``).

§3.3 evolves X^c_i with dX^c/dt = v_i and R_i with dR/dt z = omega_i x z by an
explicit Runge-Kutta method, optionally through a unit quaternion.  The reading
used here: classical four-stage RK4 on (c_i, q_i) with
    dq/dt = 1/2 (0, omega) (x) q          (omega in the lab frame, q maps body -> lab)
stage quaternions normalised before they define a pose (and the derivative), the
final quaternion normalised.  For constant omega the exact solution is
R(t) = exp(t [omega]x) R(0), i.e. Rodrigues' formula with angle |omega| t.
"""
import numpy as np


def quat_mul(a, b):
    """Hamilton product a (x) b for arrays (..., 4) in (w, x, y, z) order."""
    aw, ax, ay, az = np.moveaxis(np.asarray(a, dtype=np.float64), -1, 0)
    bw, bx, by, bz = np.moveaxis(np.asarray(b, dtype=np.float64), -1, 0)
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], axis=-1)


def normalize(q):
    q = np.asarray(q, dtype=np.float64)
    return q / np.linalg.norm(q, axis=-1, keepdims=True)


def rates(VW, q):
    """(dc/dt, dq/dt) from velocities VW (n, 6) at orientations q (n, 4)."""
    om = np.concatenate([np.zeros((len(q), 1)), VW[:, 3:]], axis=1)
    return VW[:, :3].copy(), 0.5 * quat_mul(om, q)


def rk4_step(velocity_fn, c, q, dt):
    """One classical RK4 step.  velocity_fn(c, q) -> VW (n, 6) for normalised q."""
    c0 = np.asarray(c, dtype=np.float64)
    q0 = normalize(q)
    stages = [(0.0, None), (0.5, 0), (0.5, 1), (1.0, 2)]
    kc, kq = [], []
    for a, prev in stages:
        cs = c0 if prev is None else c0 + a * dt * kc[prev]
        qs = q0 if prev is None else normalize(q0 + a * dt * kq[prev])
        VW = velocity_fn(cs, qs)
        dc, dq = rates(VW, qs)
        kc.append(dc)
        kq.append(dq)
    c1 = c0 + dt / 6.0 * (kc[0] + 2 * kc[1] + 2 * kc[2] + kc[3])
    q1 = normalize(q0 + dt / 6.0 * (kq[0] + 2 * kq[1] + 2 * kq[2] + kq[3]))
    return c1, q1


def rodrigues(omega, t):
    """exp(t [omega]x) for constant omega (general |omega|)."""
    om = np.asarray(omega, dtype=np.float64)
    th = np.linalg.norm(om) * t
    if th == 0.0:
        return np.eye(3)
    k = om / np.linalg.norm(om)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K
