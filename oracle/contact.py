"""Contact forces between touching bodies (§3.3, contact force algorithm), FP64 oracle.

Test infrastructure only (see ``oracle/__init__``).

For every pair of surfaces touching at a point x*, §3.3 adds a force F_k on one body
and -F_k on the other so that the two rigid motions agree at x* (no slip):

    v_a + w_a x (x* - c_a) = v_b + w_b x (x* - c_b).

With C the (6n x 3 n_c) map from the contact forces F_c to body forces and torques, D
the (3 n_c x 6n) map from body velocities to the velocity differences at the contact
points and M the mobility matrix, the contact forces solve (D M C) F_c = -D V_0, where
V_0 are the velocities without contact forces; then V = V_0 + M C F_c.  M C is built
one column at a time, one mobility solve per unit contact-force component.

Readings (the paper defers the details to the work it cites):
  * bodies a < b touch when the smallest distance between a node of a and a node of b
    is below delta; x* is the midpoint of that closest node pair (ties: smallest
    node indices, a's first);
  * the contact force acts on body a as +F_k and on body b as -F_k, both at x*, with
    torques about the area centroids: (x* - c_a) x F_k and -(x* - c_b) x F_k.
"""
import numpy as np


def find_contacts(prob, delta):
    """[(a, b, x*)] for every body pair a < b whose closest node pair is within delta."""
    out = []
    for a in range(prob.n):
        Xa = prob.X[prob.sl(a)]
        for b in range(a + 1, prob.n):
            Xb = prob.X[prob.sl(b)]
            d2 = np.sum((Xa[:, None, :] - Xb[None, :, :]) ** 2, axis=2)
            k = int(np.argmin(d2))          # row-major: smallest a-node, then b-node, on ties
            ia, ib = divmod(k, d2.shape[1])
            if np.sqrt(d2[ia, ib]) < delta:
                out.append((a, b, 0.5 * (Xa[ia] + Xb[ib])))
    return out


def contact_maps(prob, contacts):
    """C (6n x 3nc): body forces/torques of unit contact forces; D (3nc x 6n): velocity
    differences at the contact points.  Body loads are ordered (F, T) per body."""
    n, nc = prob.n, len(contacts)
    C = np.zeros((6 * n, 3 * nc))
    D = np.zeros((3 * nc, 6 * n))
    for k, (a, b, xs) in enumerate(contacts):
        ra, rb = xs - prob.c[a], xs - prob.c[b]
        for e in range(3):
            f = np.zeros(3)
            f[e] = 1.0
            C[6 * a:6 * a + 3, 3 * k + e] = f
            C[6 * a + 3:6 * a + 6, 3 * k + e] = np.cross(ra, f)
            C[6 * b:6 * b + 3, 3 * k + e] = -f
            C[6 * b + 3:6 * b + 6, 3 * k + e] = -np.cross(rb, f)
        # v + w x r = v - r x w: d/dv = I, d/dw = -[r]x
        def skew(r):
            return np.array([[0, -r[2], r[1]], [r[2], 0, -r[0]], [-r[1], r[0], 0]])
        D[3 * k:3 * k + 3, 6 * a:6 * a + 3] = np.eye(3)
        D[3 * k:3 * k + 3, 6 * a + 3:6 * a + 6] = -skew(ra)
        D[3 * k:3 * k + 3, 6 * b:6 * b + 3] = -np.eye(3)
        D[3 * k:3 * k + 3, 6 * b + 3:6 * b + 6] = skew(rb)
    return C, D


def solve_with_contacts(prob, FT, contacts, mobility_solve, V0=None):
    """(V_0, F_c, V): mobility_solve(FT (n, 6)) -> VW (n, 6) is the mobility problem on
    this configuration (e.g. a dense oracle solve).  V0, if given, replaces the solve
    with the loads FT (e.g. velocities driven by a magnetic traction, §4)."""
    if V0 is None:
        V0 = mobility_solve(np.asarray(FT, dtype=np.float64).reshape(prob.n, 6))
    V0 = np.asarray(V0, dtype=np.float64).reshape(prob.n, 6)
    if not contacts:
        return V0, np.zeros((0, 3)), V0
    C, D = contact_maps(prob, contacts)
    MC = np.zeros((6 * prob.n, C.shape[1]))
    for k in range(C.shape[1]):
        MC[:, k] = mobility_solve(C[:, k].reshape(prob.n, 6)).reshape(-1)
    Fc = np.linalg.solve(D @ MC, -D @ V0.reshape(-1))
    V = V0 + (MC @ Fc).reshape(prob.n, 6)
    return V0, Fc.reshape(-1, 3), V
