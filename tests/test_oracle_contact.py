"""Pins of the oracle's contact-force algorithm (§3.3).

Two touching spheres pushed together by equal and opposite forces must stop (zero net
load on each body after contact: by uniqueness V = 0) with the contact force exactly
cancelling the push; a sheared pair must move without slip at the contact point with
the mirror symmetry of the configuration; contact forces are internal (zero net force
and torque); the contact search is checked by hand."""
import math

import numpy as np

from oracle import contact as ct
from oracle import system as sysm


def unit_sphere_coef():
    k = math.sqrt(4.0 * math.pi / 3.0)
    c = np.zeros((3, 4))
    c[0, 3], c[1, 1], c[2, 2] = k, k, k
    return c


def touching_pair(p=8, gap=0.0, third=None):
    """Unit spheres at (0,0,0) and (2+gap,0,0), identity orientation: with p even the grid
    has nodes at +x and -x, so the closest node pair lies on the line of centres."""
    shape = sysm.Shape(unit_sphere_coef(), p)
    cen = [[0.0, 0, 0], [2.0 + gap, 0, 0]] + ([third] if third is not None else [])
    n = len(cen)
    return sysm.Problem([shape], [0] * n, np.array(cen), np.array([[1.0, 0, 0, 0]] * n))


def dense_mobility(prob):
    return lambda FT: sysm.solve_dense(prob, FT)[2]


def test_contact_search_by_hand():
    prob = touching_pair(gap=0.01, third=[0.0, 5.0, 0.0])
    c = ct.find_contacts(prob, 0.05)
    assert len(c) == 1 and c[0][:2] == (0, 1)
    assert np.abs(c[0][2] - np.array([1.005, 0, 0])).max() < 1e-14
    assert ct.find_contacts(prob, 0.009) == []
    assert len(ct.find_contacts(prob, 1.01 * (5.0 - 2.0))) == 2


def test_pushed_pair_stops_and_contact_force_cancels_the_push():
    # gap 0.02 < delta: "touching"; with F_c = -F every body carries zero load, so V = 0
    # for any discretization, and the contact point lies on the line of centres
    prob = touching_pair(gap=0.02)
    F = 0.7
    FT = np.zeros((2, 6))
    FT[0, 0], FT[1, 0] = F, -F
    contacts = ct.find_contacts(prob, 0.05)
    assert len(contacts) == 1
    V0, Fc, V = ct.solve_with_contacts(prob, FT, contacts, dense_mobility(prob))
    assert V0[0, 0] > 1e-3 and V0[1, 0] < -1e-3          # without contact they approach
    assert np.abs(V).max() < 1e-12
    assert np.abs(Fc[0] - np.array([-F, 0, 0])).max() < 1e-12


def test_sheared_pair_moves_without_slip_with_mirror_symmetry():
    # the node sets are centrally symmetric, so the point reflection through the contact
    # point is an exact symmetry of the discrete problem
    prob = touching_pair(gap=0.02)
    FT = np.zeros((2, 6))
    FT[0, 1], FT[1, 1] = 1.0, -1.0
    contacts = ct.find_contacts(prob, 0.05)
    V0, Fc, V = ct.solve_with_contacts(prob, FT, contacts, dense_mobility(prob))
    C, D = ct.contact_maps(prob, contacts)
    assert np.abs(D @ V.reshape(-1)).max() < 1e-12 * np.abs(V).max()
    assert np.abs(D @ V0.reshape(-1)).max() > 1e-3       # it did slip without the force
    # point reflection through the contact point maps the pair onto itself with the loads
    # reversed: v_b = -v_a, w_b = w_a
    assert np.abs(V[1, :3] + V[0, :3]).max() < 1e-10
    assert np.abs(V[1, 3:] - V[0, 3:]).max() < 1e-10
    assert abs(V[0, 5]) > 1e-3                            # the pair spins about z


def test_contact_forces_are_internal():
    rng = np.random.default_rng(4)
    prob = touching_pair(gap=0.02, third=[1.0, 1.75, 0.0])
    contacts = ct.find_contacts(prob, 0.05)
    assert len(contacts) >= 1
    C, _ = ct.contact_maps(prob, contacts)
    Fc = rng.standard_normal(C.shape[1])
    loads = (C @ Fc).reshape(prob.n, 6)
    assert np.abs(loads[:, :3].sum(axis=0)).max() < 1e-14
    total_torque = sum(loads[i, 3:] + np.cross(prob.c[i], loads[i, :3]) for i in range(prob.n))
    assert np.abs(total_torque).max() < 1e-13
