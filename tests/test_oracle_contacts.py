"""Pins of the oracle's close-pair set A(C, delta) = {l : Phi_l <= delta}
(section 3.2).

* Two independent searches agree exactly: every pair (brute force) against a
  cell list, on sphere, rod and mixed suspensions, periodic and not, and on a
  box only slightly wider than twice the interaction range.
* Each listed pair is in canonical order and its stored frame equals the
  single-pair geometry.
* The mean number of close pairs matches closed forms of the workload recipe:
  n (4/3) pi (2R + delta)^3 neighbours per sphere, and the Onsager excluded
  volume of spherocylinders for rods (6 per rod by construction).
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _same(a, b):
    assert a.nc == b.nc
    np.testing.assert_array_equal(a.i, b.i)
    np.testing.assert_array_equal(a.j, b.j)
    np.testing.assert_array_equal(a.phi, b.phi)
    np.testing.assert_array_equal(a.nrm, b.nrm)


@pytest.mark.parametrize("make", [
    lambda: W.workload(1),
    lambda: W.rods(2500, seed=3),
    lambda: W.rods_and_spheres(1500, 300, seed=4),
    lambda: W.rods(500, seed=9, min_side=2.2),       # 2 cells per axis
    lambda: W.spheres(400, 0.35, seed=11),
])
def test_brute_force_equals_cell_list(make):
    s = make()
    a = O.find_contacts(s, "brute")
    b = O.find_contacts(s, "cells")
    assert a.nc > 0
    _same(a, b)
    assert np.all(a.i < a.j)
    key = a.keys()
    assert np.all(np.diff(key) > 0)          # canonical, no duplicates
    assert np.all(a.phi <= s.delta)


def test_non_periodic_box():
    s = W.rods_and_spheres(800, 200, seed=21)
    s.periodic = 0
    s.pos = s.pos * 1.3 - 2.0                 # some particles outside the box
    a = O.find_contacts(s, "brute")
    b = O.find_contacts(s, "cells")
    _same(a, b)


def test_frames_equal_pair_geometry():
    s = W.rods_and_spheres(600, 150, seed=8)
    c = O.find_contacts(s, "cells")
    for l in range(0, c.nc, max(1, c.nc // 50)):
        i, j = c.i[l], c.j[l]
        g = O.pair_geometry(s.pos[i], s.axis[i], s.radius[i], s.half_len[i],
                            s.pos[j], s.axis[j], s.radius[j], s.half_len[j],
                            s.box, 1)
        assert g["phi"] == c.phi[l]
        np.testing.assert_array_equal(g["n"], c.nrm[l])
        np.testing.assert_array_equal(g["tau_i"], c.tau_i[l])
        np.testing.assert_array_equal(g["tau_j"], c.tau_j[l])


def test_sphere_pair_density_closed_form():
    s = W.workload(1)
    c = O.find_contacts(s, "cells")
    density = s.n / np.prod(s.box)
    expect = density * 4.0 / 3.0 * math.pi * (1.0 + s.delta) ** 3
    got = 2.0 * c.nc / s.n
    assert got == pytest.approx(expect, rel=0.08)


def test_rod_pair_density_onsager():
    s = W.rods(20000, seed=W.SEED_BASE + 2)
    c = O.find_contacts(s, "cells")
    got = 2.0 * c.nc / s.n
    assert got == pytest.approx(6.0, rel=0.03)
