"""Pins of the oracle's pair geometry and contact Jacobian D.

* Closed-form minimum separations (sphere-sphere, perpendicular / parallel /
  collinear segments, sphere against a segment's interior and end).
* Random pairs against brute-force minimisation over the two segment
  parameters (dense grid plus bounded refinement) -- independent of the
  oracle's clamping logic.
* Eq. Dtranspose: D^T = (grad_C Phi) G, i.e. D_l^T V is the rate of change of
  Phi_l under the rigid motion V; checked by central differences with exact
  rotations of the axes.
* Newton's third law (section 1: the method imposes it): D gamma carries zero
  net force and zero net moment about the origin.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _geo(ci, pi, Ri, hi, cj, pj, Rj, hj, box=(0, 0, 0), periodic=0):
    return O.pair_geometry(ci, pi, Ri, hi, cj, pj, Rj, hj, box, periodic)


EX, EY, EZ = np.eye(3)


def test_sphere_sphere_closed_form():
    g = _geo([0, 0, 0], EX, 0.5, 0.0, [1.3, 0.4, -0.2], EY, 0.25, 0.0)
    d = math.sqrt(1.3 ** 2 + 0.4 ** 2 + 0.2 ** 2)
    assert g["phi"] == pytest.approx(d - 0.75, abs=1e-15)
    np.testing.assert_allclose(g["n"], np.array([1.3, 0.4, -0.2]) / d, atol=1e-15)
    assert np.all(g["tau_i"] == 0.0) and np.all(g["tau_j"] == 0.0)


def test_perpendicular_crossing_segments():
    # rod i along x through the origin, rod j along y, lifted by 0.3 in z
    g = _geo([0, 0, 0], EX, 0.025, 0.5, [0.1, -0.2, 0.3], EY, 0.025, 0.5)
    assert g["phi"] == pytest.approx(0.3 - 0.05, abs=1e-15)
    np.testing.assert_allclose(g["n"], EZ, atol=1e-15)
    assert g["s"] == pytest.approx(0.1) and g["t"] == pytest.approx(0.2)


def test_parallel_offset_segments():
    g = _geo([0, 0, 0], EX, 0.025, 0.5, [0.3, 0.2, 0.0], EX, 0.025, 0.5)
    assert g["phi"] == pytest.approx(0.2 - 0.05, abs=1e-15)
    np.testing.assert_allclose(g["n"], EY, atol=1e-15)
    assert g["flags"] & 1
    # midpoint of the overlap [-0.2, 0.5] of the projections
    assert g["s"] == pytest.approx(0.15)


def test_antiparallel_collinear_separated():
    g = _geo([0, 0, 0], EX, 0.025, 0.5, [1.5, 0, 0], -EX, 0.025, 0.5)
    assert g["phi"] == pytest.approx(0.5 - 0.05, abs=1e-15)
    np.testing.assert_allclose(g["n"], EX, atol=1e-15)


def test_sphere_against_segment_interior_and_end():
    # sphere j near the middle of rod i
    g = _geo([0, 0, 0], EX, 0.025, 0.5, [0.2, 0.4, 0.0], EZ, 0.1, 0.0)
    assert g["phi"] == pytest.approx(0.4 - 0.125, abs=1e-15)
    assert g["s"] == pytest.approx(0.2)
    # beyond the end of the rod: nearest point is the end (0.5, 0, 0)
    g = _geo([0, 0, 0], EX, 0.025, 0.5, [0.8, 0.3, 0.0], EZ, 0.1, 0.0)
    assert g["phi"] == pytest.approx(math.sqrt(0.18) - 0.125, abs=1e-15)
    assert g["s"] == 0.5
    # swapped roles give the same separation and the opposite normal
    g2 = _geo([0.8, 0.3, 0.0], EZ, 0.1, 0.0, [0, 0, 0], EX, 0.025, 0.5)
    assert g2["phi"] == pytest.approx(g["phi"], abs=1e-15)
    np.testing.assert_allclose(g2["n"], -g["n"], atol=1e-15)


def test_periodic_minimum_image():
    box = (10.0, 10.0, 10.0)
    g = _geo([0.2, 5, 5], EX, 0.5, 0.0, [9.9, 5, 5], EX, 0.5, 0.0, box, 1)
    assert g["phi"] == pytest.approx(0.3 - 1.0, abs=1e-14)
    np.testing.assert_allclose(g["n"], -EX, atol=1e-15)


def _brute_distance(ci, pi, hi, cj, pj, hj):
    """min over s, t of |c_j + t p_j - c_i - s p_i| by a dense grid and a
    bounded Nelder-Mead-free refinement (coordinate golden sections)."""
    r = np.asarray(cj) - np.asarray(ci)
    pi, pj = np.asarray(pi), np.asarray(pj)
    ss = np.linspace(-hi, hi, 401) if hi > 0 else np.zeros(1)
    ts = np.linspace(-hj, hj, 401) if hj > 0 else np.zeros(1)
    D = (r[None, None, :] + ts[None, :, None] * pj - ss[:, None, None] * pi)
    dist2 = np.einsum("abk,abk->ab", D, D)
    a, b = np.unravel_index(np.argmin(dist2), dist2.shape)
    s, t = ss[a], ts[b]

    def f(s, t):
        d = r + t * pj - s * pi
        return float(d @ d)

    def golden(fun, lo, hi_):
        if hi_ <= lo:
            return lo
        gr = (math.sqrt(5) - 1) / 2
        x1, x2 = hi_ - gr * (hi_ - lo), lo + gr * (hi_ - lo)
        for _ in range(200):
            if fun(x1) < fun(x2):
                hi_ = x2
            else:
                lo = x1
            x1, x2 = hi_ - gr * (hi_ - lo), lo + gr * (hi_ - lo)
        return 0.5 * (lo + hi_)

    for _ in range(60):  # alternating exact line searches (convex problem)
        if hi > 0:
            s = golden(lambda x: f(x, t), -hi, hi)
        if hj > 0:
            t = golden(lambda y: f(s, y), -hj, hj)
    return math.sqrt(f(s, t))


@pytest.mark.parametrize("kind", ["rod-rod", "rod-sphere", "sphere-rod"])
def test_random_pairs_against_brute_force(kind):
    rng = np.random.default_rng(12)
    for _ in range(25):
        pi = rng.standard_normal(3); pi /= np.linalg.norm(pi)
        pj = rng.standard_normal(3); pj /= np.linalg.norm(pj)
        ci = rng.uniform(-0.3, 0.3, 3)
        cj = rng.uniform(-0.6, 0.6, 3)
        hi = 0.5 if kind in ("rod-rod", "rod-sphere") else 0.0
        hj = 0.5 if kind in ("rod-rod", "sphere-rod") else 0.0
        g = _geo(ci, pi, 0.025, hi, cj, pj, 0.03, hj)
        ref = _brute_distance(ci, pi, hi, cj, pj, hj) - 0.055
        assert g["phi"] == pytest.approx(ref, abs=1e-9)
        # the reported closest points realise the reported distance
        d = cj + g["t"] * pj - ci - g["s"] * pi
        assert np.linalg.norm(d) - 0.055 == pytest.approx(g["phi"], abs=1e-14)
        np.testing.assert_allclose(g["n"], d / np.linalg.norm(d), atol=1e-14)


def _rotate(p, omega, h):
    """Exact rotation of p by angle h|omega| about omega (Rodrigues)."""
    th = h * np.linalg.norm(omega)
    if th == 0.0:
        return p.copy()
    k = omega / np.linalg.norm(omega)
    return (p * math.cos(th) + np.cross(k, p) * math.sin(th)
            + k * (k @ p) * (1 - math.cos(th)))


@pytest.mark.parametrize("kind", ["rod-rod", "rod-sphere", "sphere-rod",
                                  "sphere-sphere"])
def test_D_is_rigid_motion_derivative_of_phi(kind):
    """Eq. Dtranspose: D_l^T V = d Phi_l / dt under rigid velocities V."""
    rng = np.random.default_rng(7)
    h = 1e-6
    checked = 0
    while checked < 30:
        pi = rng.standard_normal(3); pi /= np.linalg.norm(pi)
        pj = rng.standard_normal(3); pj /= np.linalg.norm(pj)
        ci = rng.uniform(-0.3, 0.3, 3)
        cj = rng.uniform(-0.5, 0.5, 3)
        hi = 0.5 if kind in ("rod-rod", "rod-sphere") else 0.0
        hj = 0.5 if kind in ("rod-rod", "sphere-rod") else 0.0
        g = _geo(ci, pi, 0.025, hi, cj, pj, 0.025, hj)
        # skip pairs whose closest points sit exactly at a clamp boundary
        # transition or are nearly parallel (non-unique closest points)
        if g["flags"] or min(abs(abs(g["s"]) - hi) if hi else 1,
                             abs(abs(g["t"]) - hj) if hj else 1) < 1e-4 and (
                abs(g["s"]) < hi or abs(g["t"]) < hj):
            continue
        V = rng.standard_normal(12)
        Ui, Wi, Uj, Wj = V[:3], V[3:6], V[6:9], V[9:]

        def phi_at(eps):
            gg = _geo(ci + eps * Ui, _rotate(pi, Wi, eps), 0.025, hi,
                      cj + eps * Uj, _rotate(pj, Wj, eps), 0.025, hj)
            return gg["phi"]

        fd = (phi_at(h) - phi_at(-h)) / (2 * h)
        n, ti, tj = g["n"], g["tau_i"], g["tau_j"]
        DtV = -n @ Ui - ti @ Wi + n @ Uj + tj @ Wj
        assert DtV == pytest.approx(fd, rel=1e-6, abs=1e-8)
        checked += 1


def test_newton_third_law_force_and_moment():
    """Sum of D gamma forces is zero; sum of c x F + T is zero (contact forces
    act along n through the contact points)."""
    s = W.rods_and_spheres(300, 60, seed=5)
    s.periodic = 0  # unwrapped coordinates so that c x F is meaningful
    c = O.find_contacts(s, "cells")
    assert c.nc > 50
    gamma = np.random.default_rng(1).uniform(0, 2, c.nc)
    F = O.D_apply(s.n, c, gamma)
    scale = np.abs(F).max()
    np.testing.assert_allclose(F[:, :3].sum(0), 0.0, atol=1e-12 * scale * c.nc)
    moment = np.cross(s.pos, F[:, :3]).sum(0) + F[:, 3:].sum(0)
    np.testing.assert_allclose(moment, 0.0, atol=1e-11 * scale * c.nc)


def test_mobility_block_eigenstructure():
    """Mob acts as a_par along p and a_perp across it (forces), b_par / b_perp
    for torques; spheres are isotropic."""
    rng = np.random.default_rng(3)
    p = rng.standard_normal((5, 3)); p /= np.linalg.norm(p, axis=1, keepdims=True)
    mob = rng.uniform(0.1, 2.0, (5, 4))
    perp = np.cross(p, rng.standard_normal((5, 3)))
    F = np.concatenate([p * 2.0, perp], axis=1)
    U = O.mobility(p, mob, F)
    np.testing.assert_allclose(U[:, :3], 2.0 * mob[:, 0:1] * p, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(U[:, 3:], mob[:, 3:4] * perp, rtol=1e-13, atol=1e-15)
    F2 = np.concatenate([perp, p], axis=1)
    U2 = O.mobility(p, mob, F2)
    np.testing.assert_allclose(U2[:, :3], mob[:, 1:2] * perp, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(U2[:, 3:], mob[:, 2:3] * p, rtol=1e-13, atol=1e-15)
