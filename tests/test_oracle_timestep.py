"""Pins of the oracle's time stepping (section 3.2, Eq. time-step, and the
quaternion kinematics of section 2) against closed forms and invariants."""
import math

import numpy as np
import pytest

import oracle.timestep as T
import workloads as W


def _pair(r, x0, x1, f, delta, dt, tol=1e-12, side=40.0):
    """Two spheres of radius r at centres x0, x1, forces +f / -f."""
    pos = np.array([x0, x1], dtype=np.float64)
    f_ext = np.zeros((2, 6))
    f_ext[0, :3] = f
    f_ext[1, :3] = -np.asarray(f)
    rad = np.full(2, r)
    return W.Suspension("pair", pos, np.tile([0.0, 0.0, 1.0], (2, 1)), rad, np.zeros(2),
                        W.sphere_mobility(rad), f_ext, np.full(3, side), delta, dt, tol)


def _rotate(v, w, ang):
    """Rodrigues rotation of v about unit w by ang."""
    return (v * math.cos(ang) + np.cross(w, v) * math.sin(ang)
            + w * (w @ v) * (1.0 - math.cos(ang)))


def test_quaternion_axis_round_trip():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((50, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    a = np.vstack([a, [[0, 0, 1.0], [0, 0, -1.0], [1.0, 0, 0]]])
    q = T.quat_from_axis(a)
    np.testing.assert_allclose(np.linalg.norm(q, axis=1), 1.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(T.quat_axis(q), a, rtol=0, atol=1e-14)
    for qq in q[:5]:
        R = T.rotation(qq)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1.0) < 1e-14


def test_psi_is_the_quaternion_rate_of_a_space_frame_rotation():
    """theta_dot = Psi Omega makes R(theta) rotate at Omega: d/dt R = [Omega]x R,
    checked by a central difference of R along the flow."""
    rng = np.random.default_rng(4)
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w = rng.standard_normal(3)
    h = 1e-6
    Rp = T.rotation(q + h * T.psi(q) @ w)
    Rm = T.rotation(q - h * T.psi(q) @ w)
    dR = (Rp - Rm) / (2 * h)
    wx = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    np.testing.assert_allclose(dR, wx @ T.rotation(q), atol=1e-8)


def test_free_rod_translation_and_rotation_closed_form():
    """One rod alone, force and torque along a fixed direction w normal to
    its axis: it translates at a_perp F and turns about w, each normalised
    Euler step by 2 atan(|Omega| dt / 2)."""
    p0 = np.array([1.0, 2.0, 2.0]) / 3.0
    w = np.cross(p0, [0.0, 0.0, 1.0])
    w /= np.linalg.norm(w)
    mob = W.rod_mobility()
    f = np.zeros((1, 6))
    f[0, :3] = 0.7 * w
    f[0, 3:] = 0.3 * w
    s = W.Suspension("rod", np.array([[5.0, 5.0, 5.0]]), p0[None, :], np.array([0.025]),
                     np.array([0.5]), mob[None, :], f, np.full(3, 20.0), 0.015, 0.05, 1e-12)
    K = 40
    out, quat, recs = T.run(s, K)
    assert all(r.i.size == 0 for r in recs)
    np.testing.assert_allclose(out.pos[0], s.pos[0] + K * s.dt * mob[1] * 0.7 * w, rtol=0,
                               atol=1e-13)
    om = mob[3] * 0.3
    ang = K * 2.0 * math.atan(om * s.dt / 2.0)
    np.testing.assert_allclose(out.axis[0], _rotate(p0, w, ang), rtol=0, atol=1e-13)


def test_head_on_spheres_stop_touching():
    """Phi is linear along the line of centres, so once the pair is close the
    converged LCP closes the gap exactly and keeps it closed; before that the
    spheres move freely. The centre of mass never moves."""
    r, F, dt = 0.5, 1.0, 0.05
    mt = W.sphere_mobility(r)[0]
    s = _pair(r, [10.0, 10.0, 10.0], [10.0 + 2 * r + 0.3, 10.0, 10.0], [F, 0, 0], 0.1, dt)
    com = s.pos.sum(axis=0)
    gap, closing = 0.3, 2 * mt * F * dt
    quat, rec = T.quat_from_axis(s.axis), None
    for k in range(30):
        s, quat, rec = T.step(s, quat, rec)
        gap = max(0.0, gap - closing)
        g_now = s.pos[1, 0] - s.pos[0, 0] - 2 * r
        assert abs(g_now - gap) < 1e-12, (k, g_now, gap)
        np.testing.assert_allclose(s.pos.sum(axis=0), com, rtol=0, atol=1e-12)
        assert np.all(s.pos[:, 1:] == 10.0)
    assert gap == 0.0


def test_two_spheres_pass_over_each_other():
    """The paper's two-sphere experiment with the dry mobility: spheres
    dragged by opposite forces along x with a vertical offset a go through
    (A) a close pair with zero force, (B) a positive force, (C) the force
    dying out as they roll over, (D) zero force while still close, then no
    pair; the centre of mass stays fixed and afterwards the vertical offset
    is the contact distance 2 a_c."""
    a = 1.0
    ac = 1.01 * a
    F, dt = 1.0, 0.02
    mt = W.sphere_mobility(ac)[0]
    s = _pair(ac, [10.0, 10.0, 10.0], [10.0 + 4.0 * a, 10.0 + a, 10.0], [F, 0, 0],
              0.3 * 2 * ac, dt)
    com = s.pos.sum(axis=0)
    stages = []
    min_gap = 1.0
    steps = int(round(8.0 * a / (2 * mt * F * dt)))
    quat, rec = T.quat_from_axis(s.axis), None
    for _ in range(steps):
        s, quat, rec = T.step(s, quat, rec)
        d = s.pos[1] - s.pos[0]
        min_gap = min(min_gap, np.linalg.norm(d) - 2 * ac)
        if rec.i.size == 0:
            st = "none"
        else:
            st = "force" if rec.gamma[0] > 0 else "zero"
        if not stages or stages[-1] != st:
            stages.append(st)
        np.testing.assert_allclose(s.pos.sum(axis=0), com, rtol=0, atol=1e-11)
    assert stages == ["none", "zero", "force", "zero", "none"], stages
    assert min_gap > -1e-3 * ac                      # linearised constraint, small dt
    dy = s.pos[1, 1] - s.pos[0, 1]
    assert abs(dy - 2 * ac) < 2e-3 * ac, dy


def test_warm_start_reuses_previous_gamma():
    """A warm start begins from the previous gamma of the same pairs: a step
    repeated from the same configuration starts at its own solution and
    Algorithm 1 stops at its first check (one MVOP). Warm and cold runs agree
    step by step (same pairs, gamma within the solver tolerance's reach)."""
    s = W.rods(300, seed=W.SEED_BASE + 901, pairs_per_rod=6.0)
    q0 = T.quat_from_axis(s.axis)
    _, _, rec = T.step(s, q0, None, warm=True, tol=1e-10)
    assert rec.iters > 10
    _, _, again = T.step(s, q0, rec, warm=True, tol=1e-10)
    assert np.array_equal(again.i, rec.i) and again.iters == 0 and again.mvops == 1
    np.testing.assert_array_equal(again.gamma, rec.gamma)
    _, _, rw = T.run(s, 3, warm=True, tol=1e-10)
    _, _, rc = T.run(s, 3, warm=False, tol=1e-10)
    for w, c in zip(rw, rc):
        assert np.array_equal(w.i, c.i) and np.array_equal(w.j, c.j)
        np.testing.assert_allclose(w.gamma, c.gamma, rtol=0,
                                   atol=1e-6 * np.abs(c.gamma).max())
