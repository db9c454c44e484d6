"""Pins of the oracle's particle-wall constraints (the boundary extension of
section 3.3: a D column with the particle's 6 entries only) for the planar
faces of a closed box."""
import math

import numpy as np
import pytest

import oracle as O
import oracle.timestep as T
import workloads as W

FLOOR = 1 << 4          # face 4: the lower z face


def _closed(s, walls=63):
    s.periodic = 0
    s.walls = walls
    return s


def _single(pos, axis, R, h, mob, f_ext, side=10.0, walls=FLOOR, delta=0.05, dt=0.01,
            tol=1e-12):
    s = W.Suspension("one", np.array([pos], float), np.array([axis], float) / np.linalg.norm(axis),
                     np.array([R]), np.array([h]), np.array([mob]), np.array([f_ext], float),
                     np.full(3, side), delta, dt, tol)
    return _closed(s, walls)


def test_wall_contacts_brute_force_equals_cell_list():
    s = _closed(W.rods_and_spheres(400, 80, seed=W.SEED_BASE + 960))
    s.delta = 0.05
    a, b = O.find_contacts(s, "brute"), O.find_contacts(s, "cells")
    assert np.array_equal(a.keys(), b.keys())
    assert np.count_nonzero(a.j < 0) > 20
    for f in ("phi", "nrm", "tau_i", "tau_j"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    # canonical order: by i, then j (wall codes -1 - face are negative)
    k = a.keys()
    assert np.all(np.diff(k) > 0)


def _rotate(v, w, ang):
    nw = np.linalg.norm(w)
    if nw == 0.0:
        return v
    w = w / nw
    return v * math.cos(ang) + np.cross(w, v) * math.sin(ang) + w * (w @ v) * (1 - math.cos(ang))


@pytest.mark.parametrize("face", range(6))
def test_wall_phi_and_column_against_definitions(face):
    """Phi is the smallest distance of the core segment to the plane minus
    R (checked on a fine sampling, exact at the ends); D_l^T V is the rate of
    Phi under the rigid motion V (central differences with exact rotation)."""
    rng = np.random.default_rng(face)
    a, up = face // 2, face % 2
    for _ in range(20):
        c = rng.uniform(2.0, 8.0, 3)
        c[a] = 0.3 if not up else 9.7
        p = rng.standard_normal(3)
        p /= np.linalg.norm(p)
        R, h = 0.05, rng.choice([0.0, 0.5])
        s = _single(c, p, R, h, W.rod_mobility(), np.zeros(6), walls=1 << face, delta=1.0)
        cs = O.find_contacts(s)
        assert cs.nc == 1 and cs.j[0] == -1 - face
        m = np.zeros(3)
        m[a] = -1.0 if up else 1.0
        plane = 10.0 if up else 0.0
        ts = np.linspace(-h, h, 2001)
        d = np.array([m @ (c + t * p) - m[a] * plane for t in ts])
        assert cs.phi[0] == pytest.approx(d.min() - R, abs=1e-12)
        V = rng.standard_normal(6)
        hh = 1e-6
        ph = []
        for sg in (1, -1):
            s2 = _single(c + sg * hh * V[:3], _rotate(p, V[3:], sg * hh * np.linalg.norm(V[3:])),
                         R, h, W.rod_mobility(), np.zeros(6), walls=1 << face, delta=1.0)
            ph.append(O.find_contacts(s2).phi[0])
        fd = (ph[0] - ph[1]) / (2 * hh)
        U = np.zeros((1, 6))
        U[0] = V
        assert O.DT_apply(cs, U)[0] == pytest.approx(fd, rel=1e-7, abs=1e-7)


def test_sphere_settles_on_the_floor_exactly():
    """A sphere pushed down onto the floor moves freely until it is close,
    then the converged LCP closes the gap exactly and keeps it closed (Phi is
    linear in the height)."""
    R, F, dt = 0.5, 50.0, 0.01
    mt = W.sphere_mobility(R)[0]
    s = _single([5.0, 5.0, 1.2], [0, 0, 1.0], R, 0.0, W.sphere_mobility(R), [0, 0, -F, 0, 0, 0],
                dt=dt, delta=0.1)
    quat, rec = T.quat_from_axis(s.axis), None
    gap = 1.2 - R
    for k in range(40):
        s, quat, rec = T.step(s, quat, rec)
        gap = max(0.0, gap - mt * F * dt)
        assert abs((s.pos[0, 2] - R) - gap) < 1e-12, (k, s.pos[0, 2] - R, gap)
        assert s.pos[0, 0] == 5.0 and s.pos[0, 1] == 5.0
    assert gap == 0.0


def test_tilted_rod_settles_flat():
    """A tilted rod pushed down lands on its lower end; the wall force at the
    end turns it towards the floor until it lies flat. With one constraint
    per particle and wall at the closest point, a nearly flat rod ends in a
    two-step cycle (each step lifts the lower end and lowers the other one),
    so its core stays within a depth proportional to the rotation per step
    (h Omega dt, Omega ~ b_perp h F) of the floor."""
    p = np.array([1.0, 0.0, 0.6])
    dt, h, F = 0.002, 0.5, 1.0
    mob = W.rod_mobility()
    s = _single([5.0, 5.0, 0.6], p, 0.025, h, mob, [0, 0, -F, 0, 0, 0], dt=dt, delta=0.05,
                tol=1e-12)
    quat, rec = T.quat_from_axis(s.axis), None
    tilt = [abs(s.axis[0, 2])]
    lowest = []
    for _ in range(3000):
        s, quat, rec = T.step(s, quat, rec)
        tilt.append(abs(s.axis[0, 2]))
        ends = s.pos[0, 2] + np.array([-h, h]) * s.axis[0, 2]
        lowest.append(ends.min() - 0.025)
    # the cycle turns the rod by Omega dt with Omega = b_perp h F (the wall
    # force balances F), so |p_z| ends at Omega dt / 2 and the lowered end
    # sits 2 h |p_z| below the floor
    turn = mob[3] * h * F * dt
    assert max(tilt[-50:]) <= 1.01 * turn / 2
    assert min(lowest) >= -1.01 * h * turn
    assert tilt[1000] < tilt[0]

def test_wall_adjoint_finite_differences():
    """The adjoint with wall contacts (dPhi/dc_i is the face's inward normal;
    n and tau do not move with the centre) against central differences of
    polished solves, for the contact-force loss 1/2 ||D gamma||^2."""
    rng = np.random.default_rng(961)
    ns = 6                                   # a row of spheres just above the floor
    pos = np.column_stack([2.0 + np.cumsum(np.r_[0.0, 0.99 + 0.005 * rng.random(ns - 1)]),
                           np.full(ns, 5.0), 0.495 + 0.004 * rng.random(ns)])
    pos[:, 1] += 0.01 * rng.standard_normal(ns)
    axis = np.tile([0.0, 0.0, 1.0], (ns, 1))
    rad, hl, mob = np.full(ns, 0.5), np.zeros(ns), W.sphere_mobility(np.full(ns, 0.5))
    # (each slightly overlapping the floor and its neighbours, so that every
    # contact carries a force) and two tilted rods with one end in the floor
    rp = np.array([[3.0, 7.0, 0.16], [6.0, 3.0, 0.19]])
    ra = np.array([[0.8, 0.2, 0.3], [-0.5, 0.7, 0.35]])
    ra /= np.linalg.norm(ra, axis=1, keepdims=True)
    pos = np.vstack([pos, rp])
    axis = np.vstack([axis, ra])
    rad = np.concatenate([rad, [0.025, 0.025]])
    hl = np.concatenate([hl, [0.5, 0.5]])
    mob = np.vstack([mob, np.tile(W.rod_mobility(), (2, 1))])
    n = ns + 2
    f = np.zeros((n, 6))
    f[:, :3] = 0.3 * rng.standard_normal((n, 3))
    f[:, 2] -= 3.0
    f[:ns, 0] += np.linspace(2.0, -2.0, ns)     # squeeze the row together
    s = W.Suspension("floor", pos, axis, rad, hl, mob, f, np.full(3, 10.0), 0.1, 1e-3, 1e-12)
    s = _closed(s, FLOOR | 1 | 2 | 4 | 8)
    u_nc = O.mobility(s.axis, s.mob, s.f_ext)

    def solve(sp):
        c = O.find_contacts(sp)
        q = O.build_q(c, u_nc, sp.dt)
        g, _, _ = O.bbpgd(sp, c, q, tol=1e-11)
        gp, _, passes = O.polish(sp, c, q, g)
        return c, q, gp

    c, q, gam = solve(s)
    assert np.count_nonzero((c.j < 0) & (gam > 0)) >= 3 and np.count_nonzero((c.j >= 0) & (gam > 0)) >= 2
    ev = np.linalg.eigvalsh(O.M_matrix(s, c).toarray())
    if ev[0] < 1e-10:
        pytest.skip("singular M")
    act = gam > 0
    F = O.D_apply(n, c, gam)
    _, dpos, _ = O.adjoint(s, c, q, u_nc, gam, dL_dF=F)
    hp = 1e-7
    done = 0
    for _ in range(20):
        if done >= 5:
            break
        V = rng.standard_normal((n, 3))
        V /= np.linalg.norm(V)
        L = []
        for sg in (1, -1):
            sp = W.Suspension(**{**s.__dict__, "pos": s.pos + sg * hp * V})
            cp, qp, gp = solve(sp)
            if not np.array_equal(cp.keys(), c.keys()) or not np.array_equal(gp > 0, act):
                break
            Fp = O.D_apply(n, cp, gp)
            L.append(0.5 * float(np.sum(Fp * Fp)))
        if len(L) < 2:
            continue
        fd = (L[0] - L[1]) / (2 * hp)
        assert abs(float(np.sum(dpos * V)) - fd) <= 1e-5 * np.linalg.norm(dpos)
        done += 1
    assert done >= 3
