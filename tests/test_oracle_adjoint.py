"""Pins of the oracle's implicit adjoint (not in the paper: implicit
differentiation of the LCP of LCP LCPdef on its active set).

* Two spheres head-on, closed form: gamma = -q/M with M = 2 m_t and
  q = (|c_j - c_i| - 2R)/dt + D^T U_nc, so dgamma/dq = -1/M and
  dgamma/dc_j = -n/(M dt); for L = 1/2 ||D gamma||^2 = gamma^2 the chain
  rule gives dL/dq = -2 gamma/M and dL/dc_j = -2 gamma n/(M dt).
* Central finite differences (h small) of exactly polished solves, in random
  directions of q and of the centres, for a linear loss in gamma and for the
  contact-force loss 1/2 ||D gamma||^2 (which also depends on the centres
  through D). Directions whose perturbation changes the pair set or the
  active set are redrawn.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _two_spheres(gap, U, direction):
    d = np.asarray(direction, float)
    d /= np.linalg.norm(d)
    pos = np.stack([np.zeros(3), (1.0 + gap) * d]) + 5.0
    s = W.Suspension("two", pos, np.tile([0.0, 0.0, 1.0], (2, 1)),
                     np.full(2, 0.5), np.zeros(2),
                     W.sphere_mobility(np.full(2, 0.5)), np.zeros((2, 6)),
                     np.full(3, 20.0), delta=0.1, dt=1e-3)
    u_nc = np.zeros((2, 6))
    u_nc[0, :3] = U * d
    u_nc[1, :3] = -U * d
    return s, u_nc, d


@pytest.mark.parametrize("direction", [(1, 0, 0), (0.2, 0.7, -0.4)])
def test_two_sphere_closed_form(direction):
    s, u_nc, d = _two_spheres(0.01, 30.0, direction)
    c = O.find_contacts(s)
    q = O.build_q(c, u_nc, s.dt)
    gamma, g, st = O.bbpgd(s, c, q)
    M = 2.0 / (6 * math.pi * 0.5)
    assert gamma[0] > 0
    # L = gamma
    dq, dpos, w = O.adjoint(s, c, q, u_nc, gamma, dL_dgamma=np.ones(1))
    assert dq[0] == pytest.approx(-1.0 / M, rel=1e-12)
    np.testing.assert_allclose(dpos[1], -d / (M * s.dt), rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(dpos[0], d / (M * s.dt), rtol=1e-9, atol=1e-9)
    # L = 1/2 ||D gamma||^2 = gamma^2
    F = O.D_apply(2, c, gamma)
    dq, dpos, w = O.adjoint(s, c, q, u_nc, gamma, dL_dF=F)
    assert dq[0] == pytest.approx(-2 * gamma[0] / M, rel=1e-12)
    np.testing.assert_allclose(dpos[1], -2 * gamma[0] * d / (M * s.dt),
                               rtol=1e-9, atol=1e-6)


def _system(kind, seed):
    if kind == "rods":
        s = W.rods(60, seed=seed, pairs_per_rod=5.0)
    elif kind == "spheres":
        s = W.spheres(50, 0.2, seed=seed)
    else:
        s = W.rods_and_spheres(50, 15, seed=seed)
    return s


def _solve(s, u_nc, q_override=None, ref=None):
    c = O.find_contacts(s)
    q = O.build_q(c, u_nc, s.dt) if q_override is None else q_override
    gamma, g, st = O.bbpgd(s, c, q, tol=1e-11)
    gp, gg, passes = O.polish(s, c, q, gamma)
    assert passes > 0
    return c, q, gp


def _losses(s, c, gamma, weights):
    F = O.D_apply(s.n, c, gamma)
    return float(weights @ gamma), 0.5 * float(np.sum(F * F)), F


@pytest.mark.parametrize("kind", ["rods", "mixed", "spheres"])
def test_finite_differences_q_and_positions(kind):
    seed = {"rods": 71, "mixed": 72, "spheres": 73}[kind]
    s = _system(kind, seed)
    u_nc = O.mobility(s.axis, s.mob, s.f_ext)
    c, q, gamma = _solve(s, u_nc)
    assert c.nc >= 5
    if kind == "spheres":
        ev = np.linalg.eigvalsh(O.M_matrix(s, c).toarray())
        if ev[0] < 1e-10:
            pytest.skip("singular M: gamma is not differentiable")
    act = gamma > 0
    rng = np.random.default_rng(seed)
    weights = rng.standard_normal(c.nc)
    L1, L2, F = _losses(s, c, gamma, weights)
    dq1, dpos1, _ = O.adjoint(s, c, q, u_nc, gamma, dL_dgamma=weights)
    dq2, dpos2, _ = O.adjoint(s, c, q, u_nc, gamma, dL_dF=F)
    assert np.all(dq1[~act] == 0.0)

    # directions in q
    hq = 1e-4
    done_q = 0
    for _ in range(6):
        v = rng.standard_normal(c.nc)
        v /= np.linalg.norm(v)
        outs = []
        for sgn in (1, -1):
            _, _, gp = _solve(s, u_nc, q_override=q + sgn * hq * v)
            outs.append(_losses(s, c, gp, weights)[:2] + ((gp > 0),))
        if not (np.array_equal(outs[0][2], act) and np.array_equal(outs[1][2], act)):
            continue
        fd1 = (outs[0][0] - outs[1][0]) / (2 * hq)
        fd2 = (outs[0][1] - outs[1][1]) / (2 * hq)
        assert dq1 @ v == pytest.approx(fd1, rel=1e-5, abs=1e-7 * abs(L1))
        assert dq2 @ v == pytest.approx(fd2, rel=1e-5, abs=1e-7 * abs(L2))
        done_q += 1
    assert done_q >= 3

    # directions in the centres (orientations, forces and mobility fixed)
    hp = 1e-7
    done = 0
    for _ in range(20):
        if done >= 6:
            break
        V = rng.standard_normal((s.n, 3))
        V /= np.linalg.norm(V)
        outs = []
        ok = True
        for sgn in (1, -1):
            sp = W.Suspension(**{**s.__dict__, "pos": s.pos + sgn * hp * V})
            cp, qp, gp = _solve(sp, u_nc)
            if cp.nc != c.nc or not np.array_equal(cp.keys(), c.keys()) \
                    or not np.array_equal(gp > 0, act):
                ok = False
                break
            outs.append(_losses(sp, cp, gp, weights)[:2])
        if not ok:
            continue
        fd1 = (outs[0][0] - outs[1][0]) / (2 * hp)
        fd2 = (outs[0][1] - outs[1][1]) / (2 * hp)
        g1, g2 = float(np.sum(dpos1 * V)), float(np.sum(dpos2 * V))
        scale1 = np.linalg.norm(dpos1) + 1e-300
        scale2 = np.linalg.norm(dpos2) + 1e-300
        assert abs(g1 - fd1) <= 1e-5 * scale1
        assert abs(g2 - fd2) <= 1e-5 * scale2
        done += 1
    assert done >= 3
