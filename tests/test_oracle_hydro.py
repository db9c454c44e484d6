"""Pins of the oracle's general-mobility pieces (oracle/hydro.py): the RPY
tensor against the equal-radius Rotne-Prager closed form, its branch
continuity, far field and positive definiteness, two-sphere closed forms
for sedimentation and for a head-on collision resolved through the RPY
mobility, Algorithm 1 on an explicit M against the C oracle and against
brute-force active sets, and the sedimenting cluster of section 6.3 against
the point-force estimate of a uniform cloud."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
import oracle.hydro as OM
import oracle.timestep as T
import workloads as W


def _rotne_prager(d, a, mu=1.0):
    """Rotne and Prager (1969), equal radii: the non-overlapping form and
    the overlapping form of the regularised tensor."""
    r = np.linalg.norm(d)
    e = d / r
    if r >= 2.0 * a:
        return (1.0 / (8.0 * math.pi * mu * r)) * (
            (1.0 + 2.0 * a * a / (3.0 * r * r)) * np.eye(3)
            + (1.0 - 2.0 * a * a / (r * r)) * np.outer(e, e))
    return (1.0 / (6.0 * math.pi * mu * a)) * (
        (1.0 - 9.0 * r / (32.0 * a)) * np.eye(3) + (3.0 * r / (32.0 * a)) * np.outer(e, e))


def test_equal_radii_reduce_to_rotne_prager():
    rng = np.random.default_rng(1)
    for _ in range(200):
        a = rng.uniform(0.2, 2.0)
        d = rng.standard_normal(3)
        d *= rng.uniform(0.05, 6.0) * a / np.linalg.norm(d)
        mu = rng.uniform(0.5, 3.0)
        np.testing.assert_allclose(OM.rpy_block(d, a, a, mu), _rotne_prager(d, a, mu),
                                   rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("ai,aj", [(0.5, 0.5), (0.3, 0.8), (1.0, 0.25)])
def test_branches_are_continuous(ai, aj):
    e = np.array([0.3, -0.5, 0.81])
    e /= np.linalg.norm(e)
    for r0 in (ai + aj, abs(ai - aj)):
        if r0 == 0.0:
            continue
        lo = OM.rpy_block((r0 * (1 - 1e-9)) * e, ai, aj)
        hi = OM.rpy_block((r0 * (1 + 1e-9)) * e, ai, aj)
        np.testing.assert_allclose(lo, hi, rtol=0, atol=1e-8 / (ai * aj))


def test_far_field_is_oseen():
    e = np.array([1.0, 2.0, -2.0]) / 3.0
    for r in (1e4, 1e6):
        M = OM.rpy_block(r * e, 0.4, 0.9, mu=2.0)
        oseen = (np.eye(3) + np.outer(e, e)) / (8.0 * math.pi * 2.0 * r)
        np.testing.assert_allclose(M, oseen, rtol=2e-8 * (1e4 / r) ** 2 * 10, atol=0)


def test_positive_definite_with_overlaps_and_containment():
    rng = np.random.default_rng(7)
    for trial in range(5):
        n = 60
        pos = rng.uniform(0.0, 3.0, (n, 3))
        rad = rng.uniform(0.2, 0.9, n)
        pos[1] = pos[0] + [0.01, 0.0, 0.0]      # one sphere nearly inside another
        rad[0], rad[1] = 0.9, 0.2
        pos[3] = pos[2]                           # a small sphere at a larger one's centre
        rad[2], rad[3] = 0.8, 0.3
        Mob = OM.rpy_mobility(pos, rad)
        assert np.abs(Mob - Mob.T).max() < 1e-15
        ev = np.linalg.eigvalsh(Mob)
        assert ev[0] > 0.0, (trial, ev[0])
        np.testing.assert_allclose(OM.rpy_dense(pos, rad), Mob, rtol=0, atol=1e-15)
        F = rng.standard_normal((n, 6))
        np.testing.assert_allclose(OM.rpy_apply(pos, rad, F),
                                   (Mob @ F.ravel()).reshape(n, 6), rtol=0, atol=1e-13)


def test_two_sphere_sedimentation_closed_forms():
    """Two equal spheres under the same force: along their line of centres
    U = F/(6 pi mu a) (1 + 3a/(2r) - a^3/r^3), across it
    U = F/(6 pi mu a) (1 + 3a/(4r) + a^3/(2r^3)) (the RPY far-field results)."""
    a, r, mu = 0.7, 3.1, 1.3
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, r]])
    u0 = 1.0 / (6.0 * math.pi * mu * a)
    for axis, fac in ((2, 1 + 1.5 * a / r - a ** 3 / r ** 3),
                      (0, 1 + 0.75 * a / r + 0.5 * a ** 3 / r ** 3)):
        F = np.zeros((2, 6))
        F[:, axis] = 1.0
        U = OM.rpy_apply(pos, np.full(2, a), F, mu)
        np.testing.assert_allclose(U[:, axis], u0 * fac, rtol=1e-13)
        U[:, axis] = 0.0
        assert np.abs(U).max() < 1e-15


def test_head_on_collision_through_rpy():
    """Two equal spheres pushed together along their line of centres: the
    scalar LCP has M = n^T (2 Mob_self - 2 Mob_ij) n and the converged
    solution closes the gap exactly (Phi is linear along the line)."""
    a, gap, F, dt = 0.5, 0.03, 20.0, 0.1
    r = 2 * a + gap
    pos = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
    f = np.zeros((2, 6))
    f[0, 0], f[1, 0] = F, -F
    s = W.Suspension("pair", pos, np.tile([0.0, 0.0, 1.0], (2, 1)), np.full(2, a), np.zeros(2),
                     W.sphere_mobility(np.full(2, a)), f, np.full(3, 10.0), 0.1, dt, 1e-13,
                     periodic=0)
    quat = T.quat_from_axis(s.axis)
    s1, _, rec = T.step(s, quat, None, hydro="rpy")
    assert rec.i.size == 1 and rec.status == 0
    m_rel = 2.0 / (6.0 * math.pi * a) - 2.0 * (1.0 / (4.0 * math.pi * r)) * (1.0 - 2 * a * a / (3 * r * r))
    gamma = F - gap / (dt * m_rel)
    assert gamma > 0.0
    assert rec.gamma[0] == pytest.approx(gamma, rel=1e-10)
    assert s1.pos[1, 0] - s1.pos[0, 0] == pytest.approx(2 * a, abs=1e-12)


def test_bbpgd_dense_equals_c_oracle_on_the_dry_mobility():
    s = W.spheres(150, 0.3, W.SEED_BASE + 903)
    c, u, q = O.setup(s)
    M = O.M_matrix(s, c).toarray()
    d = O.M_diag(s, c)
    for bb in (1, 2, 3):
        gc, g_c, stc = O.bbpgd(s, c, q, tol=1e-10, bb=bb)
        gd, g_d, std = OM.bbpgd_dense(M, q, d, tol=1e-10, bb=bb)
        assert std.status == 0 and stc.status == 0
        assert abs(std.iters - stc.iters) <= max(3, stc.iters // 10), (bb, std.iters, stc.iters)
        np.testing.assert_allclose(gd, gc, rtol=0, atol=1e-7 * max(1.0, np.abs(gc).max()))


def test_bbpgd_dense_degenerate_and_limits():
    # g0 in the null space of M: the fallback step 1 / max diag
    M = np.array([[1.0, -1.0], [-1.0, 1.0]])
    q = np.array([-1.0, -1.0])
    g, gg, st = OM.bbpgd_dense(M, q, np.diag(M), tol=1e-12, max_iter=50)
    assert st.n_degenerate >= 1 and st.alpha > 0
    # max_iter = 0 reports not converged after the two start-up products
    _, _, st0 = OM.bbpgd_dense(np.eye(3), -np.ones(3), np.ones(3), tol=1e-12, max_iter=0)
    assert (st0.status, st0.iters, st0.mvops) == (1, 0, 2)
    # gamma0 already optimal: one product, no step
    _, _, st1 = OM.bbpgd_dense(np.eye(3), -np.ones(3), np.ones(3), gamma0=np.ones(3), tol=1e-12)
    assert (st1.status, st1.iters, st1.mvops) == (0, 0, 1)


def _brute_force_lcp(M, q):
    n = q.size
    for k in range(n + 1):
        for act in itertools.combinations(range(n), k):
            act = list(act)
            gam = np.zeros(n)
            if act:
                gam[act] = np.linalg.solve(M[np.ix_(act, act)], -q[act])
            g = M @ gam + q
            if (gam >= -1e-12).all() and (g >= -1e-12).all():
                return gam
    raise AssertionError("no complementary solution")


def test_rpy_lcp_against_brute_force_active_sets():
    rng = np.random.default_rng(11)
    done = 0
    for trial in range(40):
        n = 6
        pos = rng.uniform(0.0, 1.6, (n, 3))
        rad = np.full(n, 0.35)
        f = rng.standard_normal((n, 6))
        s = W.Suspension("tiny", pos, np.tile([0.0, 0.0, 1.0], (n, 1)), rad, np.zeros(n),
                         W.sphere_mobility(rad), f, np.full(3, 4.0), 0.1, 0.01, 1e-12, periodic=0)
        c = O.find_contacts(s)
        if not 2 <= c.nc <= 10:
            continue
        Mob = OM.rpy_dense(s.pos, rad)
        M = OM.contact_matrix(O.D_matrix(n, c), Mob)
        if np.linalg.eigvalsh(M)[0] < 1e-8:
            continue
        u_nc = (Mob @ f.ravel()).reshape(n, 6)
        q = O.build_q(c, u_nc, s.dt)
        gam, g, st = OM.bbpgd_dense(M, q, O.M_diag(s, c), tol=1e-12)
        assert st.status == 0
        ref = _brute_force_lcp(M, q)
        np.testing.assert_allclose(gam, ref, rtol=0, atol=1e-8 * max(1.0, np.abs(ref).max()))
        done += 1
    assert done >= 10


def test_rpy_solve_kkt_on_overlapping_spheres():
    s = W.spheres(300, 0.3, W.SEED_BASE + 904)
    s.periodic = 0
    c = O.find_contacts(s)
    Mob = OM.rpy_dense(s.pos, s.radius)
    u_nc = (Mob @ s.f_ext.ravel()).reshape(s.n, 6)
    q = O.build_q(c, u_nc, s.dt)
    M = OM.contact_matrix(O.D_matrix(s.n, c), Mob)
    assert np.abs(M - M.T).max() < 1e-12 * np.abs(M).max()
    gam, g, st = OM.bbpgd_dense(M, q, O.M_diag(s, c), tol=1e-9)
    assert st.status == 0 and st.n_active > 50
    assert gam.min() >= 0.0 and g.min() > -1e-9
    assert abs(gam @ g) < 1e-6 * max(1.0, np.abs(gam).max())


def test_cluster_sediments_like_a_point_force_cloud():
    """The section 6.3 cluster: 1000 spheres, hydrodynamic volume fraction
    0.2, equal forces. Spheres in a crowd fall faster than alone; for point
    forces spread uniformly over a ball of radius R the mean velocity is
    F/(6 pi mu a) + (N - 1) F / (5 pi mu R) (the mean of (1 + cos^2)/r over
    two uniform points of a ball is 8/(5R)); the RPY corrections and the
    collision-free margin keep the cluster within a few percent of it."""
    s = W.sphere_cluster(1000, W.SEED_BASE + 900)
    quat = T.quat_from_axis(s.axis)
    _, _, rec = T.step(s, quat, None, hydro="rpy")
    assert rec.status == 0
    R = float(np.max(np.linalg.norm(s.pos, axis=1)))
    est = 1.0 / (6.0 * math.pi) + (s.n - 1) / (5.0 * math.pi * R)
    uz = -rec.U[:, 2]
    assert uz.min() > 1.0 / (6.0 * math.pi)
    assert abs(uz.mean() / est - 1.0) < 0.08, (uz.mean(), est)
    # the core falls faster than the surface
    rr = np.linalg.norm(s.pos, axis=1)
    assert uz[rr < 0.5 * R].mean() > uz[rr > 0.8 * R].mean()


def test_rpy_gradient_against_central_differences():
    rng = np.random.default_rng(3)
    for trial in range(3):
        n = 12
        pos = rng.uniform(0.0, 2.0, (n, 3))
        rad = rng.uniform(0.2, 0.6, n)
        if trial == 2:
            pos[1] = pos[0] + [0.05, 0.02, 0.0]      # one sphere inside another
            rad[0], rad[1] = 0.6, 0.2
        a = rng.standard_normal((n, 6))
        f = rng.standard_normal((n, 6))
        g = OM.rpy_grad(pos, rad, a, f, 1.3)
        h = 1e-6
        fd = np.zeros((n, 3))
        for k in range(n):
            for c in range(3):
                pp, pm = pos.copy(), pos.copy()
                pp[k, c] += h
                pm[k, c] -= h
                fd[k, c] = (a.ravel() @ OM.rpy_dense(pp, rad, 1.3) @ f.ravel()
                            - a.ravel() @ OM.rpy_dense(pm, rad, 1.3) @ f.ravel()) / (2 * h)
        np.testing.assert_allclose(g, fd, rtol=0, atol=1e-7 * np.abs(g).max())


def _rpy_solve(s):
    c = O.find_contacts(s)
    Mob = OM.rpy_dense(s.pos, s.radius)
    u_nc = (Mob @ s.f_ext.ravel()).reshape(s.n, 6)
    q = O.build_q(c, u_nc, s.dt)
    M = OM.contact_matrix(O.D_matrix(s.n, c), Mob)
    g, _, st = OM.bbpgd_dense(M, q, O.M_diag(s, c), tol=1e-11)
    gp, _, passes = OM.polish_dense(M, q, g)
    assert passes > 0
    return c, gp


@pytest.mark.parametrize("loss", ["force", "linear"])
def test_rpy_adjoint_against_central_differences(loss):
    """dL/dc from adjoint_rpy against central differences of polished RPY
    solves (contacts, U_nc = Mob(c) F_ext, q and M all rebuilt), for
    L = 1/2 ||D gamma||^2 and L = wts . gamma."""
    s = W.spheres(40, 0.35, W.SEED_BASE + 911)
    s.periodic = 0
    s.dt = 0.01
    rng = np.random.default_rng(12)
    c, gam = _rpy_solve(s)
    act = gam > 0.0
    assert act.sum() >= 5
    wts = rng.standard_normal(c.nc)
    if loss == "force":
        F = O.D_apply(s.n, c, gam)
        _, dpos, _ = OM.adjoint_rpy(s, c, gam, dL_dF=F)
    else:
        _, dpos, _ = OM.adjoint_rpy(s, c, gam, dL_dgamma=wts)
    hp = 1e-7
    done = 0
    for _ in range(20):
        if done >= 4:
            break
        V = rng.standard_normal((s.n, 3))
        V /= np.linalg.norm(V)
        L = []
        for sg in (1, -1):
            sp = W.Suspension(**{**s.__dict__, "pos": s.pos + sg * hp * V})
            cp, gp = _rpy_solve(sp)
            if not np.array_equal(cp.keys(), c.keys()) or not np.array_equal(gp > 0, act):
                break
            if loss == "force":
                Fp = O.D_apply(s.n, cp, gp)
                L.append(0.5 * float(np.sum(Fp * Fp)))
            else:
                L.append(float(wts @ gp))
        if len(L) < 2:
            continue
        fd = (L[0] - L[1]) / (2 * hp)
        assert abs(float(np.sum(dpos * V)) - fd) <= 1e-5 * np.linalg.norm(dpos), (fd, np.sum(dpos * V))
        done += 1
    assert done >= 3


def test_rpy_adjoint_is_translation_invariant():
    """In unbounded fluid the loss depends on relative positions only, so
    the centre gradient sums to zero (a sign slip between the two ends of a
    pair term, in the contacts or in the mobility's gradient, breaks it)."""
    s = W.spheres(60, 0.35, W.SEED_BASE + 912)
    s.periodic = 0
    s.dt = 0.01
    c, gam = _rpy_solve(s)
    assert (gam > 0).sum() >= 5
    for kw in ({"dL_dF": O.D_apply(s.n, c, gam)},
               {"dL_dgamma": np.random.default_rng(4).standard_normal(c.nc)}):
        _, dpos, _ = OM.adjoint_rpy(s, c, gam, **kw)
        assert np.abs(dpos.sum(axis=0)).max() < 1e-10 * np.abs(dpos).max()
        g = OM.rpy_grad(s.pos, s.radius, O.D_apply(s.n, c, gam), s.f_ext)
        assert np.abs(g.sum(axis=0)).max() < 1e-11 * np.abs(g).max()
