"""Pins of the oracle's LCP data and its BBPGD solve (Algorithm 1).

* Two spheres head-on (closed form): M = 2 m_t, q = Phi/dt - 2U, the solution
  max(0, -q/M), and the exact Euler-updated gap |c_j - c_i + dt (U_j - U_i)|
  - 2R equals dt * g = 0: the converged force closes the gap exactly.
* Scalar LCP control flow (section 6.2): with gamma_0 = 0 and q >= 0 the
  solve stops after 1 MVOP; with q < 0 it converges in exactly 1 descent
  step (3 MVOPs).
* Independent pairs: M is diagonal and gamma_l = max(0, -q_l / M_ll).
* Brute-force active-set enumeration on small systems (an LCP with a
  P-matrix has one solution) and, on larger ones, scipy's NNLS applied to the
  equivalent least-squares problem ||L^T gamma + L^{-1} q|| with M = L L^T.
* KKT invariants on every output; symmetry and positive semidefiniteness of
  M; the SPD error bound of Eq. abserrcqp.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def _two_spheres(gap, U, R=0.5, direction=(1.0, 0.0, 0.0), dt=1e-3):
    d = np.asarray(direction, float)
    d /= np.linalg.norm(d)
    pos = np.stack([np.zeros(3), (2 * R + gap) * d]) + 5.0
    s = W.Suspension("two", pos, np.tile([0.0, 0.0, 1.0], (2, 1)),
                     np.full(2, R), np.zeros(2), W.sphere_mobility(np.full(2, R)),
                     np.zeros((2, 6)), np.full(3, 20.0), delta=0.1, dt=dt)
    u_nc = np.zeros((2, 6))
    u_nc[0, :3] = U * d
    u_nc[1, :3] = -U * d
    return s, u_nc


@pytest.mark.parametrize("direction", [(1, 0, 0), (0.3, -0.5, 0.8)])
@pytest.mark.parametrize("gap,U", [(0.02, 40.0), (-0.05, 1.0), (0.05, 3.0)])
def test_two_sphere_head_on_closed_form(direction, gap, U):
    s, u_nc = _two_spheres(gap, U, direction=direction)
    c = O.find_contacts(s)
    assert c.nc == 1
    q = O.build_q(c, u_nc, s.dt)
    mt = 1.0 / (6 * math.pi * 0.5)
    M = 2 * mt
    assert q[0] == pytest.approx(gap / s.dt - 2 * U, rel=1e-12)
    assert O.mvop(s, c, np.ones(1))[0] == pytest.approx(M, rel=1e-14)
    gamma, g, st = O.bbpgd(s, c, q)
    expect = max(0.0, -q[0] / M)
    assert gamma[0] == pytest.approx(expect, rel=1e-12, abs=1e-12)
    if expect > 0:
        assert (st.iters, st.mvops) == (1, 3)
        # exact (nonlinear) gap after the Euler step with U_nc + Mob D gamma
        u_tot = u_nc + O.mobility(s.axis, s.mob, O.D_apply(2, c, gamma))
        newpos = s.pos + s.dt * u_tot[:, :3]
        gap_new = np.linalg.norm(newpos[1] - newpos[0]) - 1.0
        assert abs(gap_new) < 1e-12
        assert gap_new == pytest.approx(s.dt * g[0], abs=1e-13)
    else:
        assert (st.iters, st.mvops) == (0, 1)


def test_independent_pairs_diagonal():
    rng = np.random.default_rng(4)
    pos, axis = [], []
    for k in range(12):
        base = np.array([4.0 * k + 2.0, 2.0, 2.0])
        p = rng.standard_normal(3); p /= np.linalg.norm(p)
        pos += [base, base + rng.uniform(-0.02, 0.02, 3)]
        axis += [p, rng.standard_normal(3)]
    axis = np.array(axis); axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    n = len(pos)
    s = W.Suspension("pairs", np.array(pos), axis, np.full(n, 0.025),
                     np.full(n, 0.5), np.tile(W.rod_mobility(), (n, 1)),
                     rng.standard_normal((n, 6)), np.array([60.0, 8.0, 8.0]),
                     delta=0.015, dt=1e-4)
    c, u_nc, q = O.setup(s)
    assert c.nc == 12 and np.all(c.i // 2 == c.j // 2)
    Mdense = O.M_matrix(s, c).toarray()
    assert np.count_nonzero(Mdense - np.diag(np.diag(Mdense))) == 0
    gamma, g, st = O.bbpgd(s, c, q, tol=1e-12)
    np.testing.assert_allclose(gamma, np.maximum(0, -q / np.diag(Mdense)),
                               rtol=1e-9, atol=1e-9)


def _enumerate_lcp(M, q):
    n = len(q)
    sols = []
    for r in range(n + 1):
        for S in itertools.combinations(range(n), r):
            S = list(S)
            gam = np.zeros(n)
            if S:
                gam[S] = np.linalg.solve(M[np.ix_(S, S)], -q[S])
            g = M @ gam + q
            if np.all(gam >= -1e-12) and np.all(g >= -1e-9 * (1 + np.abs(q).max())):
                sols.append(gam)
    return sols


def _small_cluster(seed, n=7, side=0.5):
    rng = np.random.default_rng(seed)
    s = W.rods(n, seed=seed, density=1.0)
    s.box = np.full(3, 30.0)
    s.pos = rng.uniform(0, side, (n, 3)) + 5.0
    return s


@pytest.mark.parametrize("seed", [1, 3, 4, 5, 8, 9, 12])
def test_against_active_set_enumeration(seed):
    s = _small_cluster(seed)
    c, u_nc, q = O.setup(s)
    if not (2 <= c.nc <= 13):
        pytest.skip(f"cluster has {c.nc} pairs")
    M = O.M_matrix(s, c).toarray()
    sols = _enumerate_lcp(M, q)
    assert len(sols) == 1
    gamma, g, st = O.bbpgd(s, c, q)
    assert st.status == 0
    ev = np.linalg.eigvalsh(M)
    bound = (np.linalg.norm(M, 2) + 1) / ev[0] * st.residual
    assert np.linalg.norm(gamma - sols[0]) <= bound * (1 + 1e-9) + 1e-12


def _nnls_solution(M, q):
    """min 1/2 x^T M x + q^T x over x >= 0 as NNLS: with M = L L^T this is
    min ||L^T x + L^{-1} q||^2 / 2."""
    from scipy.optimize import nnls
    L = np.linalg.cholesky(M)
    rhs = -np.linalg.solve(L, q)
    x, _ = nnls(L.T, rhs, maxiter=50 * len(q))
    return x


@pytest.mark.parametrize("make", [
    lambda: W.rods(600, seed=32),
    lambda: W.rods_and_spheres(400, 80, seed=33),
])
def test_against_nnls(make):
    s = make()
    c, u_nc, q = O.setup(s)
    M = O.M_matrix(s, c).toarray()
    ev = np.linalg.eigvalsh(M)
    assert ev[0] > 0
    ref = _nnls_solution(M, q)
    gamma, g, st = O.bbpgd(s, c, q)
    assert st.status == 0
    bound = (np.linalg.norm(M, 2) + 1) / ev[0] * st.residual
    err = np.linalg.norm(gamma - ref)
    assert err <= bound + 1e-9 * np.linalg.norm(ref)
    assert err <= 1e-6 * np.linalg.norm(ref)
    # the polished active-set solution is the NNLS solution to roundoff
    gp, gpg, passes = O.polish(s, c, q, gamma)
    assert passes > 0
    np.testing.assert_allclose(gp, ref, atol=1e-8 * np.abs(ref).max())


def test_sphere_systems_unique_force_and_gradient():
    """Randomly overlapping spheres form over-braced clusters, so M is only
    semidefinite (section 3.3.2 allows this): gamma is then not unique, but
    for a convex QP M gamma is the same at every minimiser, hence so are
    g = M gamma + q and F_c = D gamma (M d = 0 implies ||Mob^1/2 D d|| = 0)."""
    s = W.spheres(300, 0.3, seed=31)
    c, u_nc, q = O.setup(s)
    ev = np.linalg.eigvalsh(O.M_matrix(s, c).toarray())
    assert ev[0] < 1e-12 * ev[-1]             # genuinely singular
    runs = [O.bbpgd(s, c, q, bb=bb, tol=1e-10) for bb in (1, 2)]
    (g1, gg1, st1), (g2, gg2, st2) = runs
    assert st1.status == 0 and st2.status == 0
    np.testing.assert_allclose(gg1, gg2, atol=1e-7)
    F1, F2 = O.D_apply(s.n, c, g1), O.D_apply(s.n, c, g2)
    np.testing.assert_allclose(F1, F2, atol=1e-7 * np.abs(F1).max())


def _kkt(gamma, g, tol):
    assert np.all(gamma >= 0.0)
    assert np.all(g >= -tol)
    assert np.linalg.norm(np.minimum(gamma, g)) < tol
    assert np.all(np.abs(gamma * g) <= tol * np.maximum(1.0, np.maximum(gamma, np.abs(g))))


@pytest.mark.parametrize("bb", [1, 2, 3])
def test_kkt_invariants_and_bb_variants(bb):
    s = W.rods(3000, seed=41)
    c, u_nc, q = O.setup(s)
    gamma, g, st = O.bbpgd(s, c, q, bb=bb)
    assert st.status == 0 and st.mvops == st.iters + 2
    _kkt(gamma, g, s.tol)
    # the reported g is M gamma + q
    np.testing.assert_allclose(g, O.mvop(s, c, gamma) + q, rtol=0,
                               atol=1e-9 * np.abs(q).max())


def test_bb_variants_agree():
    s = W.rods_and_spheres(1200, 200, seed=42)
    c, u_nc, q = O.setup(s)
    sols = [O.bbpgd(s, c, q, bb=bb, tol=1e-9)[0] for bb in (1, 2, 3)]
    for x in sols[1:]:
        assert np.linalg.norm(x - sols[0]) <= 1e-7 * np.linalg.norm(sols[0])


def test_M_symmetric_psd_and_matches_assembled():
    s = W.rods_and_spheres(500, 100, seed=43)
    c, u_nc, q = O.setup(s)
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal((2, c.nc))
    Mx, My = O.mvop(s, c, x), O.mvop(s, c, y)
    assert x @ My == pytest.approx(y @ Mx, rel=1e-12)
    assert x @ Mx > 0
    Ms = O.M_matrix(s, c)
    np.testing.assert_allclose(Ms @ x, Mx, rtol=1e-12, atol=1e-12 * np.abs(Mx).max())
    np.testing.assert_allclose(O.M_diag(s, c), Ms.diagonal(), rtol=1e-13)


def test_degenerate_inputs():
    # no pairs at all
    s = W.spheres(20, 0.001, seed=5)
    c, u_nc, q = O.setup(s)
    assert c.nc == 0
    gamma, g, st = O.bbpgd(s, c, q)
    assert (st.status, st.iters, st.mvops) == (0, 0, 1)
    # separating pairs only: q >= 0 everywhere -> zero force after one MVOP
    s = W.spheres(300, 0.3, seed=6)
    c, u_nc, q = O.setup(s)
    qpos = np.abs(q) + 1.0
    gamma, g, st = O.bbpgd(s, c, qpos)
    assert (st.iters, st.mvops) == (0, 1) and np.all(gamma == 0.0)


def test_max_iter_reports_not_converged():
    s = W.rods(2000, seed=44)
    c, u_nc, q = O.setup(s)
    gamma, g, st = O.bbpgd(s, c, q, max_iter=3)
    assert st.status == 1 and st.iters == 3 and st.mvops == 5
    assert np.all(gamma >= 0)


def test_tolerance_tightening_costs_few_steps():
    """Section 6.4 reports that each tenfold tightening of the tolerance costs
    only a few more steps; here the dry problem needs more steps overall, so
    only monotonicity and a sublinear growth are checked."""
    s = W.workload(1)
    c, u_nc, q = O.setup(s)
    its = [O.bbpgd(s, c, q, tol=t)[2].iters for t in (1e-4, 1e-6, 1e-8)]
    assert its[0] <= its[1] <= its[2]
    assert its[2] < 4 * its[0] + 50
