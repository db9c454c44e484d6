"""Algorithm 1 with the RPY mobility in one persistent launch
(sc_solve_lcp_rpy) against the oracle's Algorithm 1 on the explicit
M = D^T Mob D, against the per-phase solve (sc_solve_lcp_mob with
sc_rpy_apply), and its edge cases: warm start at the solution, iteration
caps, no contacts, a forced barrier time-out, other grids, walls."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import oracle.hydro as OM  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _setup(s):
    import paper_1909_06623_amd as sc
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box), periodic=False, walls=s.walls, lo=tuple(s.lo))
    R = sc.RPY(P.pos, P.radius)
    u_nc = R.apply(torch.from_numpy(s.f_ext).cuda())
    con = sc.build_contacts(P, box, s.delta, u_nc, s.dt, assemble=False)
    return P, R, con


def _oracle(s):
    c = O.find_contacts(s)
    Mob = OM.rpy_dense(s.pos, s.radius)
    q_o = O.build_q(c, (Mob @ s.f_ext.ravel()).reshape(s.n, 6), s.dt)
    M = OM.contact_matrix(O.D_matrix(s.n, c), Mob)
    return c, Mob, q_o, M


@pytest.mark.parametrize("n,bb", [(300, 1), (900, 1), (900, 2), (1100, 3)])
def test_persistent_rpy_solve_matches_oracle(n, bb):
    import paper_1909_06623_amd as sc
    s = W.spheres(n, 0.3, W.SEED_BASE + 906 + n)
    s.periodic = 0
    _say(f"persistent rpy solve, {n} spheres, bb={bb}")
    P, R, con = _setup(s)
    c, Mob, q_o, M = _oracle(s)
    assert con.count == c.nc
    pm = con.canonical_order().cpu().numpy()
    # 1e-9 (|g| ~ 1e4 here): at 1e-10 BB2 on 900 spheres stalls on both GPU
    # paths, its s^T y lost in the rounding of the matrix-free product
    tol = 1e-9
    gam, g, st, f_c, u_c = sc.solve_lcp_rpy(P, con, R, tol=tol, bb=bb, want_fc=True)
    assert st["status"] == 0 and st["op"] == 4 and st["n_active"] > 30
    assert st["mvops"] == st["iters"] + 2
    go, g_o, sto = OM.bbpgd_dense(M, q_o, O.M_diag(s, c), tol=tol, bb=bb)
    assert sto.status == 0
    sc_ = max(1.0, np.abs(go).max())
    np.testing.assert_allclose(gam.cpu().numpy()[pm], go, rtol=0, atol=1e-6 * sc_)
    np.testing.assert_allclose(g.cpu().numpy()[pm], g_o, rtol=0, atol=1e-6 * sc_)
    assert float(gam.min()) >= 0.0 and float(g.min()) > -1e-9
    F_o = O.D_apply(s.n, c, go)
    np.testing.assert_allclose(f_c.cpu().numpy(), F_o, rtol=0, atol=1e-6 * np.abs(F_o).max())
    U_o = (Mob @ F_o.ravel()).reshape(s.n, 6)
    np.testing.assert_allclose(u_c.cpu().numpy(), U_o, rtol=0, atol=1e-6 * np.abs(U_o).max())
    # the per-phase solve reaches the same point; repeated launches are bitwise equal
    gm, _, stm, _, _ = sc.solve_lcp_mob(P, con, R, tol=tol, bb=bb)
    assert stm["status"] == 0
    np.testing.assert_allclose(gam.cpu().numpy(), gm.cpu().numpy(), rtol=0, atol=1e-6 * sc_)
    gam2, g2, st2, _, _ = sc.solve_lcp_rpy(P, con, R, tol=tol, bb=bb)
    assert torch.equal(gam2, gam) and torch.equal(g2, g) and st2["iters"] == st["iters"]


def test_persistent_rpy_solve_edge_cases():
    import paper_1909_06623_amd as sc
    import paper_1909_06623_amd._abi as A
    s = W.spheres(200, 0.3, W.SEED_BASE + 907)
    s.periodic = 0
    _say("persistent rpy solve edge cases")
    P, R, con = _setup(s)
    gam, g, st, _, _ = sc.solve_lcp_rpy(P, con, R, tol=1e-10)
    assert st["status"] == 0
    assert st["op"] == A.SC_OP_RPY and st["lanes_per_particle"] == 4  # threads per source's F
    # warm start at the solution: one product, no step
    gam2, g2, st2, _, _ = sc.solve_lcp_rpy(P, con, R, tol=1e-6, gamma0=gam)
    assert (st2["status"], st2["iters"], st2["mvops"]) == (0, 0, 1)
    assert torch.equal(gam2, gam)
    # max_iter = 0: not converged after the two start-up products
    _, _, st0, _, _ = sc.solve_lcp_rpy(P, con, R, tol=1e-10, max_iter=0)
    assert (st0["status"], st0["iters"], st0["mvops"]) == (A.SC_NOT_CONVERGED, 0, 2)
    _, _, st3, _, _ = sc.solve_lcp_rpy(P, con, R, tol=1e-14, max_iter=7)
    assert (st3["status"], st3["iters"], st3["mvops"]) == (A.SC_NOT_CONVERGED, 7, 9)
    with pytest.raises(sc.ScError):
        sc.solve_lcp_rpy(P, con, R, tol=1e-14, max_iter=7, raise_on_nonconverged=True)
    # a barrier wait capped at one poll: the time-out is reported and the
    # next solve is unaffected
    _, _, stt, _, _ = sc.solve_lcp_rpy(P, con, R, tol=1e-10, spin_limit=1)
    assert stt["status"] == A.SC_ERR_TIMEOUT
    gam6, _, st6, _, _ = sc.solve_lcp_rpy(P, con, R, tol=1e-10)
    assert torch.equal(gam6, gam) and st6["iters"] == st["iters"]
    # other grids: the same point within the tolerance
    for grid in (8, 24, 64):
        gg, _, stg, _, _ = sc.solve_lcp_rpy(P, con, R, tol=1e-10, grid=grid)
        assert stg["status"] == 0 and stg["grid"] == grid
        np.testing.assert_allclose(gg.cpu().numpy(), gam.cpu().numpy(), rtol=0,
                                   atol=1e-6 * max(1.0, float(gam.abs().max())))
    # bad arguments are rejected before any device work
    with pytest.raises(sc.ScError):
        sc.solve_lcp_rpy(P, con, R, tol=0.0)
    with pytest.raises(sc.ScError):
        sc.solve_lcp_rpy(P, con, R, bb=4)
    # no contacts
    far = W.Suspension("far", np.array([[0.0, 0, 0], [5.0, 0, 0]]), np.tile([0, 0, 1.0], (2, 1)),
                       np.full(2, 0.5), np.zeros(2), W.sphere_mobility(np.full(2, 0.5)),
                       np.ones((2, 6)), np.full(3, 10.0), 0.1, 0.01, 1e-6, periodic=0)
    P2, R2, con2 = _setup(far)
    assert con2.count == 0
    _, _, st7, f7, u7 = sc.solve_lcp_rpy(P2, con2, R2, want_fc=True)
    assert st7["status"] == 0 and float(f7.abs().max()) == 0.0 and float(u7.abs().max()) == 0.0


def test_persistent_rpy_solve_with_walls_matches_oracle():
    import paper_1909_06623_amd as sc
    rng = np.random.default_rng(21)
    n = 120
    pos = np.column_stack([rng.uniform(0.6, 7.4, n), rng.uniform(0.6, 7.4, n),
                           rng.uniform(0.45, 1.6, n)])
    rad = np.full(n, 0.5)
    f = np.zeros((n, 6))
    f[:, 2] = -5.0
    f[:, :3] += rng.standard_normal((n, 3))
    s = W.Suspension("floor_rpy", pos, np.tile([0.0, 0.0, 1.0], (n, 1)), rad, np.zeros(n),
                     W.sphere_mobility(rad), f, np.full(3, 8.0), 0.1, 0.01, 1e-10, periodic=0,
                     walls=63)
    _say("persistent rpy solve with walls")
    P, R, con = _setup(s)
    c, Mob, q_o, M = _oracle(s)
    assert con.count == c.nc and np.count_nonzero(c.j < 0) >= 10
    gam, g, st, f_c, _ = sc.solve_lcp_rpy(P, con, R, tol=1e-10, want_fc=True)
    assert st["status"] == 0
    go, _, sto = OM.bbpgd_dense(M, q_o, O.M_diag(s, c), tol=1e-10)
    pm = con.canonical_order().cpu().numpy()
    np.testing.assert_allclose(gam.cpu().numpy()[pm], go, rtol=0,
                               atol=1e-6 * max(1.0, np.abs(go).max()))
    F_o = O.D_apply(n, c, go)
    np.testing.assert_allclose(f_c.cpu().numpy(), F_o, rtol=0, atol=1e-6 * np.abs(F_o).max())


@pytest.mark.parametrize("n", [4000, 20000])
def test_persistent_rpy_solve_with_multi_tile_units_properties(n):
    """Sizes whose pair units span several 256-source LDS tiles (the tile
    prefetch path), too large for the oracle's dense M: KKT, the per-phase
    solve's point, F_c = D gamma against the oracle's D on the oracle's
    contact list, and sampled rows of U_c against the oracle's pair formula."""
    import math
    import paper_1909_06623_amd as sc
    s = W.spheres(n, 0.3, W.SEED_BASE + 909)
    s.periodic = 0
    _say(f"persistent rpy solve, {n} spheres, properties")
    P, R, con = _setup(s)
    tol = 1e-6
    gam, g, st, f_c, u_c = sc.solve_lcp_rpy(P, con, R, tol=tol, want_fc=True)
    assert st["status"] == 0 and st["n_active"] > n // 2
    ga, gg = gam.cpu().numpy(), g.cpu().numpy()
    assert ga.min() >= 0.0 and gg.min() > -tol
    assert np.linalg.norm(np.minimum(ga, gg)) < tol
    gm, _, stm, _, _ = sc.solve_lcp_mob(P, con, R, tol=tol)
    assert stm["status"] == 0
    np.testing.assert_allclose(ga, gm.cpu().numpy(), rtol=0,
                               atol=1e-5 * max(1.0, np.abs(ga).max()))
    c = O.find_contacts(s)
    assert con.count == c.nc
    pm = con.canonical_order().cpu().numpy()
    F_o = O.D_apply(s.n, c, ga[pm])
    np.testing.assert_allclose(f_c.cpu().numpy(), F_o, rtol=0, atol=1e-12 * np.abs(F_o).max())
    rows = np.random.default_rng(17).choice(s.n, 3, replace=False)
    Fc = f_c.cpu().numpy()
    for r in rows:
        acc = Fc[r, :3] / (6.0 * math.pi * s.radius[r])
        for j in range(s.n):
            if j != r:
                acc = acc + OM.rpy_block(s.pos[r] - s.pos[j], s.radius[r], s.radius[j],
                                         1.0) @ Fc[j, :3]
        np.testing.assert_allclose(u_c.cpu().numpy()[r, :3], acc, rtol=0,
                                   atol=1e-11 * max(1.0, np.abs(acc).max()))
