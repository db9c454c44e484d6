"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

The library lists contacts in solver order (cell-ranked); the oracle in the
plain enumeration order (by i, then j). Both are deterministic; comparisons go
through the permutation that sorts the library's pairs by (i, j).

Bars:
* contact lists: bit-exact equality of the sets of pairs (index work), and a
  run-to-run identical order; frames, Phi and q equal to rounding (the two
  sides evaluate the same closed forms in possibly different operation
  orders);
* one product M x and a fixed number of BBPGD steps: relative 1e-12 / 1e-9;
* converged solves: the tolerance of the workload (||min(gamma, g)|| < tol),
  relative gamma error <= 1e-6 where M is SPD (checked at a tight tolerance
  when the SPD error bound of Eq. abserrcqp at the workload tolerance is
  looser than that), and the unique quantities g and D gamma where it is
  only semidefinite (randomly overlapping spheres);
* bitwise reproducibility run to run.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _sc():
    import paper_1909_06623_amd as sc
    return sc


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _setup_gpu(s, capacity=None):
    sc = _sc()
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box), lo=tuple(s.lo), periodic=bool(s.periodic))
    u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
    con = sc.build_contacts(P, box, s.delta, u_nc, s.dt, capacity=capacity)
    return P, box, u_nc, con


def _perm(con):
    """Library index of each contact in the oracle's (i, j) order."""
    return con.canonical_order().cpu().numpy()


def _contacts_equal(con, c):
    assert con.count == c.nc
    assert con.n_borderline == 0
    pm = _perm(con)
    np.testing.assert_array_equal(con.i.cpu().numpy()[pm], c.i)
    np.testing.assert_array_equal(con.j.cpu().numpy()[pm], c.j)
    phi = con.phi[: con.count].cpu().numpy()[pm]
    np.testing.assert_allclose(phi, c.phi, rtol=0, atol=1e-13)
    np.testing.assert_allclose(con.nrm.cpu().numpy()[pm], c.nrm, rtol=0, atol=1e-12)
    np.testing.assert_allclose(con.tau_i.cpu().numpy()[pm], c.tau_i, rtol=0, atol=1e-12)
    np.testing.assert_allclose(con.tau_j.cpu().numpy()[pm], c.tau_j, rtol=0, atol=1e-12)
    return pm


CASES = {
    "spheres1000": lambda: W.workload(1),
    "rods5000": lambda: W.rods(5000, seed=W.SEED_BASE + 2),
    "mixed": lambda: W.rods_and_spheres(3000, 600, seed=W.SEED_BASE + 3),
    "rods_small_box": lambda: W.rods(600, seed=17, min_side=2.2),
    "spheres_dense": lambda: W.spheres(700, 0.4, seed=18),
}


@pytest.mark.parametrize("name", list(CASES))
def test_contacts_and_q(name):
    s = CASES[name]()
    _say(f"contacts {name} N={s.n}")
    P, box, u_nc, con = _setup_gpu(s)
    c, u_orc, q_orc = O.setup(s)
    np.testing.assert_allclose(u_nc.cpu().numpy(), u_orc, rtol=1e-14, atol=1e-15)
    pm = _contacts_equal(con, c)
    q = con.q[: con.count].cpu().numpy()[pm]
    np.testing.assert_allclose(q, q_orc, rtol=1e-12, atol=1e-9)
    # the solver order is a pure function of the inputs
    sc = _sc()
    con2 = sc.build_contacts(P, box, s.delta, u_nc, s.dt)
    assert torch.equal(con2.i, con.i) and torch.equal(con2.j, con.j)
    assert torch.equal(con2.q[: con.count], con.q[: con.count])


def test_non_periodic_contacts():
    s = W.rods_and_spheres(1500, 300, seed=23)
    s.periodic = 0
    s.pos = s.pos * 1.2 - 1.0
    _say("contacts non-periodic")
    P, box, u_nc, con = _setup_gpu(s)
    c, u_orc, q_orc = O.setup(s)
    _contacts_equal(con, c)


@pytest.mark.parametrize("name", ["spheres1000", "mixed"])
def test_mvop(name):
    s = CASES[name]()
    _say(f"mvop {name}")
    sc = _sc()
    P, box, u_nc, con = _setup_gpu(s)
    c, u_orc, q_orc = O.setup(s)
    pm = _perm(con)
    x = np.random.default_rng(5).standard_normal(c.nc)      # oracle order
    xg = np.empty_like(x)
    xg[pm] = x                                               # library order
    y = sc.mvop(P, con, torch.from_numpy(xg).cuda()).cpu().numpy()[pm]
    ref = O.mvop(s, c, x)
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


OPS = {"chain": 1, "matrix": 2}


@pytest.mark.parametrize("op", list(OPS))
@pytest.mark.parametrize("bb", [1, 2, 3])
def test_fixed_steps_match(bb, op):
    s = W.rods(3000, seed=31)
    _say(f"fixed steps bb={bb} op={op}")
    sc = _sc()
    P, box, u_nc, con = _setup_gpu(s)
    c, u_orc, q_orc = O.setup(s)
    pm = _perm(con)
    gam, g, st, _, _ = sc.solve_lcp(P, con, tol=s.tol, max_iter=6, bb=bb, op=OPS[op])
    assert st["op"] == OPS[op]
    go, gg, sto = O.bbpgd(s, c, q_orc, max_iter=6, bb=bb)
    assert st["status"] == 1 and sto.status == 1
    assert (st["iters"], st["mvops"]) == (6, 8)
    np.testing.assert_allclose(gam.cpu().numpy()[pm], go, rtol=1e-9,
                               atol=1e-9 * np.abs(go).max())
    np.testing.assert_allclose(g.cpu().numpy()[pm], gg, rtol=1e-9, atol=1e-9 * np.abs(gg).max())
    assert st["alpha"] == pytest.approx(sto.alpha, rel=1e-9)


def _kkt(gam, g, tol):
    assert np.all(gam >= 0.0)
    assert np.linalg.norm(np.minimum(gam, g)) < tol
    assert np.all(g >= -tol)
    assert np.all(np.abs(gam * g) <= tol * np.maximum(1.0, np.maximum(gam, np.abs(g))))


_EIG = {}   # extreme eigenvalues of M per case, shared by the two products


@pytest.mark.parametrize("op", list(OPS))
@pytest.mark.parametrize("name", ["rods5000", "mixed", "rods_small_box"])
def test_converged_solve_spd(name, op):
    s = CASES[name]()
    _say(f"solve {name} op={op}")
    sc = _sc()
    P, box, u_nc, con = _setup_gpu(s)
    c, u_orc, q_orc = O.setup(s)
    pm = _perm(con)
    gam, g, st, f_c, u_c = sc.solve_lcp(P, con, tol=s.tol, want_fc=True, op=OPS[op])
    assert st["status"] == 0
    gam, g = gam.cpu().numpy()[pm], g.cpu().numpy()[pm]
    _kkt(gam, g, s.tol)
    assert st["residual"] == pytest.approx(np.linalg.norm(np.minimum(gam, g)), rel=1e-6)
    # outputs are consistent: g = M gamma + q, f_c = D gamma, u_c = Mob f_c
    np.testing.assert_allclose(g, O.mvop(s, c, gam) + q_orc, rtol=0,
                               atol=1e-9 * np.abs(q_orc).max())
    F = O.D_apply(s.n, c, gam)
    np.testing.assert_allclose(f_c.cpu().numpy(), F, rtol=0, atol=1e-11 * np.abs(F).max())
    np.testing.assert_allclose(u_c.cpu().numpy(), O.mobility(s.axis, s.mob, F), rtol=0,
                               atol=1e-11 * np.abs(F).max())
    # against the exact LCP solution (the oracle's iterate, polished): any
    # iterate meeting the tolerance lies within Eq. abserrcqp's bound
    # 2 (||M|| + 1) / lambda_min * tol of it, computed here from M's extreme
    # eigenvalues, and the solve must also meet the 1e-6 relative bar (the
    # bound alone allows 3e-5 to 4e-3 on these systems)
    import scipy.sparse.linalg as spla
    go, gg, sto = O.bbpgd(s, c, q_orc)
    assert sto.status == 0
    gp, _, passes = O.polish(s, c, q_orc, go)
    assert passes >= 1
    if name not in _EIG:
        M = O.M_matrix(s, c)
        _EIG[name] = (float(spla.eigsh(M, k=1, which="LA", return_eigenvectors=False)[0]),
                      float(spla.eigsh(M, k=1, sigma=0.0, which="LM",
                                       return_eigenvectors=False)[0]))
    lmax, lmin = _EIG[name]
    bound = 2.0 * (lmax + 1.0) / lmin * s.tol
    err = np.linalg.norm(gam - gp)
    rel = err / np.linalg.norm(gp)
    # and at a tight tolerance
    gt, _, stt, _, _ = sc.solve_lcp(P, con, tol=1e-9, op=OPS[op])
    assert stt["status"] == 0
    rel_t = np.linalg.norm(gt.cpu().numpy()[pm] - gp) / np.linalg.norm(gp)
    print(f"[result] {name}: iters gpu {st['iters']} oracle {sto.iters}; lambda in "
          f"[{lmin:.2e}, {lmax:.2e}], bound {bound:.2e} (rel {bound / np.linalg.norm(gp):.2e}); "
          f"rel err tol1e-6 {rel:.2e} tol1e-9 {rel_t:.2e}", flush=True)
    assert err <= bound
    assert rel <= 1e-6
    assert rel_t <= 1e-6


@pytest.mark.parametrize("op", list(OPS))
def test_converged_solve_semidefinite_spheres(op):
    s = W.workload(1)
    _say(f"solve spheres1000 (semidefinite M) op={op}")
    sc = _sc()
    P, box, u_nc, con = _setup_gpu(s)
    c, u_orc, q_orc = O.setup(s)
    pm = _perm(con)
    gam, g, st, f_c, u_c = sc.solve_lcp(P, con, tol=1e-9, want_fc=True, op=OPS[op])
    go, gg, sto = O.bbpgd(s, c, q_orc, tol=1e-9)
    assert st["status"] == 0 and sto.status == 0
    gam, g = gam.cpu().numpy()[pm], g.cpu().numpy()[pm]
    _kkt(gam, g, 1e-9)
    np.testing.assert_allclose(g, gg, atol=1e-7)
    F = O.D_apply(s.n, c, go)
    np.testing.assert_allclose(f_c.cpu().numpy(), F, atol=1e-7 * np.abs(F).max())


@pytest.mark.parametrize("op", list(OPS))
def test_bitwise_reproducible(op):
    s = W.rods(4000, seed=44)
    _say(f"reproducibility op={op}")
    sc = _sc()
    P, box, u_nc, con = _setup_gpu(s)
    a = sc.solve_lcp(P, con, tol=s.tol, op=OPS[op])
    b = sc.solve_lcp(P, con, tol=s.tol, op=OPS[op])
    assert a[2]["iters"] == b[2]["iters"]
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_chain_lds_share_changes_nothing():
    """The matrix-free chain keeps each workgroup's incidence ranges, codes
    and D columns in LDS, up to a capacity; past it they are read from global
    memory, and with lds_entries_per_wave = -1 all of them are. The
    arithmetic and its order are the same either way, so iterates, step sizes
    and residuals are bitwise equal for every share, and a few fixed steps
    meet the oracle's."""
    s = W.rods(3000, seed=31)
    _say("chain LDS shares")
    sc = _sc()
    P, box, u_nc, con = _setup_gpu(s)
    c, u_orc, q_orc = O.setup(s)
    pm = _perm(con)
    go, gg, sto = O.bbpgd(s, c, q_orc, max_iter=8)
    ref = None
    for grid, cache in ((0, 0), (0, -1), (0, 3), (0, 17), (40, 0), (40, 5), (40, -1)):
        gam, g, st, _, _ = sc.solve_lcp(P, con, max_iter=8, op=1, grid=grid,
                                        lds_entries_per_wave=cache)
        assert st["op"] == 1 and st["iters"] == 8
        if cache > 0:
            assert st["lds_entries_per_wave"] == cache
        elif cache < 0:
            assert st["lds_entries_per_wave"] == 0
        else:
            assert st["lds_entries_per_wave"] > 0
        np.testing.assert_allclose(gam.cpu().numpy()[pm], go, rtol=1e-9,
                                   atol=1e-9 * np.abs(go).max())
        key = (st["grid"], st["lanes_per_particle"])
        if ref is None or ref[0] != key:
            ref = (key, gam.clone(), g.clone(), st["alpha"], st["residual"])
        else:
            assert torch.equal(gam, ref[1]) and torch.equal(g, ref[2]), (grid, cache)
            assert (st["alpha"], st["residual"]) == (ref[3], ref[4]), (grid, cache)


def test_chain_rank_ranges_past_lds():
    """On one workgroup, 40,000 rods have more incidence ranges than LDS
    holds: the chain reads the ranges from global memory and still keeps as
    many incidences as fit in LDS. Iterates are bitwise those without any
    LDS copy, and a few fixed steps meet the oracle's."""
    s = W.rods(40000, seed=32)
    _say("chain: ranges past LDS (one workgroup, 40,000 rods)")
    sc = _sc()
    P, box, u_nc, con = _setup_gpu(s)
    c, u_orc, q_orc = O.setup(s)
    pm = _perm(con)
    go, gg, sto = O.bbpgd(s, c, q_orc, max_iter=4)
    a = sc.solve_lcp(P, con, max_iter=4, op=1, grid=1)
    b = sc.solve_lcp(P, con, max_iter=4, op=1, grid=1, lds_entries_per_wave=-1)
    assert a[2]["grid"] == 1 and a[2]["lds_entries_per_wave"] > 0
    assert b[2]["lds_entries_per_wave"] == 0
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    np.testing.assert_allclose(a[0].cpu().numpy()[pm], go, rtol=1e-9,
                               atol=1e-9 * np.abs(go).max())


@pytest.mark.parametrize("spw", [1, 2, 4])
def test_matrix_launch_shapes_agree(spw):
    """Every launch shape of the one-pass solve runs the same algorithm: a
    few fixed steps agree with the oracle, M's nonzero count is
    sum_k deg(k)^2 - n_c, and the product M gamma_0 + q (a solve with no
    descent step) is bitwise the same for every shape, since each row is
    summed in storage order by one lane."""
    s = W.rods_and_spheres(2500, 500, seed=45)
    _say(f"matrix slices_per_wave={spw}")
    sc = _sc()
    P, box, u_nc, con = _setup_gpu(s)
    c, u_orc, q_orc = O.setup(s)
    deg = np.bincount(c.i, minlength=s.n) + np.bincount(c.j, minlength=s.n)
    assert con.nnz == int(np.sum(deg.astype(np.int64) ** 2)) - c.nc
    assert con.count % 64 != 0  # a ragged last slice
    pm = _perm(con)
    go, gg, sto = O.bbpgd(s, c, q_orc, max_iter=5)
    for block, grid, cache in ((256, 0, 0), (1024, 0, 0), (1024, 24, 0), (256, 3, 0),
                               (1024, 8, 96)):
        gam, g, st, _, _ = sc.solve_lcp(P, con, max_iter=5, op=2, slices_per_wave=spw,
                                        block=block, grid=grid, lds_entries_per_wave=cache)
        assert (st["slices_per_wave"], st["block"], st["op"]) == (spw, block, 2)
        np.testing.assert_allclose(gam.cpu().numpy()[pm], go, rtol=1e-9,
                                   atol=1e-9 * np.abs(go).max())
    rng = np.random.default_rng(4545)
    x_o = rng.uniform(0.0, 1.0, c.nc) * (rng.uniform(size=c.nc) < 0.6)
    x_lib = np.empty_like(x_o)
    x_lib[pm] = x_o
    ref = None
    # entries held in LDS (all, a prefix per wave, none) change nothing either
    for block, grid, cache in ((1024, 0, 0), (256, 0, 0), (1024, 8, 0), (256, 40, 0),
                               (1024, 8, 96), (256, 3, 250), (1024, 0, -1)):
        _, g, st, _, _ = sc.solve_lcp(P, con, max_iter=0, op=2, slices_per_wave=spw,
                                      block=block, grid=grid, lds_entries_per_wave=cache,
                                      gamma0=torch.from_numpy(x_lib))
        if cache > 0:
            assert st["lds_entries_per_wave"] == cache
        elif cache < 0:
            assert st["lds_entries_per_wave"] == 0
        if ref is None:
            ref = g.clone()
        else:
            assert torch.equal(g, ref), (block, grid, cache)
    want = O.mvop(s, c, x_o) + q_orc
    np.testing.assert_allclose(ref.cpu().numpy()[pm], want, rtol=1e-12,
                               atol=1e-12 * np.abs(want).max())


def test_matrix_default_grid_follows_the_size_of_m():
    """With the grid left open the assembled-M solve takes 8 round(sqrt(nnz)
    / 40) workgroups (at least 8, at most one per CU), and the solve it runs
    converges to the same point as the full grid's: g = M gamma + q and
    F_c = D gamma agree with the oracle's at the tolerance's error bound."""
    sc = _sc()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for s in (W.workload(1), W.rods(4000, seed=44), W.rods_and_spheres(2500, 500, seed=45)):
        _say(f"default grid: {s.name}")
        P, box, u_nc, con = _setup_gpu(s)
        want = 8 * max(1, int(round(np.sqrt(con.nnz) / 40.0)))
        want = min(want, cus - cus % 8)
        gam, g, st, f_c, _ = sc.solve_lcp(P, con, tol=1e-9, want_fc=True, op=2)
        gam2, g2, st2, f_c2, _ = sc.solve_lcp(P, con, tol=1e-9, want_fc=True, op=2, grid=cus)
        assert st["grid"] == want and st2["grid"] == cus - cus % 8
        assert st["status"] == 0 and st2["status"] == 0
        c, u_orc, q_orc = O.setup(s)
        pm = _perm(con)
        go, gg, sto = O.bbpgd(s, c, q_orc, tol=1e-9)
        F = O.D_apply(s.n, c, go)
        for g_, f_ in ((g, f_c), (g2, f_c2)):
            np.testing.assert_allclose(g_.cpu().numpy()[pm], gg, rtol=0,
                                       atol=1e-6 * max(1.0, np.abs(gg).max()))
            np.testing.assert_allclose(f_.cpu().numpy(), F, rtol=0,
                                       atol=1e-6 * max(1.0, np.abs(F).max()))


def test_matrix_tiny_systems():
    """Fewer rows than one slice (most workgroups own no slice)."""
    sc = _sc()
    big = W.rods(1200, seed=46)
    cb = O.find_contacts(big)
    for k in (1, 4, 12):
        idx = np.unique(np.concatenate([cb.i[:k], cb.j[:k]]))
        s = big.subset(idx)
        _say(f"matrix tiny: {len(idx)} rods")
        P, box, u_nc, con = _setup_gpu(s)
        c, u_orc, q_orc = O.setup(s)
        assert 1 <= c.nc < 64 and con.count == c.nc
        pm = _perm(con)
        gam, g, st, _, _ = sc.solve_lcp(P, con, tol=1e-10, op=2)
        go, gg, sto = O.bbpgd(s, c, q_orc, tol=1e-10)
        assert st["status"] == 0 and st["op"] == 2
        np.testing.assert_allclose(g.cpu().numpy()[pm], gg, rtol=1e-6,
                                   atol=1e-6 * np.abs(gg).max())
        np.testing.assert_allclose(gam.cpu().numpy()[pm], go, rtol=1e-6,
                                   atol=1e-6 * np.abs(go).max())


def test_edge_cases():
    sc = _sc()
    import paper_1909_06623_amd._abi as A
    _say("edge: empty system")
    s = W.spheres(10, 0.3, seed=1)
    e = s.subset(np.arange(0))
    P = sc.Particles.from_suspension(e)
    box = sc.Box(tuple(s.box))
    con = sc.build_contacts(P, box, s.delta, torch.zeros((0, 6), dtype=torch.float64), s.dt)
    assert con.count == 0
    _say("edge: dilute, no pairs")
    s = W.spheres(27, 0.3, seed=2)
    g = np.stack(np.meshgrid(*[np.arange(3)] * 3, indexing="ij"), -1).reshape(-1, 3)
    s.pos = 4.0 * g + 1.0          # lattice spacing 4 > 2R + delta
    s.box = np.full(3, 12.0)
    P, box, u_nc, con = _setup_gpu(s)
    assert con.count == 0
    gam, g, st, f_c, u_c = sc.solve_lcp(P, con, want_fc=True)
    assert (st["status"], st["iters"], st["mvops"]) == (0, 0, 1)
    assert torch.all(f_c == 0)
    _say("edge: separating pairs only")
    s = W.workload(1)
    P, box, u_nc, con = _setup_gpu(s)
    con.q[: con.count] = torch.abs(con.q[: con.count]) + 1.0
    gam, g, st, _, _ = sc.solve_lcp(P, con)
    assert (st["iters"], st["mvops"]) == (0, 1) and torch.all(gam == 0)
    _say("edge: max_iter 0 and warm start")
    s = W.rods(2000, seed=3)
    P, box, u_nc, con = _setup_gpu(s)
    gam, g, st, _, _ = sc.solve_lcp(P, con, max_iter=0)
    assert (st["status"], st["iters"], st["mvops"]) == (1, 0, 2)
    gam, g, st, _, _ = sc.solve_lcp(P, con, tol=1e-8)
    assert st["status"] == 0
    gam2, g2, st2, _, _ = sc.solve_lcp(P, con, tol=1e-6, gamma0=gam)
    assert (st2["iters"], st2["mvops"]) == (0, 1)
    _say("edge: capacity too small (raw ABI)")
    con_small = sc.Contacts(P.n, 10)
    cc = con_small.c()
    pc, bc = P.c(), box.c()
    ws = sc.Workspace()
    wsp, wsn = ws.get(P.n, con.capacity)
    import ctypes
    rc = A.lib().sc_build_contacts(ctypes.byref(pc), ctypes.byref(bc), s.delta,
                                   ctypes.c_void_p(u_nc.data_ptr()), s.dt, ctypes.byref(cc),
                                   wsp, wsn, ctypes.c_void_p(0))
    assert rc == A.SC_ERR_CAPACITY and cc.count == con.count
    _say("edge: box too small")
    s2 = W.rods(200, seed=4, min_side=1.5)
    P2 = sc.Particles.from_suspension(s2)
    with pytest.raises(sc.ScError) as ei:
        sc.build_contacts(P2, sc.Box(tuple(s2.box)), s2.delta,
                          torch.zeros((s2.n, 6), dtype=torch.float64), s2.dt)
    assert ei.value.code == A.SC_ERR_BOX
    _say("edge: NaN in u_nc")
    bad = u_nc.clone()
    bad[5, 0] = float("nan")
    with pytest.raises(sc.ScError) as ei:
        sc.build_contacts(P, box, s.delta, bad, s.dt)
    assert ei.value.code == A.SC_ERR_NONFINITE
    _say("edge: non-unit rod axis")
    P3 = sc.Particles(P.pos, P.axis * 1.01, P.radius, P.half_len, P.mob)
    with pytest.raises(sc.ScError) as ei:
        sc.build_contacts(P3, box, s.delta, u_nc, s.dt)
    assert ei.value.code == A.SC_ERR_NONFINITE
    _say("edge: NaN in q reaches the solver")
    con.q[3] = float("nan")
    gam, g, st, _, _ = sc.solve_lcp(P, con)
    assert st["status"] == A.SC_ERR_NONFINITE
