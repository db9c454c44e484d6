"""Time stepping on the GPU (sc_advance, sc_quat_from_axis, sc_map_gamma and
the TimeStepper loop) against the oracle's time stepping."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import oracle.timestep as T  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def test_advance_and_quaternions_match_oracle():
    import paper_1909_06623_amd as sc
    from paper_1909_06623_amd import timestep as ts
    _say("advance kernel vs oracle")
    rng = np.random.default_rng(12)
    n = 1000
    axis = rng.standard_normal((n, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    axis[:3] = [[0, 0, 1.0], [0, 0, -1.0], [0, 1.0, 0]]
    pos = rng.uniform(0, 10, (n, 3))
    U1, U2 = rng.standard_normal((n, 6)), rng.standard_normal((n, 6))
    q_o = T.quat_from_axis(axis)
    P = sc.Particles.from_arrays(pos, axis, np.full(n, 0.1), np.full(n, 0.3),
                                 np.tile(W.rod_mobility(), (n, 1)))
    q = ts.quat_from_axis(P.axis).clone()
    np.testing.assert_allclose(q.cpu().numpy(), q_o, rtol=0, atol=1e-15)
    dt = 0.01
    ts.advance(P, q, torch.from_numpy(U1).cuda(), torch.from_numpy(U2).cuda(), dt)
    pos_o, q_o2, ax_o = T.advance(pos, q_o, U1 + U2, dt)
    np.testing.assert_allclose(P.pos.cpu().numpy(), pos_o, rtol=0, atol=1e-14)
    np.testing.assert_allclose(q.cpu().numpy(), q_o2, rtol=0, atol=1e-14)
    np.testing.assert_allclose(P.axis.cpu().numpy(), ax_o, rtol=0, atol=1e-14)


def test_map_gamma_takes_the_previous_gamma_of_each_pair():
    import paper_1909_06623_amd as sc
    from paper_1909_06623_amd import timestep as ts
    s = W.rods(3000, seed=W.SEED_BASE + 902)
    _say(f"map_gamma N={s.n}")
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box))
    u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
    a = sc.build_contacts(P, box, s.delta, u_nc, s.dt)
    ga = torch.rand(a.count, dtype=torch.float64, device="cuda") + 1.0
    rng = np.random.default_rng(1)
    P.pos.add_(torch.from_numpy(0.01 * rng.standard_normal((s.n, 3))).cuda())
    b = sc.build_contacts(P, box, s.delta, u_nc, s.dt)
    g0 = ts.map_gamma(s.n, a, ga, b).cpu().numpy()
    old = {(int(i), int(j)): float(g) for i, j, g in
           zip(a.i.cpu().numpy(), a.j.cpu().numpy(), ga.cpu().numpy())}
    want = np.array([old.get((int(i), int(j)), 0.0)
                     for i, j in zip(b.i.cpu().numpy(), b.j.cpu().numpy())])
    assert np.array_equal(g0, want)
    kept = np.count_nonzero(want)
    _say(f"pairs kept {kept} of {b.count}")
    assert 0 < kept < b.count


def _gpu_stepper(s, tol, warm=True):
    import paper_1909_06623_amd as sc
    from paper_1909_06623_amd import timestep as ts
    P = sc.Particles.from_suspension(s)
    return P, ts.TimeStepper(P, sc.Box(tuple(s.box)), s.delta, s.dt,
                             torch.from_numpy(s.f_ext).cuda(), tol=tol, warm_start=warm)


def test_two_spheres_pass_over_matches_oracle():
    """The paper's two-sphere experiment (dry mobility): the GPU trajectory
    follows the oracle's step by step, through the same stages."""
    a, ac, F, dt = 1.0, 1.01, 1.0, 0.02
    pos = np.array([[10.0, 10.0, 10.0], [10.0 + 4.0 * a, 10.0 + a, 10.0]])
    f_ext = np.zeros((2, 6))
    f_ext[0, 0], f_ext[1, 0] = F, -F
    rad = np.full(2, ac)
    s = W.Suspension("pair", pos, np.tile([0.0, 0.0, 1.0], (2, 1)), rad, np.zeros(2),
                     W.sphere_mobility(rad), f_ext, np.full(3, 40.0), 0.6 * ac, dt, 1e-12)
    _say("two spheres passing, GPU vs oracle")
    P, stp = _gpu_stepper(s, 1e-12)
    quat, rec = T.quat_from_axis(s.axis), None
    mt = W.sphere_mobility(ac)[0]
    stages_g, stages_o = [], []
    for _ in range(int(round(8.0 * a / (2 * mt * F * dt)))):
        info = stp.step()
        s, quat, rec = T.step(s, quat, rec, tol=1e-12)
        np.testing.assert_allclose(P.pos.cpu().numpy(), s.pos, rtol=0, atol=1e-11)
        for stages, nc, gam in ((stages_g, info.contacts.count, info.gamma.cpu().numpy()),
                                (stages_o, rec.i.size, rec.gamma)):
            st = "none" if nc == 0 else ("force" if gam[0] > 0 else "zero")
            if not stages or stages[-1] != st:
                stages.append(st)
    assert stages_g == stages_o == ["none", "zero", "force", "zero", "none"]


@pytest.mark.parametrize("warm", [True, False])
def test_rod_suspension_trajectory_matches_oracle(warm):
    s = W.rods_and_spheres(500, 100, seed=W.SEED_BASE + 903)
    _say(f"trajectory N={s.n} warm={warm}")
    P, stp = _gpu_stepper(s, 1e-10, warm)
    quat, rec = T.quat_from_axis(s.axis), None
    for k in range(4):
        info = stp.step()
        c_prev = O.find_contacts(s)
        s, quat, rec = T.step(s, quat, rec, warm=warm, tol=1e-10)
        con = info.contacts
        pm = con.canonical_order().cpu().numpy()
        assert np.array_equal(con.i.cpu().numpy()[pm], rec.i)
        assert np.array_equal(con.j.cpu().numpy()[pm], rec.j)
        assert np.array_equal(rec.i, c_prev.i)
        gam = info.gamma.cpu().numpy()[pm]
        np.testing.assert_allclose(gam, rec.gamma, rtol=0, atol=1e-6 * max(1.0, np.abs(rec.gamma).max()))
        scale = np.abs(s.pos).max()
        np.testing.assert_allclose(P.pos.cpu().numpy(), s.pos, rtol=0, atol=1e-9 * scale)
        np.testing.assert_allclose(P.axis.cpu().numpy(), s.axis, rtol=0, atol=1e-9)
        _say(f"step {k}: contacts {con.count}, iters gpu {info.stats['iters']} oracle {rec.iters}")


def test_time_stepper_with_mobility_objects():
    """TimeStepper(mobility=...): the dry mobility through the callback path
    follows the default (persistent, assembled-M) stepper; RPY given as an
    object steps exactly as RPY given by its radii; the persistent and the
    per-phase RPY solves step to the same centres."""
    import paper_1909_06623_amd as sc
    from paper_1909_06623_amd import timestep as ts
    s = W.spheres(400, 0.3, W.SEED_BASE + 919)
    s.periodic = 0
    s.tol = 1e-10
    print("[case] time stepper with mobility objects", flush=True)
    box = sc.Box(tuple(s.box), periodic=False)
    fe = torch.from_numpy(s.f_ext).cuda()
    Pa, Pb = sc.Particles.from_suspension(s), sc.Particles.from_suspension(s)
    a = ts.TimeStepper(Pa, box, s.delta, s.dt, fe, tol=s.tol)
    b = ts.TimeStepper(Pb, box, s.delta, s.dt, fe, tol=s.tol, mobility=sc.DryMobility(Pb))
    for _ in range(4):
        a.step()
        b.step()
    np.testing.assert_allclose(Pb.pos.cpu().numpy(), Pa.pos.cpu().numpy(), rtol=0, atol=1e-9)
    Pc, Pd = sc.Particles.from_suspension(s), sc.Particles.from_suspension(s)
    c = ts.TimeStepper(Pc, box, s.delta, s.dt, fe, tol=s.tol, hydro_radius=Pc.radius.clone())
    d = ts.TimeStepper(Pd, box, s.delta, s.dt, fe, tol=s.tol,
                       mobility=sc.RPY(Pd.pos, Pd.radius.clone()))
    Pe = sc.Particles.from_suspension(s)
    e = ts.TimeStepper(Pe, box, s.delta, s.dt, fe, tol=s.tol, hydro_radius=Pe.radius.clone(),
                       persistent=False)
    assert c.persistent and d.persistent and not e.persistent
    for _ in range(4):
        c.step()
        d.step()
        e.step()
    assert torch.equal(Pc.pos, Pd.pos)
    # the persistent RPY solve and the per-phase one step to the same centres
    np.testing.assert_allclose(Pe.pos.cpu().numpy(), Pc.pos.cpu().numpy(), rtol=0, atol=1e-9)
