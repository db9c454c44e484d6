"""Failure handling of the persistent solvers, forced from the host: a spin
limit of one poll makes every grid-barrier wait give up, so the solve must
report SC_ERR_TIMEOUT with every workgroup leaving its loop (the kernel ends
normally), and the next solve must be unaffected."""
import pytest

torch = pytest.importorskip("torch")

import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("op", [1, 2])
def test_barrier_timeout_is_reported_and_leaves_no_trace(op):
    import paper_1909_06623_amd as sc
    import paper_1909_06623_amd._abi as A
    s = W.rods(3000, seed=W.SEED_BASE + 950)
    print(f"[case] forced barrier timeout, op={op}", flush=True)
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box))
    u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
    con = sc.build_contacts(P, box, s.delta, u_nc, s.dt)
    gam, _, st, _, _ = sc.solve_lcp(P, con, tol=1e-8, op=op)
    assert st["status"] == A.SC_OK
    gam = gam.clone()
    _, _, st_t, _, _ = sc.solve_lcp(P, con, tol=1e-8, op=op, spin_limit=1)
    assert st_t["status"] == A.SC_ERR_TIMEOUT
    gam2, _, st2, _, _ = sc.solve_lcp(P, con, tol=1e-8, op=op)
    assert st2["status"] == A.SC_OK and st2["iters"] == st["iters"]
    assert torch.equal(gam2, gam)


def test_stepper_raises_on_a_failed_solve_and_moves_nothing():
    """A step whose solve times out raises before the particles advance."""
    import paper_1909_06623_amd as sc
    import paper_1909_06623_amd._abi as A
    from paper_1909_06623_amd.timestep import TimeStepper
    s = W.rods(3000, seed=W.SEED_BASE + 951)
    print("[case] stepper with a forced barrier timeout", flush=True)
    P = sc.Particles.from_suspension(s)
    pos0, axis0 = P.pos.clone(), P.axis.clone()
    stp = TimeStepper(P, sc.Box(tuple(s.box)), s.delta, s.dt, torch.from_numpy(s.f_ext).cuda(),
                      tol=s.tol, spin_limit=1)
    with pytest.raises(A.ScError) as e:
        stp.step()
    assert e.value.code == A.SC_ERR_TIMEOUT
    assert torch.equal(P.pos, pos0) and torch.equal(P.axis, axis0)
    # the same stepper without the forced limit steps normally
    stp.spin_limit = 0
    info = stp.step()
    assert info.stats["status"] == A.SC_OK and not torch.equal(P.pos, pos0)


def test_autograd_forward_raises_on_a_failed_solve():
    import paper_1909_06623_amd as sc
    import paper_1909_06623_amd._abi as A
    from paper_1909_06623_amd.autograd import collision_solve, lcp_solve
    s = W.rods(2000, seed=W.SEED_BASE + 952)
    print("[case] autograd with a forced barrier timeout", flush=True)
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box))
    u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
    pos = P.pos.clone().requires_grad_(True)
    with pytest.raises(A.ScError) as e:
        collision_solve(pos, P, box, u_nc, s.dt, s.delta, tol=1e-8, spin_limit=1)
    assert e.value.code == A.SC_ERR_TIMEOUT
    con = sc.build_contacts(P, box, s.delta, u_nc, s.dt)
    q = con.q[: con.count].clone().requires_grad_(True)
    with pytest.raises(A.ScError) as e:
        lcp_solve(q, P, box, con, u_nc, s.dt, tol=1e-8, spin_limit=1)
    assert e.value.code == A.SC_ERR_TIMEOUT
    # and without it the same call differentiates
    gamma, f_c, info = collision_solve(pos, P, box, u_nc, s.dt, s.delta, tol=1e-8)
    (0.5 * (f_c * f_c).sum()).backward()
    assert info.adjoint_stats["status"] == A.SC_OK and torch.isfinite(pos.grad).all()
