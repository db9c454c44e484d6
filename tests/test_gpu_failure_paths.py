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
