"""sc_solve_lcp_noalloc (the solve with the library's own device scratch
array as workspace) against sc_solve_lcp on the same contacts: two calls in
a row, the second on a smaller system, each bitwise equal to the solve with
a caller workspace (same kernels, same launch shape, fixed-order sums)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _case(sc, s):
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box), lo=tuple(s.lo), periodic=bool(s.periodic))
    u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
    con = sc.build_contacts(P, box, s.delta, u_nc, s.dt)
    return P, con


def _solve_both(sc, P, con, tol, op):
    ref_gam, ref_g, ref_st, ref_fc, ref_uc = sc.solve_lcp(P, con, tol=tol, want_fc=True, op=op)
    nc = con.count
    gam = torch.full((max(1, nc),), float("nan"), dtype=torch.float64, device="cuda")
    g = torch.full_like(gam, float("nan"))
    f_c = torch.full((P.n, 6), float("nan"), dtype=torch.float64, device="cuda")
    u_c = torch.full_like(f_c, float("nan"))
    rc, st = sc.solve_lcp_noalloc(P, con, gam, g, tol=tol, f_c=f_c, u_c=u_c, op=op)
    torch.cuda.synchronize()
    assert rc == 0, (rc, st)
    for key in ("status", "iters", "mvops", "n_active", "grid", "op", "n_degenerate"):
        assert st[key] == ref_st[key], (key, st[key], ref_st[key])
    assert st["residual"] == ref_st["residual"] and st["residual"] < tol
    assert torch.equal(gam[:nc], ref_gam) and torch.equal(g[:nc], ref_g)
    assert torch.equal(f_c, ref_fc) and torch.equal(u_c, ref_uc)
    return st


@pytest.mark.parametrize("op", [0, 1])
def test_noalloc_solve_equals_workspace_solve_twice(op):
    import paper_1909_06623_amd as sc
    big = W.rods_and_spheres(3000, 600, seed=W.SEED_BASE + 71)
    small = W.spheres(400, 0.3, W.SEED_BASE + 72)
    for s in (big, small):
        print(f"[case] noalloc op={op} {s.name} N={s.n}", flush=True)
        P, con = _case(sc, s)
        assert con.count > 0
        st = _solve_both(sc, P, con, s.tol, op)
        print(f"[case]   n_c={con.count} iters={st['iters']} op={st['op']}", flush=True)


def test_noalloc_rejects_oversized_systems_before_device_work():
    import paper_1909_06623_amd as sc
    from paper_1909_06623_amd import _abi as A
    L = A.lib()
    p = A.sc_particles(100000, 0, 0, 0, 0, 0, 0)
    c = A.sc_contacts()
    c.capacity, c.count = 4_000_000, 0
    opts = A.sc_solve_opts(1e-6, 100, 1, 0, 0)
    st = A.sc_stats()
    rc = L.sc_solve_lcp_noalloc(ctypes.byref(p), ctypes.byref(c), ctypes.byref(opts), None, None,
                                None, None, ctypes.byref(st), None)
    assert rc == A.SC_ERR_WORKSPACE
    # and a valid call afterwards still works
    s = W.spheres(300, 0.3, W.SEED_BASE + 73)
    P, con = _case(sc, s)
    _solve_both(sc, P, con, s.tol, 0)
    assert np.isfinite(s.tol)
