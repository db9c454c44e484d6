"""GPU parity of the implicit adjoint against the oracle's adjoint (which is
itself pinned by finite differences and a closed form)."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def test_two_sphere_closed_form():
    import paper_1909_06623_amd as sc
    _say("adjoint two spheres")
    d = np.array([0.2, 0.7, -0.4])
    d /= np.linalg.norm(d)
    pos = np.stack([np.zeros(3), 1.01 * d]) + 5.0
    P = sc.Particles.from_arrays(pos, np.tile([0.0, 0.0, 1.0], (2, 1)), np.full(2, 0.5),
                                 np.zeros(2), W.sphere_mobility(np.full(2, 0.5)))
    box = sc.Box((20.0, 20.0, 20.0))
    u_nc = torch.zeros((2, 6), dtype=torch.float64, device="cuda")
    u_nc[0, :3] = torch.from_numpy(30.0 * d)
    u_nc[1, :3] = torch.from_numpy(-30.0 * d)
    dt = 1e-3
    con = sc.build_contacts(P, box, 0.1, u_nc, dt)
    assert con.count == 1
    gam, g, st, f_c, u_c = sc.solve_lcp(P, con, tol=1e-12, want_fc=True)
    M = 2.0 / (6 * math.pi * 0.5)
    dq, dpos, sta = sc.solve_lcp_adjoint(P, box, con, u_nc, dt, gam,
                                         dL_dgamma=torch.ones(1, dtype=torch.float64,
                                                              device="cuda"))
    assert float(dq[0]) == pytest.approx(-1.0 / M, rel=1e-12)
    np.testing.assert_allclose(dpos.cpu().numpy()[1], -d / (M * dt), rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(dpos.cpu().numpy()[0], d / (M * dt), rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("op", [1, 2])
@pytest.mark.parametrize("kind", ["rods", "mixed"])
def test_against_oracle_adjoint(kind, op):
    import paper_1909_06623_amd as sc
    s = (W.rods(1500, seed=81) if kind == "rods"
         else W.rods_and_spheres(1000, 200, seed=82))
    _say(f"adjoint {kind} N={s.n}")
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box))
    u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
    con = sc.build_contacts(P, box, s.delta, u_nc, s.dt)
    gam, g, st, f_c, u_c = sc.solve_lcp(P, con, tol=1e-10, want_fc=True)
    assert st["status"] == 0
    c, u_orc, q = O.setup(s)
    pm = con.canonical_order().cpu().numpy()
    go, _, sto = O.bbpgd(s, c, q, tol=1e-10)
    gp, _, passes = O.polish(s, c, q, go)
    g_gpu = gam.cpu().numpy()[pm]
    if not np.array_equal(g_gpu > 0, gp > 0):
        pytest.skip("active sets differ at tol 1e-10 (weakly active contacts)")
    rng = np.random.default_rng(3)
    wts = rng.standard_normal(c.nc)          # oracle order
    wg = np.empty_like(wts)
    wg[pm] = wts                              # library order
    # loss 1: linear in gamma
    dq, dpos, sta = sc.solve_lcp_adjoint(P, box, con, u_nc, s.dt, gam,
                                         dL_dgamma=torch.from_numpy(wg).cuda(), tol=1e-12,
                                         op=op)
    assert sta["op"] == op
    rq, rpos, _ = O.adjoint(s, c, q, u_orc, gp, dL_dgamma=wts)
    print(f"[result] CG iters {sta['iters']} rel res {sta['residual']:.1e}", flush=True)
    np.testing.assert_allclose(dq.cpu().numpy()[pm], rq, rtol=0, atol=1e-6 * np.abs(rq).max())
    np.testing.assert_allclose(dpos.cpu().numpy(), rpos, rtol=0,
                               atol=1e-6 * np.abs(rpos).max())
    # loss 2: 1/2 ||D gamma||^2
    dq, dpos, sta = sc.solve_lcp_adjoint(P, box, con, u_nc, s.dt, gam, dL_df=f_c, tol=1e-12,
                                         op=op)
    F = O.D_apply(s.n, c, gp)
    rq, rpos, _ = O.adjoint(s, c, q, u_orc, gp, dL_dF=F)
    np.testing.assert_allclose(dq.cpu().numpy()[pm], rq, rtol=0, atol=1e-6 * np.abs(rq).max())
    np.testing.assert_allclose(dpos.cpu().numpy(), rpos, rtol=0,
                               atol=1e-6 * np.abs(rpos).max())


def test_chain_cg_lds_share_changes_nothing():
    """The matrix-free CG keeps pass A's incidence data in LDS up to a
    capacity (lds_entries_per_wave caps it, -1 turns it off); the arithmetic
    and its order do not change, so the gradients are bitwise equal for every
    share."""
    import paper_1909_06623_amd as sc
    s = W.rods(2500, seed=83)
    _say("chain CG LDS shares")
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box))
    u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
    con = sc.build_contacts(P, box, s.delta, u_nc, s.dt)
    gam, g, st, f_c, u_c = sc.solve_lcp(P, con, tol=1e-10, want_fc=True)
    assert st["status"] == 0
    ref = None
    for cache in (0, -1, 2, 11):
        dq, dpos, sta = sc.solve_lcp_adjoint(P, box, con, u_nc, s.dt, gam, dL_df=f_c, tol=1e-10,
                                             op=1, lds_entries_per_wave=cache)
        assert sta["status"] == 0 and sta["op"] == 1
        if cache > 0:
            assert sta["lds_entries_per_wave"] == cache
        elif cache < 0:
            assert sta["lds_entries_per_wave"] == 0
        if ref is None:
            ref = (dq.clone(), dpos.clone(), sta["iters"])
        else:
            assert sta["iters"] == ref[2]
            assert torch.equal(dq, ref[0]) and torch.equal(dpos, ref[1]), cache
