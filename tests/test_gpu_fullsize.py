"""Parity at full size, in the launch configuration bench.py times.

100,000 rods (the benchmark workload): contact lists equal the oracle's
exactly, q agrees, the converged gamma agrees within 1e-6 relative (both
sides solved to 1e-9; the oracle's solution polished on its active set),
the solve bench.py times (tol 1e-6) satisfies the KKT conditions, and the
adjoint of L = 1/2 ||D gamma||^2 agrees with the oracle's.

1,000,000 rods + 100,000 spheres: the oracle cannot enumerate this in
test time, so the checks are sampled or hold at any size: Phi of sampled
reported pairs recomputed by the oracle, the exact pair set inside an
interior sub-box, and the KKT conditions of the solve."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _gpu(s):
    import paper_1909_06623_amd as sc
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box))
    u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
    con = sc.build_contacts(P, box, s.delta, u_nc, s.dt)
    return P, box, u_nc, con


def _kkt(gam, g, tol):
    assert np.all(gam >= 0.0)
    assert np.linalg.norm(np.minimum(gam, g)) < tol
    assert np.all(np.abs(gam * g) <= tol * np.maximum(1.0, np.maximum(gam, np.abs(g))))
    assert np.all(g >= -tol)


@pytest.mark.timeout(900)
def test_rods100k_bench_configuration():
    import paper_1909_06623_amd as sc
    s = W.workload(2)
    _say(f"full size {s.name}: N={s.n}")
    P, box, u_nc, con = _gpu(s)
    c, u_orc, q_o = O.setup(s)
    _say(f"contacts {con.count} vs oracle {c.nc}")
    assert con.count == c.nc and con.n_borderline == 0
    pm = con.canonical_order().cpu().numpy()
    assert np.array_equal(con.i.cpu().numpy()[pm], c.i)
    assert np.array_equal(con.j.cpu().numpy()[pm], c.j)
    np.testing.assert_allclose(con.q[: con.count].cpu().numpy()[pm], q_o, rtol=1e-11,
                               atol=1e-11 * np.abs(q_o).max())
    # the solve bench.py times
    gam6, g6, st6, _, _ = sc.solve_lcp(P, con, tol=s.tol)
    assert st6["status"] == 0 and st6["op"] == 2 and st6["block"] == 1024
    _kkt(gam6.cpu().numpy(), g6.cpu().numpy(), s.tol)
    # converged parity
    gam9, g9, st9, f_c, _ = sc.solve_lcp(P, con, tol=1e-9, want_fc=True)
    assert st9["status"] == 0
    go, _, sto = O.bbpgd(s, c, q_o, tol=1e-9)
    gp, gpg, passes = O.polish(s, c, q_o, go)
    assert passes >= 1
    ga9 = gam9.cpu().numpy()[pm]
    rel9 = np.linalg.norm(ga9 - gp) / np.linalg.norm(gp)
    rel6 = np.linalg.norm(gam6.cpu().numpy()[pm] - gp) / np.linalg.norm(gp)
    _say(f"iters gpu {st9['iters']} oracle {sto.iters}; rel gamma err {rel9:.2e} (tol 1e-9), "
         f"{rel6:.2e} (tol 1e-6)")
    assert rel9 <= 1e-6
    assert rel6 <= 1e-6
    # adjoint of L = 1/2 ||D gamma||^2 (the adjoint configuration)
    if not np.array_equal(ga9 > 0, gp > 0):
        pytest.skip("active sets differ (weakly active contacts)")
    dq, dpos, sta = sc.solve_lcp_adjoint(P, box, con, u_nc, s.dt, gam9, dL_df=f_c, tol=1e-12)
    rq, rpos, _ = O.adjoint(s, c, q_o, u_orc, gp, dL_dF=O.D_apply(s.n, c, gp), method="cg")
    np.testing.assert_allclose(dq.cpu().numpy()[pm], rq, rtol=0, atol=1e-6 * np.abs(rq).max())
    np.testing.assert_allclose(dpos.cpu().numpy(), rpos, rtol=0,
                               atol=1e-6 * np.abs(rpos).max())


@pytest.mark.timeout(900)
def test_rods1M_spheres100k_sampled():
    import paper_1909_06623_amd as sc
    s = W.workload(3)
    _say(f"full size {s.name}: N={s.n}")
    P, box, u_nc, con = _gpu(s)
    nc = con.count
    _say(f"contacts {nc}, nnz {con.nnz}")
    ci = con.i.cpu().numpy()
    cj = con.j.cpu().numpy()
    phi = con.phi[:nc].cpu().numpy()
    assert np.all(ci < cj) and np.all(phi <= s.delta)
    # sampled pairs: Phi recomputed by the oracle
    rng = np.random.default_rng(31)
    pick = rng.choice(nc, size=2000, replace=False)
    for l in pick:
        i, j = int(ci[l]), int(cj[l])
        ph = O.pair_geometry(s.pos[i], s.axis[i], s.radius[i], s.half_len[i],
                             s.pos[j], s.axis[j], s.radius[j], s.half_len[j],
                             box=s.box, periodic=1)["phi"]
        assert abs(ph - phi[l]) <= 1e-12 * max(1.0, abs(ph))
    # exact pair set inside an interior sub-box: every partner of a particle
    # there lies within the interaction range, so the oracle's pairs among
    # the particles of the widened box contain all of them
    r = s.interaction_range()
    lo, hi = 8.0, 14.0
    outer = np.flatnonzero(np.all((s.pos >= lo - r) & (s.pos < hi + r), axis=1))
    inner = np.zeros(s.n, dtype=bool)
    inner[np.all((s.pos >= lo) & (s.pos < hi), axis=1)] = True
    sub = s.subset(outer)
    cs = O.find_contacts(sub)
    oi, oj = outer[cs.i], outer[cs.j]
    keep = inner[oi] & inner[oj]
    want = set(zip(oi[keep].tolist(), oj[keep].tolist()))
    both = inner[ci] & inner[cj]
    got = set(zip(ci[both].tolist(), cj[both].tolist()))
    _say(f"sub-box pairs: {len(got)} vs oracle {len(want)}")
    assert len(want) > 1000 and got == want
    # the solve (forward only for this configuration)
    gam, g, st, _, _ = sc.solve_lcp(P, con, tol=s.tol)
    _say(f"solve: {st['status']} iters {st['iters']} ms {st['kernel_ms']:.1f}")
    assert st["status"] == 0
    _kkt(gam.cpu().numpy(), g.cpu().numpy(), s.tol)
