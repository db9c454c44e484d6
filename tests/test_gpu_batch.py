"""Batched persistent solve: every instance of a batch of uneven, mixed
sphere/rod suspensions agrees with the oracle; results are reproducible
(eager and graph replays bitwise equal); the autotuner reports its timings."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _instances(count, n_max, seed, full=False):
    import paper_1909_06623_amd as sc
    sus, _ = W.batched_instances(count=count, seed=seed, n_min=30, n_max=n_max)
    items = []
    for s in sus:
        P = sc.Particles.from_suspension(s)
        box = sc.Box(tuple(s.box))
        u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
        con = sc.build_contacts(P, box, s.delta, u_nc, s.dt)
        items.append((P, con, box, u_nc, s.dt) if full else (P, con))
    return sus, items


def _check_instance(s, con, gam, g, tol_rel, tol):
    c, u_orc, q = O.setup(s)
    assert con.count == c.nc
    if c.nc == 0:
        return
    pm = con.canonical_order().cpu().numpy()
    gg = g.cpu().numpy()[pm]
    ga = gam.cpu().numpy()[pm]
    go, g_o, sto = O.bbpgd(s, c, q, tol=1e-10)
    # g = M gamma + q and F_c = D gamma are unique at the minimum (also for
    # the singular M of overlapping sphere clusters)
    np.testing.assert_allclose(gg, g_o, rtol=0, atol=tol_rel * max(1.0, np.abs(g_o).max()))
    F = O.D_apply(s.n, c, ga)
    Fo = O.D_apply(s.n, c, go)
    np.testing.assert_allclose(F, Fo, rtol=0, atol=tol_rel * max(1.0, np.abs(Fo).max()))
    assert np.all(ga >= 0.0)
    assert np.linalg.norm(np.minimum(ga, gg)) < tol


@pytest.mark.parametrize("team", [1, 4])
def test_batch_matches_oracle_and_is_reproducible(team):
    import paper_1909_06623_amd as sc
    sus, items = _instances(14, 2500, seed=W.SEED_BASE + 700)
    _say(f"batch team={team}: {len(items)} instances, "
         f"n_c {sum(c.count for _, c in items)}")
    b = sc.Batch(items, tol=1e-9, team=team)
    b.solve()
    st, _, info = b.stats()
    assert info["team"] == team
    assert all(x["status"] == 0 for x in st), [x["status"] for x in st]
    g1 = [x.clone() for x in b.gamma]
    for s, (P, con), gam, g in zip(sus, items, b.gamma, b.g):
        _check_instance(s, con, gam, g, 1e-6, 1e-9)
    b.solve()
    assert all(torch.equal(a, x) for a, x in zip(g1, b.gamma))
    for _ in range(3):  # graph replays, with eager work in between
        b.graph_solve()
        st2, _, _ = b.stats()
        assert [x["iters"] for x in st2] == [x["iters"] for x in st]
        assert all(torch.equal(a, x) for a, x in zip(g1, b.gamma))
        b.solve()
        torch.cuda.synchronize()
    b.close()


def test_batch_autotune_and_tiny_instances():
    import paper_1909_06623_amd as sc
    sus, items = _instances(9, 400, seed=W.SEED_BASE + 701)
    _say(f"batch autotune: {len(items)} instances")
    b = sc.Batch(items, tol=1e-8, team=0)
    b.solve()
    st, _, info = b.stats()
    assert info["team"] in (1, 2, 4, 8, 16, 32)
    assert all(t > 0 for t in info["tune_ms"])
    assert all(x["status"] == 0 for x in st)
    for s, (P, con), gam, g in zip(sus, items, b.gamma, b.g):
        _check_instance(s, con, gam, g, 1e-5, 1e-8)
    b.close()


def test_batch_empty_and_contactless():
    import paper_1909_06623_amd as sc
    _say("batch: no instances; an instance without contacts")
    b = sc.Batch([], tol=1e-6, team=1)
    b.solve()
    st, _, info = b.stats()
    assert st == []
    s = W.spheres(27, 0.3, seed=2)
    g = np.stack(np.meshgrid(*[np.arange(3)] * 3, indexing="ij"), -1).reshape(-1, 3)
    s.pos = 4.0 * g + 1.0
    s.box = np.full(3, 12.0)
    P = sc.Particles.from_suspension(s)
    con = sc.build_contacts(P, sc.Box(tuple(s.box)), s.delta,
                            sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda()), s.dt)
    assert con.count == 0
    s2, items = _instances(2, 300, seed=W.SEED_BASE + 702)
    b = sc.Batch([(P, con)] + items, tol=1e-8, team=2)
    b.solve()
    st, _, _ = b.stats()
    assert [x["status"] for x in st] == [0, 0, 0]
    assert st[0]["mvops"] == 1


@pytest.mark.parametrize("team,adjoint_team,adjoint_block", [(1, 0, 0), (8, 0, 0), (8, 2, 1024)])
def test_batch_adjoint_matches_single_instance_and_oracle(team, adjoint_team, adjoint_block):
    """Forward + adjoint of L = 1/2 ||D gamma||^2 for every instance in one
    persistent launch: the gradients equal the single-instance adjoint of the
    batch's own solution (both are the same implicit solve), and agree with
    the oracle's adjoint on rod instances whose active sets match."""
    import paper_1909_06623_amd as sc
    sus, items = _instances(10, 1500, seed=W.SEED_BASE + 703, full=True)
    _say(f"batch adjoint team={team} adjoint_team={adjoint_team}: {len(items)} instances")
    b = sc.Batch(items, tol=1e-10, team=team, adjoint=1, adjoint_tol=1e-12,
                 adjoint_team=adjoint_team, adjoint_block=adjoint_block)
    b.solve()
    st, adj, info = b.stats()
    assert info["team"] == team and info["team_adjoint"] == (adjoint_team or team)
    assert info["block"] == 1024 and info["adjoint_block"] == (adjoint_block or 512)
    assert all(x["grid"] == (adjoint_team or team) for x in adj)
    assert all(x["block"] == (adjoint_block or 512) for x in adj)
    assert all(x["status"] == 0 for x in st)
    assert all(x["status"] == 0 for x in adj), [x["status"] for x in adj]
    checked = 0
    for s, (P, con, box, u_nc, dt), gam, dq, dpos in zip(sus, items, b.gamma, b.dL_dq,
                                                          b.dL_dpos):
        if con.count == 0:
            continue
        _, _, _, f_c, _ = sc.solve_lcp(P, con, tol=1e-10, want_fc=True, max_iter=0,
                                       gamma0=gam)
        rq, rpos, _ = sc.solve_lcp_adjoint(P, box, con, u_nc, dt, gam, dL_df=f_c, tol=1e-12)
        np.testing.assert_allclose(dq.cpu().numpy(), rq.cpu().numpy(), rtol=0,
                                   atol=1e-8 * max(1.0, float(rq.abs().max())))
        np.testing.assert_allclose(dpos.cpu().numpy(), rpos.cpu().numpy(), rtol=0,
                                   atol=1e-8 * max(1.0, float(rpos.abs().max())))
        if "rods" not in s.name:
            continue
        c, u_orc, q = O.setup(s)
        pm = con.canonical_order().cpu().numpy()
        go, _, _ = O.bbpgd(s, c, q, tol=1e-10)
        gp, _, _ = O.polish(s, c, q, go)
        if not np.array_equal(gam.cpu().numpy()[pm] > 0, gp > 0):
            continue
        oq, opos, _ = O.adjoint(s, c, q, u_orc, gp, dL_dF=O.D_apply(s.n, c, gp))
        np.testing.assert_allclose(dq.cpu().numpy()[pm], oq, rtol=0,
                                   atol=1e-6 * np.abs(oq).max())
        np.testing.assert_allclose(dpos.cpu().numpy(), opos, rtol=0,
                                   atol=1e-6 * np.abs(opos).max())
        checked += 1
    _say(f"oracle-checked rod instances: {checked}")
    assert checked >= 1
    # graph replay reproduces the gradients bitwise
    d1 = [x.clone() for x in b.dL_dpos]
    b.graph_solve()
    torch.cuda.synchronize()
    assert all(torch.equal(a, x) for a, x in zip(d1, b.dL_dpos))
    b.close()


def test_batch_autotune_picks_each_launch_and_reproduces():
    """With team = 0 and the adjoint on, the autotuner times the forward and
    the adjoint launch apart for every nonzeros-per-workgroup target and
    keeps the fastest of each; a batch created with the two picked targets
    gives bitwise the same solutions and gradients."""
    import paper_1909_06623_amd as sc
    sus, items = _instances(6, 1200, seed=W.SEED_BASE + 705, full=True)
    _say(f"batch adjoint autotune: {len(items)} instances")
    b = sc.Batch(items, tol=1e-10, team=0, adjoint=1, adjoint_tol=1e-12)
    b.solve()
    st, adj, info = b.stats()
    # policies: size classes for 4096 * 2^i nonzeros per workgroup, then one
    # team size 2^i
    def index(target, team):
        return [4096 << i for i in range(6)].index(target) if target else 6 + team.bit_length() - 1
    pol = sc.Batch.tuned_policy(info)
    assert all(t > 0 for t in info["tune_ms"]) and all(t > 0 for t in info["tune_adjoint_ms"])
    assert info["tune_ms"][index(info["nnz_per_workgroup"], info["team"])] == \
        min(info["tune_ms"])
    assert info["tune_adjoint_ms"][index(info["adjoint_nnz_per_workgroup"],
                                         info["team_adjoint"])] == min(info["tune_adjoint_ms"])
    assert all(x["status"] == 0 for x in st) and all(x["status"] == 0 for x in adj)
    f = sc.Batch(items, tol=1e-10, adjoint=1, adjoint_tol=1e-12, **pol)
    f.solve()
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(b.gamma, f.gamma))
    assert all(torch.equal(x, y) for x, y in zip(b.dL_dq, f.dL_dq))
    assert all(torch.equal(x, y) for x, y in zip(b.dL_dpos, f.dL_dpos))
    b.close()
    f.close()


def _team_class(nnz, target, tmax=32):
    t = 1
    while t < tmax and t * target < nnz:
        t *= 2
    return t


def test_batch_size_classes_match_oracle_and_single_instances():
    """Size classes: instance k runs on the smallest power of two t with
    t * nnz_per_workgroup >= its nonzeros; teams of 32 halve as the queue
    reaches smaller classes. With a small target the instances spread over
    several classes; every solution matches the oracle, each instance's team
    size is its class, the forward and adjoint are bitwise those of a batch
    that holds that instance alone at the same team size, and a graph replay
    repeats the eager results bitwise."""
    import paper_1909_06623_amd as sc
    sus, items = _instances(12, 2500, seed=W.SEED_BASE + 706, full=True)
    target = 1500
    _say(f"batch size classes: {len(items)} instances, target {target}")
    b = sc.Batch(items, tol=1e-10, team=0, nnz_per_workgroup=target, adjoint=1,
                 adjoint_tol=1e-12, adjoint_nnz_per_workgroup=4 * target)
    b.solve()
    st, adj, info = b.stats()
    assert info["nnz_per_workgroup"] == target and info["adjoint_nnz_per_workgroup"] == 4 * target
    want = [_team_class(con.nnz, target) for _, con, _, _, _ in items]
    want_a = [_team_class(con.nnz, 4 * target) for _, con, _, _, _ in items]
    assert [x["grid"] for x in st] == want and [x["grid"] for x in adj] == want_a
    assert len(set(want)) >= 3, want
    assert all(x["status"] == 0 for x in st) and all(x["status"] == 0 for x in adj)
    for s, (P, con, _, _, _), gam, g in zip(sus, items, b.gamma, b.g):
        _check_instance(s, con, gam, g, 1e-6, 1e-9)
    # each instance alone at its class's team size: bitwise the same
    for k in (0, len(items) // 2, len(items) - 1):
        one = sc.Batch([items[k]], tol=1e-10, team=want[k], adjoint=1, adjoint_tol=1e-12,
                       adjoint_team=want_a[k])
        one.solve()
        torch.cuda.synchronize()
        assert torch.equal(one.gamma[0], b.gamma[k]) and torch.equal(one.dL_dq[0], b.dL_dq[k])
        assert torch.equal(one.dL_dpos[0], b.dL_dpos[k])
        one.close()
    g1 = [x.clone() for x in b.gamma]
    d1 = [x.clone() for x in b.dL_dpos]
    b.graph_solve()
    b.graph_solve()
    torch.cuda.synchronize()
    assert all(torch.equal(a, x) for a, x in zip(g1, b.gamma))
    assert all(torch.equal(a, x) for a, x in zip(d1, b.dL_dpos))
    b.close()


def test_batch_status_paths_eager_and_graph():
    """Per-instance status codes come back from the batch in eager and in
    graph mode: a NaN in one instance's q gives SC_ERR_NONFINITE for that
    instance only, and a small iteration cap SC_NOT_CONVERGED for the rest."""
    import paper_1909_06623_amd as sc
    import paper_1909_06623_amd._abi as A
    sus, items = _instances(4, 800, seed=W.SEED_BASE + 704)
    items = [it for it in items if it[1].count > 10][:3]
    assert len(items) == 3
    _say("batch status paths")
    items[1][1].q[2] = float("nan")
    b = sc.Batch(items, tol=1e-12, max_iter=5, team=2)
    for run in (b.solve, b.graph_solve, b.graph_solve):
        run()
        st, _, _ = b.stats()
        assert [x["status"] for x in st] == [A.SC_NOT_CONVERGED, A.SC_ERR_NONFINITE,
                                             A.SC_NOT_CONVERGED]
        assert st[0]["iters"] == 5 and st[2]["iters"] == 5
    b.close()
