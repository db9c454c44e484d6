"""Batches that build their own contacts on the device (build=True): every
instance's contact list, q and M equal those of its own build_contacts bit
for bit, so solves and adjoints equal the prebuilt-contacts batch's bit for
bit; graph replays follow positions that move between solves; an instance
whose build fails reports its status without disturbing the others."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _setup(count, n_max, seed):
    import paper_1909_06623_amd as sc
    sus, _ = W.batched_instances(count=count, seed=seed, n_min=30, n_max=n_max)
    out = []
    for s in sus:
        P = sc.Particles.from_suspension(s)
        box = sc.Box(tuple(s.box))
        u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
        out.append((s, P, box, u_nc))
    return out


def _same_contacts(bcon, con):
    n = con.count
    assert bcon.count == n
    for name in ("ci", "cj", "phi", "q", "frame"):
        assert torch.equal(getattr(bcon, name)[:n], getattr(con, name)[:n]), name


def _check_against_single(b, inst, team, tol, adjoint):
    """Contacts equal each instance's own build; gamma (and gradients) equal a
    prebuilt-contacts batch of the same team size."""
    import paper_1909_06623_amd as sc
    cnt = b.counts()
    singles = []
    for k, ((s, P, box, u_nc), (nc, nnz, status)) in enumerate(zip(inst, cnt)):
        assert status == 0, (k, status)
        con = sc.build_contacts(P, box, s.delta, u_nc, s.dt)
        assert nc == con.count and nnz == con.nnz, (k, nc, con.count, nnz, con.nnz)
        _same_contacts(b.contacts[k], con)
        singles.append(con)
    items = [(P, con, box, u_nc, s.dt) if adjoint else (P, con)
             for (s, P, box, u_nc), con in zip(inst, singles)]
    ref = sc.Batch(items, tol=tol, team=team, adjoint=adjoint, adjoint_tol=1e-12)
    ref.solve()
    st, _, _ = ref.stats()
    st_b, _, _ = b.stats()
    assert [x["iters"] for x in st] == [x["iters"] for x in st_b]
    for k, con in enumerate(singles):
        nc = con.count
        assert torch.equal(b.gamma[k][:nc], ref.gamma[k]), k
        assert torch.equal(b.g[k][:nc], ref.g[k]), k
        if adjoint:
            assert torch.equal(b.dL_dq[k][:nc], ref.dL_dq[k]), k
            assert torch.equal(b.dL_dpos[k], ref.dL_dpos[k]), k
    ref.close()
    return singles


@pytest.mark.parametrize("team", [1, 4])
def test_built_batch_equals_single_builds(team):
    import paper_1909_06623_amd as sc
    inst = _setup(12, 2500, W.SEED_BASE + 710)
    _say(f"built batch team={team}: {len(inst)} instances, N {sum(P.n for _, P, _, _ in inst)}")
    b = sc.Batch([(P, box, s.delta, u_nc, s.dt) for s, P, box, u_nc in inst], tol=1e-9,
                 team=team, build=True)
    b.solve()
    st, _, info = b.stats()
    assert all(x["status"] == 0 for x in st), [x["status"] for x in st]
    singles = _check_against_single(b, inst, team, 1e-9, 0)
    # two instances against the oracle's contact set and converged solution
    for (s, P, box, u_nc), con, gam in list(zip(inst, singles, b.gamma))[:2]:
        c, _, q = O.setup(s)
        pm = con.canonical_order().cpu().numpy()
        assert np.array_equal(con.i.cpu().numpy()[pm], c.i)
        assert np.array_equal(con.j.cpu().numpy()[pm], c.j)
        if c.nc:
            go, g_o, _ = O.bbpgd(s, c, q, tol=1e-10)
            F = O.D_apply(s.n, c, gam[: con.count].cpu().numpy()[pm])
            Fo = O.D_apply(s.n, c, go)
            np.testing.assert_allclose(F, Fo, rtol=0, atol=1e-6 * max(1.0, np.abs(Fo).max()))
    b.close()


def test_built_batch_graph_follows_moving_positions():
    """Build + solve + adjoint captured once and replayed after the particles
    moved (in place): every replay equals fresh builds and solves at the new
    positions; eager solves between replays agree too."""
    import paper_1909_06623_amd as sc
    inst = _setup(8, 1500, W.SEED_BASE + 711)
    _say(f"built batch graph: {len(inst)} instances")
    b = sc.Batch([(P, box, s.delta, u_nc, s.dt) for s, P, box, u_nc in inst], tol=1e-9,
                 team=2, build=True, adjoint=1, adjoint_tol=1e-12)
    rng = np.random.default_rng(5)
    counts = []
    for step in range(3):
        b.graph_solve()
        torch.cuda.synchronize()
        st, adj, _ = b.stats()
        assert all(x["status"] == 0 for x in st) and all(x["status"] == 0 for x in adj)
        counts.append([c for c, _, _ in b.counts()])
        _say(f"replay {step}: contacts {sum(counts[-1])}")
        _check_against_single(b, inst, 2, 1e-9, 1)
        g_graph = [x.clone() for x in b.gamma]
        b.solve()
        assert all(torch.equal(a, x) for a, x in zip(g_graph, b.gamma))
        for s, P, box, u_nc in inst:
            s.pos = s.pos + 0.004 * rng.standard_normal(s.pos.shape)
            P.pos.copy_(torch.from_numpy(s.pos))
    assert counts[0] != counts[-1]  # the contact sets did change
    b.close()


def test_built_batch_status_per_instance():
    """A contact capacity too small, a NaN centre and a radius grown past the
    planned search grid each fail their own instance only."""
    import paper_1909_06623_amd as sc
    import paper_1909_06623_amd._abi as A
    inst = [x for x in _setup(8, 800, W.SEED_BASE + 712)]
    ncs = [sc.build_contacts(P, box, s.delta, u_nc, s.dt) for s, P, box, u_nc in inst]
    pick = [k for k, c in enumerate(ncs) if c.count > 20][:4]
    assert len(pick) == 4
    inst = [inst[k] for k in pick]
    ncs = [ncs[k] for k in pick]
    caps = [c.count + 16 for c in ncs]
    caps[0] = ncs[0].count - 5                      # too few contact rows
    nnzs = [c.nnz + 64 for c in ncs]
    _say("built batch status paths")
    b = sc.Batch([(P, box, s.delta, u_nc, s.dt) for s, P, box, u_nc in inst], tol=1e-9,
                 team=2, build=True, capacity=caps, nnz_capacity=nnzs)
    inst[1][1].pos[3, 1] = float("nan")             # bad data
    inst[2][1].radius[0] *= 1.5                     # outgrows the planned grid
    for run in (b.solve, b.graph_solve):
        run()
        st, _, _ = b.stats()
        cnt = b.counts()
        assert [c[2] for c in cnt] == [A.SC_ERR_CAPACITY, A.SC_ERR_NONFINITE, A.SC_ERR_BOX,
                                       A.SC_OK]
        assert [x["status"] for x in st] == [A.SC_ERR_CAPACITY, A.SC_ERR_NONFINITE,
                                             A.SC_ERR_BOX, A.SC_OK]
        _same_contacts(b.contacts[3], ncs[3])
    # a nonzero capacity too small
    s, P, box, u_nc = inst[3]
    b2 = sc.Batch([(P, box, s.delta, u_nc, s.dt)], tol=1e-9, team=1, build=True,
                  capacity=[ncs[3].count], nnz_capacity=[ncs[3].nnz - 1])
    b2.solve()
    assert b2.counts()[0][2] == A.SC_ERR_CAPACITY
    b2.close()
    b.close()



def test_one_system_step_without_host_synchronisation():
    """A batch of one system with build=True is one whole step (contact
    build, M, solve and adjoint) with no host synchronisation inside: its
    graph, captured once and replayed after the particles moved, equals a
    fresh build_contacts and a prebuilt-contacts solve at the new positions,
    and the forces D gamma meet the oracle's (unique at the LCP solution)."""
    import paper_1909_06623_amd as sc
    s = W.rods(2000, seed=W.SEED_BASE + 707)
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box))
    u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
    inst = [(s, P, box, u_nc)]
    _say(f"one-system built batch: N {s.n}")
    b = sc.Batch([(P, box, s.delta, u_nc, s.dt)], tol=1e-9, team=4, build=True, adjoint=1,
                 adjoint_tol=1e-12)
    rng = np.random.default_rng(707)
    for step in range(2):
        b.graph_solve()
        torch.cuda.synchronize()
        st, adj, _ = b.stats()
        assert st[0]["status"] == 0 and adj[0]["status"] == 0
        con, = _check_against_single(b, inst, 4, 1e-9, 1)
        _say(f"replay {step}: contacts {con.count}, iterations {st[0]['iters']}")
        c, _, q = O.setup(s)
        pm = con.canonical_order().cpu().numpy()
        assert np.array_equal(con.i.cpu().numpy()[pm], c.i)
        assert np.array_equal(con.j.cpu().numpy()[pm], c.j)
        go, _, _ = O.bbpgd(s, c, q, tol=1e-10)
        F = O.D_apply(s.n, c, b.gamma[0][: con.count].cpu().numpy()[pm])
        Fo = O.D_apply(s.n, c, go)
        np.testing.assert_allclose(F, Fo, rtol=0, atol=1e-6 * max(1.0, np.abs(Fo).max()))
        s.pos = s.pos + 0.004 * rng.standard_normal(s.pos.shape)
        P.pos.copy_(torch.from_numpy(s.pos))
    b.close()
