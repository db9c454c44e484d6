"""The boundary's stream-ordered forms: sc_canonical_order (the library's
permutation to the canonical (i, j) order of section 3.1's one constraint
per pair i < j) and sc_solve_lcp_async (the solve with its status left on
the device): equal to the synchronising solve bit for bit, eagerly and as a
HIP graph replayed several times with other work in between."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _setup(s):
    import paper_1909_06623_amd as sc
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box), lo=tuple(s.lo), periodic=bool(s.periodic), walls=int(s.walls))
    u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
    con = sc.build_contacts(P, box, s.delta, u_nc, s.dt)
    return P, box, u_nc, con


def _walls_case():
    s = W.rods_and_spheres(800, 200, seed=W.SEED_BASE + 81)
    s.periodic = 0
    s.walls = 63
    return s


@pytest.mark.parametrize("kind", ["mixed", "walls", "spheres"])
def test_canonical_order_from_the_library(kind):
    s = {"mixed": lambda: W.rods_and_spheres(3000, 600, seed=W.SEED_BASE + 80),
         "walls": _walls_case,
         "spheres": lambda: W.spheres(2000, 0.3, W.SEED_BASE + 82)}[kind]()
    _say(f"canonical order {kind}: N={s.n}")
    P, box, u_nc, con = _setup(s)
    perm = con.canonical_order().cpu().numpy()
    ci, cj = con.i.cpu().numpy(), con.j.cpu().numpy()
    assert np.array_equal(np.sort(perm), np.arange(con.count))      # a permutation
    assert np.array_equal(perm, np.lexsort((cj, ci)))               # by ci, then cj
    c = O.find_contacts(s)
    assert np.array_equal(ci[perm], c.i) and np.array_equal(cj[perm], c.j)
    if kind == "walls":
        assert np.any(cj < 0)


def _async_equals_sync(sc, P, con, tol, op, ws):
    ref = sc.solve_lcp(P, con, tol=tol, want_fc=True, op=op, workspace=ws)
    nc = con.count
    gam = torch.full((max(1, nc),), float("nan"), dtype=torch.float64, device="cuda")
    g = torch.full_like(gam, float("nan"))
    f_c = torch.full((P.n, 6), float("nan"), dtype=torch.float64, device="cuda")
    u_c = torch.full_like(f_c, float("nan"))
    stats = torch.zeros(sc.STATS_BYTES, dtype=torch.uint8, device="cuda")
    sc.solve_lcp_async(P, con, gam, g, stats, tol=tol, f_c=f_c, u_c=u_c, op=op, workspace=ws)
    st = sc.stats_from_device(stats)
    for key in ("status", "iters", "mvops", "n_active", "residual", "alpha", "n_degenerate",
                "grid", "block", "op", "lanes_per_particle", "slices_per_wave"):
        assert st[key] == ref[2][key], (key, st[key], ref[2][key])
    assert torch.equal(gam[:nc], ref[0]) and torch.equal(g[:nc], ref[1])
    assert torch.equal(f_c, ref[3]) and torch.equal(u_c, ref[4])
    return ref, st


@pytest.mark.parametrize("op", [1, 2])
def test_async_solve_equals_the_synchronising_solve(op):
    import paper_1909_06623_amd as sc
    s = W.rods_and_spheres(3000, 600, seed=W.SEED_BASE + 83)
    _say(f"async solve op={op}: N={s.n}")
    P, box, u_nc, con = _setup(s)
    ws = sc.Workspace()
    ref, st = _async_equals_sync(sc, P, con, s.tol, op, ws)
    assert st["status"] == 0 and st["iters"] > 10
    # the solve's own outcome lives in the device record, the call itself succeeds
    stats = torch.zeros(sc.STATS_BYTES, dtype=torch.uint8, device="cuda")
    gam = torch.empty(con.count, dtype=torch.float64, device="cuda")
    g = torch.empty_like(gam)
    sc.solve_lcp_async(P, con, gam, g, stats, tol=1e-14, max_iter=3, op=op, workspace=ws)
    st3 = sc.stats_from_device(stats)
    assert (st3["status"], st3["iters"], st3["mvops"]) == (1, 3, 5)
    sc.solve_lcp_async(P, con, gam, g, stats, tol=1e-8, op=op, spin_limit=1, workspace=ws)
    assert sc.stats_from_device(stats)["status"] == -7      # SC_ERR_TIMEOUT, reported
    # a warm start at the solution: one product, no step
    g0 = ref[0].clone()
    gam.copy_(g0)
    sc.solve_lcp_async(P, con, gam, g, stats, tol=s.tol, warm_start=True, op=op, workspace=ws)
    stw = sc.stats_from_device(stats)
    assert (stw["status"], stw["iters"], stw["mvops"]) == (0, 0, 1)
    assert torch.equal(gam, g0)


def test_async_solve_without_contacts():
    import paper_1909_06623_amd as sc
    s = W.spheres(27, 0.3, seed=2)
    grid = np.stack(np.meshgrid(*[np.arange(3)] * 3, indexing="ij"), -1).reshape(-1, 3)
    s.pos = 4.0 * grid + 1.0
    s.box = np.full(3, 12.0)
    P, box, u_nc, con = _setup(s)
    assert con.count == 0
    stats = torch.zeros(sc.STATS_BYTES, dtype=torch.uint8, device="cuda")
    f_c = torch.full((P.n, 6), float("nan"), dtype=torch.float64, device="cuda")
    u_c = torch.full_like(f_c, float("nan"))
    one = torch.empty(1, dtype=torch.float64, device="cuda")
    sc.solve_lcp_async(P, con, one, one.clone(), stats, f_c=f_c, u_c=u_c)
    st = sc.stats_from_device(stats)
    assert (st["status"], st["mvops"]) == (0, 1)
    assert float(f_c.abs().max()) == 0.0 and float(u_c.abs().max()) == 0.0


@pytest.mark.parametrize("op", [1, 2])
def test_async_solve_in_a_graph_replays_the_eager_solve(op):
    """Captured with torch.cuda.graph (the persistent kernel's node marked
    cooperative by the call) and replayed three times, each replay after
    other eager work and a synchronisation, each bitwise the eager result."""
    import paper_1909_06623_amd as sc
    s = W.rods(4000, seed=W.SEED_BASE + 84)
    _say(f"graph-captured async solve op={op}: N={s.n}")
    P, box, u_nc, con = _setup(s)
    ws = sc.Workspace()
    ws.get(P.n, con.capacity)
    ref, _ = _async_equals_sync(sc, P, con, s.tol, op, ws)
    nc = con.count
    gam = torch.zeros(nc, dtype=torch.float64, device="cuda")
    g = torch.zeros_like(gam)
    f_c = torch.zeros((P.n, 6), dtype=torch.float64, device="cuda")
    u_c = torch.zeros_like(f_c)
    stats = torch.zeros(sc.STATS_BYTES, dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        sc.solve_lcp_async(P, con, gam, g, stats, tol=s.tol, f_c=f_c, u_c=u_c, op=op,
                           workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        sc.solve_lcp_async(P, con, gam, g, stats, tol=s.tol, f_c=f_c, u_c=u_c, op=op,
                           workspace=ws)
    other = W.rods(1500, seed=W.SEED_BASE + 85)
    Po, _, _, co = _setup(other)
    for rep in range(3):
        for t in (gam, g, f_c, u_c):
            t.fill_(float("nan"))
        stats.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        st = sc.stats_from_device(stats)
        assert st["status"] == 0 and st["iters"] == ref[2]["iters"], (rep, st)
        assert torch.equal(gam, ref[0]) and torch.equal(g, ref[1]), rep
        assert torch.equal(f_c, ref[3]) and torch.equal(u_c, ref[4]), rep
        # eager work of the program between replays
        sc.solve_lcp(Po, co, tol=other.tol)
        torch.cuda.synchronize()
    del graph
