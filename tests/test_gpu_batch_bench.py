"""The batched launch bench.py times, checked instance by instance against
the oracle: the 512 suspensions of uneven size (N log-uniform in [200,
20000], spheres and rods), contacts and M built on the device, the team
policy (size classes or one team size) chosen by the autotuner, Algorithm 1 (section 3.3.1) to 1e-6 and the
adjoint of L = 1/2 ||D gamma||^2 to a CG tolerance of 1e-8, replayed as one
HIP graph. An instance's arithmetic depends only on its team size, so these
are the results the benchmark's replays produce.

Forty instances are compared (the 24 largest and 16 drawn from the rest):
the contact set exactly (section 3.2's close pairs), the KKT conditions,
g = M gamma + q and F_c = D gamma (unique at the minimum also where M is
only semidefinite, as for overlapping spheres) against the oracle's
solution, gamma itself on rod instances (M SPD) within 1e-6 relative of the
oracle's polished solution (Eq. abserrcqp bounds the distance of any
tol-level iterate from it), and the adjoint's dL/dq and dL/d(centres) on rod
instances whose active set equals the oracle's."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _host_threads():
    env = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return max(1, min(16, env or (os.cpu_count() or 1)))


@pytest.mark.timeout(1200)
def test_bench_batched_launch_against_oracle():
    import paper_1909_06623_amd as sc
    sus, _ = W.batched_instances(count=512)
    items = []
    for s in sus:
        P = sc.Particles.from_suspension(s)
        box = sc.Box(tuple(s.box))
        u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
        items.append((P, box, s.delta, u_nc, s.dt))
    tol, atol = 1e-6, 1e-8   # the benchmark's tolerances
    b = sc.Batch(items, tol=tol, team=0, adjoint=1, adjoint_tol=atol, build=True)
    b.graph_solve()
    b.graph_solve()
    torch.cuda.synchronize()
    st, adj, info = b.stats()
    cnt = b.counts()
    _say(f"batch: {len(sus)} instances, tuned policy {sc.Batch.tuned_policy(info)}, "
         f"{sum(c for c, _, _ in cnt)} contacts, tune_ms {info['tune_ms']}, "
         f"adjoint {info['tune_adjoint_ms']}")
    assert info["team"] in (1, 2, 4, 8, 16, 32)
    assert all(x["status"] == 0 for x in st), [x["status"] for x in st if x["status"]]
    assert all(x["status"] == 0 for x in adj)
    assert all(z == 0 for _, _, z in cnt)
    order = np.argsort([-s.n for s in sus], kind="stable")
    rng = np.random.default_rng(17)
    pick = list(order[:24]) + list(rng.choice(order[24:], size=16, replace=False))
    nt = _host_threads()
    n_rods = n_adj = 0
    worst = {"g": 0.0, "F": 0.0, "gamma": 0.0, "dq": 0.0, "dpos": 0.0}
    for k in pick:
        s = sus[k]
        con = b.contacts[k]
        nc = cnt[k][0]
        _say(f"instance {k} {s.name}: N={s.n}, n_c={nc}, iters {st[k]['iters']}, "
             f"adjoint CG {adj[k]['iters']}")
        with O.threads(nt):
            c, u_orc, q = O.setup(s)
            assert nc == c.nc
            if nc == 0:
                continue
            pm = con.canonical_order().cpu().numpy()
            assert np.array_equal(con.i.cpu().numpy()[pm], c.i)
            assert np.array_equal(con.j.cpu().numpy()[pm], c.j)
            ga = b.gamma[k][:nc].cpu().numpy()[pm]
            gg = b.g[k][:nc].cpu().numpy()[pm]
            assert np.all(ga >= 0.0) and np.linalg.norm(np.minimum(ga, gg)) < tol
            go, g_o, sto = O.bbpgd(s, c, q, tol=1e-10)
        assert sto.status == 0
        rods = bool(np.all(s.half_len > 0))
        if rods:
            gp, g_p, passes = O.polish(s, c, q, go)
            assert passes >= 1
            go, g_o = gp, g_p
            rel = np.linalg.norm(ga - go) / np.linalg.norm(go)
            worst["gamma"] = max(worst["gamma"], rel)
            assert rel <= 1e-6, (k, rel)
            n_rods += 1
        eg = np.abs(gg - g_o).max() / max(1.0, np.abs(g_o).max())
        F, Fo = O.D_apply(s.n, c, ga), O.D_apply(s.n, c, go)
        eF = np.abs(F - Fo).max() / max(1.0, np.abs(Fo).max())
        worst["g"], worst["F"] = max(worst["g"], eg), max(worst["F"], eF)
        assert eg <= 1e-6 and eF <= 1e-6, (k, eg, eF)
        if rods and np.array_equal(ga > 0, go > 0):
            oq, opos, _ = O.adjoint(s, c, q, u_orc, go, dL_dF=O.D_apply(s.n, c, go))
            dq = b.dL_dq[k][:nc].cpu().numpy()[pm]
            dpos = b.dL_dpos[k].cpu().numpy()
            eq = np.abs(dq - oq).max() / np.abs(oq).max()
            ep = np.abs(dpos - opos).max() / np.abs(opos).max()
            worst["dq"], worst["dpos"] = max(worst["dq"], eq), max(worst["dpos"], ep)
            assert eq <= 1e-6 and ep <= 1e-6, (k, eq, ep)
            n_adj += 1
    _say(f"checked {len(pick)} instances ({n_rods} rod instances with gamma, {n_adj} "
         f"adjoints); worst relative errors {worst}")
    assert n_rods >= 8 and n_adj >= 4
    b.close()
