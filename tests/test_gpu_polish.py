"""GPU parity of the active-set polish (sc_polish_lcp) against the oracle's.

The polish is not in the paper: it takes the active set A = {gamma > 0} of a
converged iterate of Algorithm 1, solves M_AA gamma_A = -q_A exactly (to the
CG tolerance), sets gamma = 0 off A and moves violators (gamma < 0 in A,
g < 0 off A) between passes, like the oracle's `polish`. Where M is SPD the
LCP solution is unique, so the polished gamma must equal the oracle's
polished gamma to the CG tolerance times the conditioning; where M is only
semidefinite (overlapping spheres) the polish may fail, and then returns
its input unchanged with the input's g.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _sc():
    import paper_1909_06623_amd as sc
    return sc


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _setup(s):
    sc = _sc()
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box), lo=tuple(s.lo), periodic=bool(s.periodic))
    u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
    con = sc.build_contacts(P, box, s.delta, u_nc, s.dt)
    return P, con


@pytest.mark.parametrize("op", [1, 2])
@pytest.mark.parametrize("name", ["rods4000", "mixed"])
def test_polish_equals_the_oracle_polish(name, op):
    sc = _sc()
    s = (W.rods(4000, seed=44) if name == "rods4000"
         else W.rods_and_spheres(2500, 500, seed=45))
    _say(f"polish {name} op={op}")
    P, con = _setup(s)
    c, u_orc, q = O.setup(s)
    pm = con.canonical_order().cpu().numpy()
    gam, g, st, _, _ = sc.solve_lcp(P, con, tol=1e-6, op=op)
    assert st["status"] == 0
    gp, gg, stp, f_c, u_c = sc.polish_lcp(P, con, gam, tol=1e-13, want_fc=True, op=op)
    assert stp["status"] == 0 and stp["mvops"] >= 1 and stp["iters"] > 0
    go, _, sto = O.bbpgd(s, c, q, tol=1e-6)
    gpo, ggo, passes = O.polish(s, c, q, go)
    assert passes >= 1
    gp_o = gp.cpu().numpy()[pm]
    # the same unique LCP solution: relative error at the CG tolerance's level
    rel = np.linalg.norm(gp_o - gpo) / np.linalg.norm(gpo)
    _say(f"  {stp['mvops']} passes, {stp['iters']} CG iterations, |A| {stp['n_active']}, "
         f"residual {stp['residual']:.2e}, rel gamma err vs oracle polish {rel:.2e}")
    assert rel <= 1e-10
    assert stp["n_active"] == int(np.sum(gpo > 0))
    np.testing.assert_array_equal(gp_o > 0, gpo > 0)
    np.testing.assert_allclose(gg.cpu().numpy()[pm], ggo, rtol=0,
                               atol=1e-9 * max(1.0, np.abs(ggo).max()))
    # KKT of the returned point: the residual the stats report, and g, D gamma
    gpn, ggn = gp.cpu().numpy(), gg.cpu().numpy()
    assert np.all(gpn >= 0.0)
    assert abs(np.linalg.norm(np.minimum(gpn, ggn)) - stp["residual"]) <= 1e-12 + 1e-9 * \
        stp["residual"]
    F = O.D_apply(s.n, c, gpo)
    np.testing.assert_allclose(f_c.cpu().numpy(), F, rtol=0, atol=1e-9 * np.abs(F).max())


def test_polish_moves_a_wrong_active_set():
    """Start from a perturbed iterate whose active set is wrong in a few
    places (some active contacts zeroed, some inactive ones made positive):
    the passes move the violators and reach the oracle's polished solution."""
    sc = _sc()
    s = W.rods(3000, seed=46)
    _say("polish from a wrong active set")
    P, con = _setup(s)
    c, u_orc, q = O.setup(s)
    pm = con.canonical_order().cpu().numpy()
    gam, g, st, _, _ = sc.solve_lcp(P, con, tol=1e-8)
    x = gam.cpu().numpy().copy()
    act = np.flatnonzero(x > 0)
    ina = np.flatnonzero(x == 0)
    rng = np.random.default_rng(4646)
    assert act.size > 20 and ina.size > 20
    x[rng.choice(act, 10, replace=False)] = 0.0
    x[rng.choice(ina, 10, replace=False)] = 1e-3
    gp, gg, stp, _, _ = sc.polish_lcp(P, con, torch.from_numpy(x).cuda(), tol=1e-13)
    go, _, _ = O.bbpgd(s, c, q, tol=1e-8)
    gpo, _, _ = O.polish(s, c, q, go)
    _say(f"  {stp['mvops']} passes, status {stp['status']}")
    assert stp["status"] == 0 and stp["mvops"] >= 2
    rel = np.linalg.norm(gp.cpu().numpy()[pm] - gpo) / np.linalg.norm(gpo)
    assert rel <= 1e-10


def test_polish_on_semidefinite_spheres_returns_a_valid_point():
    """Overlapping spheres make M singular: the polished point, if the polish
    succeeds, satisfies the LCP (gamma >= 0, g >= 0 up to rounding,
    complementarity); if it does not, the input comes back with its own g."""
    sc = _sc()
    s = W.workload(1)
    _say("polish spheres1000 (semidefinite M)")
    P, con = _setup(s)
    gam, g, st, _, _ = sc.solve_lcp(P, con, tol=1e-9)
    gp, gg, stp, _, _ = sc.polish_lcp(P, con, gam, tol=1e-13, max_pass=5)
    gpn, ggn = gp.cpu().numpy(), gg.cpu().numpy()
    _say(f"  status {stp['status']}, {stp['mvops']} passes, residual {stp['residual']:.2e}")
    assert stp["status"] in (0, 1)
    if stp["status"] == 0:
        assert np.all(gpn >= 0.0)
        scale = np.abs(ggn).max()
        assert ggn.min() >= -1e-9 * scale
        assert stp["residual"] <= 1e-9 * scale
    else:
        assert torch.equal(gp, gam)
        np.testing.assert_allclose(ggn, g.cpu().numpy(), rtol=0,
                                   atol=1e-12 * np.abs(ggn).max())


def test_polish_edge_cases():
    """No contacts; an all-zero input (every contact inactive: the first pass
    takes the contacts with q < 0 into A)."""
    sc = _sc()
    s = W.rods(400, seed=47, min_side=2.2)
    P, con = _setup(s)
    assert con.count > 0
    z = torch.zeros(con.count, dtype=torch.float64, device="cuda")
    gp, gg, stp, _, _ = sc.polish_lcp(P, con, z, tol=1e-13)
    c, u_orc, q = O.setup(s)
    go, _, _ = O.bbpgd(s, c, q, tol=1e-10)
    gpo, _, _ = O.polish(s, c, q, go)
    pm = con.canonical_order().cpu().numpy()
    assert stp["status"] == 0 and stp["mvops"] >= 2
    assert np.linalg.norm(gp.cpu().numpy()[pm] - gpo) <= 1e-10 * np.linalg.norm(gpo)
    # a system without contacts
    far = W.rods(50, seed=48, min_side=40.0)
    P2, con2 = _setup(far)
    if con2.count == 0:
        gp2, gg2, st2, f2, u2 = sc.polish_lcp(P2, con2, torch.zeros(0, dtype=torch.float64,
                                                                    device="cuda"),
                                              want_fc=True)
        assert st2["status"] == 0 and gp2.numel() == 0
        assert float(f2.abs().max()) == 0.0
