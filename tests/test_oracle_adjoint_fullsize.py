"""The oracle's adjoint on the 100,000-rod adjoint configuration (loss
L = 1/2 ||D gamma||^2, the contact forces and torques) against central
differences of the exact LCP solution, h = 1e-6, on 20 random unit
directions in q and 20 in the centres.

The solution is exact on its active set A: gamma_A = -M_AA^-1 q_A, gamma = 0
off A (Algorithm 1 to 1e-6, then the active-set polish). A direction is
redrawn (and counted) when the pair set at c +- h V differs from the one at
c, or when gamma +- on A is not positive or g +- off A not positive (the
active set would change).

The two perturbed solutions are not solved for separately: their
difference is formed from the two perturbed systems themselves, by one
solve of the averaged system (M+ gamma+ = -q+ and M- gamma- = -q- give
Mbar dgamma = -(q+ - q-) - dM (gamma+ + gamma-) with Mbar, dM the half sum
and half difference of M+ and M-, and gamma+ + gamma- = 2 gamma + O(h^2)).
Subtracting two solutions, each accurate only to about cond(M_AA) times
the rounding of its right-hand side, would lose the O(h) difference in the
rounding of two O(1) vectors. L(+) - L(-) is formed likewise as
(F+ - F-) . (F+ + F-) / 2 with F+ - F- = Dbar dgamma + 2 dD gamma from the
averaged and half-differenced contact frames. In the centres the applied
displacement is the one the rounded positions actually carry. M+ and M-
are the oracle's assembled M at those centres, and the solves are
Jacobi-preconditioned conjugate gradients on A.

What remains in the centre directions is the rounding of the perturbed
geometry (Phi, n and tau at c +- h V, about 1e-16 of each), which the solve
amplifies by cond(M_AA) and the difference quotient by 1 / h: it shrinks
about tenfold when h grows tenfold, which the first directions repeated at
h = 1e-5 show (a wrong gradient would not shrink).

By default 3 + 3 directions run (the CPU suite's time); SC_FD_FULL=1 runs
the configuration's 20 + 20.

The pins: the q-directions, where M_AA is the same on both sides, test the
adjoint's transpose solve (dL/dq = -w with M_AA w = D^T F_c on A) against
forward solves with other right-hand sides; the centre directions test the
geometric terms (the derivatives of n, tau and Phi under moving centres)
against the oracle's own contact geometry evaluated at moved centres."""
import dataclasses
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

H = 1e-6
# 20 + 20 directions (the adjoint configuration's count) with SC_FD_FULL=1;
# by default 3 + 3, so that the CPU suite stays within a few minutes
NDIR = 20 if os.environ.get("SC_FD_FULL") == "1" else 3
NSCALE = 5 if NDIR == 20 else 2


def _threads():
    return max(1, min(8, os.cpu_count() or 1))


def _cg(A, b, rtol=1e-14):
    """Jacobi-preconditioned conjugate gradients on the SPD sparse A, to
    ||r|| <= rtol ||b||."""
    import scipy.sparse.linalg as spla
    d = A.diagonal()
    pre = spla.LinearOperator(A.shape, matvec=lambda x: x / d)
    x, info = spla.cg(A, b, rtol=rtol, atol=0.0, maxiter=20000, M=pre)
    assert info == 0, info
    return x


def _block(M, idx):
    import scipy.sparse as sp
    return sp.csr_matrix(M[idx][:, idx])


def _fd_q(base, v):
    s, c, q, gam, act, F0, M0 = (base[k] for k in ("s", "c", "q", "gam", "act", "F0", "M0"))
    idx = np.flatnonzero(act)
    dg = np.zeros(c.nc)
    dg[idx] = _cg(base["Maa"], -2.0 * H * v[idx])
    for sg in (1, -1):
        gs = gam + sg * 0.5 * dg
        gg = M0 @ gs + q + sg * H * v
        if not (np.all(gs[idx] > 0.0) and np.all(gg[~act] > 0.0)):
            return None
    return float(np.sum(O.D_apply(s.n, c, dg) * F0)) / (2.0 * H)


def _fd_c(base, V, h):
    s, c, u, gam, act = (base[k] for k in ("s", "c", "u", "gam", "act"))
    idx = np.flatnonzero(act)
    side = []
    for sg in (1, -1):
        pos = s.pos + sg * h * V
        sp_ = dataclasses.replace(s, pos=pos)
        c2 = O.find_contacts(sp_)
        if not (np.array_equal(c2.i, c.i) and np.array_equal(c2.j, c.j)):
            return None
        side.append((pos, c2, O.build_q(c2, u, s.dt), O.M_matrix(sp_, c2)))
    (pp, cp, qp, Mp), (pm, cm, qm, Mm) = side
    rhs = -(qp - qm) - (Mp - Mm) @ gam           # - dM (2 gamma), dM = (M+ - M-) / 2
    dg = np.zeros(c.nc)
    dg[idx] = _cg(_block(0.5 * (Mp + Mm), idx), rhs[idx])
    for sg, (_, cX, qX, MX) in zip((1, -1), side):
        gs = gam + sg * 0.5 * dg
        gg = MX @ gs + qX
        if not (np.all(gs[idx] > 0.0) and np.all(gg[~act] > 0.0)):
            return None
    avg = dataclasses.replace(c, nrm=0.5 * (cp.nrm + cm.nrm), tau_i=0.5 * (cp.tau_i + cm.tau_i),
                              tau_j=0.5 * (cp.tau_j + cm.tau_j))
    dif = dataclasses.replace(c, nrm=0.5 * (cp.nrm - cm.nrm), tau_i=0.5 * (cp.tau_i - cm.tau_i),
                              tau_j=0.5 * (cp.tau_j - cm.tau_j))
    dF = O.D_apply(s.n, avg, dg) + 2.0 * O.D_apply(s.n, dif, gam)
    Fsum = O.D_apply(s.n, cp, gam + 0.5 * dg) + O.D_apply(s.n, cm, gam - 0.5 * dg)
    fd = float(np.sum(dF * Fsum)) / (4.0 * h)
    v_eff = ((pp - s.pos) - (pm - s.pos)) / (2.0 * h)   # the displacement the rounding kept
    return fd, v_eff


@pytest.mark.timeout(1800)
def test_adjoint_against_central_differences_at_100k_rods():
    s = W.workload(4)
    with O.threads(_threads()):
        c, u, q = O.setup(s)
        go, _, st = O.bbpgd(s, c, q)
        assert st.status == 0
        gam, _, passes = O.polish(s, c, q, go)
        assert passes >= 1
        act = gam > 0.0
        F0 = O.D_apply(s.n, c, gam)
        dq, dpos, _ = O.adjoint(s, c, q, u, gam, dL_dF=F0, method="cg")
        M0 = O.M_matrix(s, c)
        base = dict(s=s, c=c, u=u, q=q, gam=gam, act=act, F0=F0, M0=M0,
                    Maa=_block(M0, np.flatnonzero(act)))
        rng = np.random.default_rng(2024)
        errs = {"q": [], "c": [], "c_typ": [], "c_1e-5": []}
        # the size of a directional derivative along a random unit direction
        # of the centres: a direction along which the gradient happens to be
        # small makes the relative error large without the difference being
        # any worse, so the centre errors are also taken relative to this
        typ = float(np.linalg.norm(dpos)) / np.sqrt(dpos.size)
        redrawn = {"q": 0, "c": 0}
        while len(errs["q"]) < NDIR:
            v = rng.standard_normal(c.nc)
            v /= np.linalg.norm(v)
            fd = _fd_q(base, v)
            if fd is None:
                redrawn["q"] += 1
                continue
            an = float(np.dot(dq, v))
            errs["q"].append(abs(fd - an) / abs(an))
        while len(errs["c"]) < NDIR and redrawn["c"] < 3 * NDIR:
            V = rng.standard_normal((s.n, 3))
            V /= np.linalg.norm(V)
            r = _fd_c(base, V, H)
            if r is None:
                redrawn["c"] += 1
                continue
            fd, v_eff = r
            an = float(np.sum(dpos * v_eff))
            errs["c"].append(abs(fd - an) / abs(an))
            errs["c_typ"].append(abs(fd - an) / typ)
            if len(errs["c_1e-5"]) < NSCALE:
                r5 = _fd_c(base, V, 10.0 * H)
                if r5 is not None:
                    an5 = float(np.sum(dpos * r5[1]))
                    errs["c_1e-5"].append((errs["c"][-1], abs(r5[0] - an5) / abs(an5)))
    rq, rc, rt = np.array(errs["q"]), np.array(errs["c"]), np.array(errs["c_typ"])
    print(f"[fd] q-directions: {len(rq)} used, {redrawn['q']} redrawn; relative error median "
          f"{np.median(rq):.2e}, max {rq.max():.2e}", flush=True)
    print(f"[fd] centre directions: {len(rc)} used, {redrawn['c']} redrawn; relative error "
          f"median {np.median(rc):.2e}, max {rc.max():.2e} (relative to the typical "
          f"directional derivative: median {np.median(rt):.2e}, max {rt.max():.2e}); the same "
          f"directions at h = 1e-6 "
          f"and 1e-5: {[(f'{a:.1e}', f'{b:.1e}') for a, b in errs['c_1e-5']]}", flush=True)
    assert len(rq) == NDIR and len(rc) == NDIR
    assert rq.max() <= 1e-9
    assert np.median(rc) <= 1e-5 and np.median(rt) <= 1e-5 and rt.max() <= 1e-4
    # the remainder is rounding amplified by 1 / h, not a wrong gradient
    pairs = np.array(errs["c_1e-5"])
    assert len(pairs) >= 1 and np.median(pairs[:, 1]) <= np.median(pairs[:, 0]) / 3.0
