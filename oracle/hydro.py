"""Non-diagonal mobilities and Algorithm 1 behind a general mobility (test
infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module).

The collision solve needs the mobility only through products U = Mob F with
Mob symmetric positive definite (section 2 defines Mob as the dense SPD map
from forces and torques to velocities; in section 3.3 each product M x is
one mobility problem for the contact force D x; the abstract and section 1
name the Rotne-Prager-Yamakawa tensor as one such mobility, and section 8
allows any mobility solver that keeps Mob SPD). This module holds:

* ``rpy_block``: the translational RPY coupling of two spheres of radii a_i,
  a_j, in the form of Zuk, Wajnryb, Mizerski and Szymczak (J. Fluid Mech.
  2014) for unequal radii, with its two overlap branches;
* ``rpy_mobility``: the dense 6N x 6N mobility of N spheres in unbounded
  fluid: RPY couplings between translations, the single-sphere rotational
  mobility 1/(8 pi mu a^3) on the diagonal, no rotational couplings between
  spheres (a reading: this keeps the matrix SPD, being block diagonal in
  translations and rotations with an SPD translational block);
  ``rpy_dense`` evaluates the same formulas on arrays of all pairs;
* ``rpy_grad``: the centre gradient of a^T Mob(c) f for the RPY mobility,
  from the derivatives of the coefficient functions of each branch;
* ``adjoint_rpy``: the implicit adjoint of the converged LCP behind the RPY
  mobility (not in the paper), on the explicit M;
* ``bbpgd_dense``: Algorithm 1 on an explicit M, step for step as the C
  oracle's ``orc_bbpgd`` (BB1/BB2/alternating step sizes, a non-positive
  denominator keeps the previous step, a non-positive g0^T M g0 falls back
  to 1 / max of a given diagonal).

Pins (tests/test_oracle_hydro.py): the equal-radius Rotne-Prager closed
form (both branches), continuity at r = a_i + a_j and r = |a_i - a_j|, the
Oseen far field, positive definiteness, the two-sphere sedimentation
velocities, ``bbpgd_dense`` against the C oracle on the dry mobility,
KKT plus brute-force active sets with the RPY mobility, ``rpy_grad``
against central differences, and ``adjoint_rpy`` against central
differences of polished solves (parity unpinned by the paper: the adjoint
is not in it).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


def rpy_block(d, ai, aj, mu=1.0):
    """3x3 translational RPY mobility coupling sphere i (radius ai) to a
    force on sphere j (radius aj), d = c_i - c_j (i != j). Two coincident
    spheres of equal radius couple like one sphere (the matrix is then only
    semidefinite)."""
    r = float(np.sqrt(d @ d))
    eye = np.eye(3)
    if r <= abs(ai - aj):
        return eye / (6.0 * math.pi * mu * max(ai, aj))
    e = d / r
    outer = np.outer(e, e)
    if r > ai + aj:
        c = 1.0 / (8.0 * math.pi * mu * r)
        s2 = ai * ai + aj * aj
        return c * ((1.0 + s2 / (3.0 * r * r)) * eye + (1.0 - s2 / (r * r)) * outer)
    dd = (ai - aj) ** 2
    pre = 1.0 / (6.0 * math.pi * mu * ai * aj)
    a = (16.0 * r ** 3 * (ai + aj) - (dd + 3.0 * r * r) ** 2) / (32.0 * r ** 3)
    b = 3.0 * (dd - r * r) ** 2 / (32.0 * r ** 3)
    return pre * (a * eye + b * outer)


def rpy_mobility(pos, radius, mu=1.0):
    """Dense 6N x 6N mobility (rows/cols per particle: U xyz, Omega xyz)."""
    pos = np.asarray(pos, dtype=np.float64)
    radius = np.asarray(radius, dtype=np.float64)
    n = pos.shape[0]
    Mob = np.zeros((6 * n, 6 * n))
    for i in range(n):
        ai = radius[i]
        Mob[6 * i:6 * i + 3, 6 * i:6 * i + 3] = np.eye(3) / (6.0 * math.pi * mu * ai)
        Mob[6 * i + 3:6 * i + 6, 6 * i + 3:6 * i + 6] = np.eye(3) / (8.0 * math.pi * mu * ai ** 3)
        for j in range(n):
            if j != i:
                Mob[6 * i:6 * i + 3, 6 * j:6 * j + 3] = rpy_block(pos[i] - pos[j], ai, radius[j], mu)
    return Mob


def rpy_dense(pos, radius, mu=1.0):
    """``rpy_mobility`` with the pair formulas evaluated on arrays of all
    pairs at once (same branches, same expressions)."""
    pos = np.asarray(pos, dtype=np.float64)
    radius = np.asarray(radius, dtype=np.float64)
    n = pos.shape[0]
    d = pos[:, None, :] - pos[None, :, :]
    r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
    ai = radius[:, None] * np.ones((1, n))
    aj = radius[None, :] * np.ones((n, 1))
    pos_r = r > 0.0
    rs = np.where(pos_r, r, 1.0)
    e = np.where(pos_r[..., None], d / rs[..., None], 0.0)
    far = r > ai + aj
    inside = r <= np.abs(ai - aj)
    s2 = ai * ai + aj * aj
    c = 1.0 / (8.0 * math.pi * mu * rs)
    a_far = c * (1.0 + s2 / (3.0 * rs * rs))
    b_far = c * (1.0 - s2 / (rs * rs))
    dd = (ai - aj) ** 2
    pre = 1.0 / (6.0 * math.pi * mu * ai * aj)
    a_ov = pre * (16.0 * rs ** 3 * (ai + aj) - (dd + 3.0 * rs * rs) ** 2) / (32.0 * rs ** 3)
    b_ov = pre * 3.0 * (dd - rs * rs) ** 2 / (32.0 * rs ** 3)
    a_in = 1.0 / (6.0 * math.pi * mu * np.maximum(ai, aj))
    A = np.where(far, a_far, np.where(inside, a_in, a_ov))
    B = np.where(far, b_far, np.where(inside, 0.0, b_ov))
    blk = A[..., None, None] * np.eye(3) + B[..., None, None] * (e[..., :, None] * e[..., None, :])
    idx = np.arange(n)
    blk[idx, idx] = np.eye(3) / (6.0 * math.pi * mu * radius)[:, None, None]
    Mob = np.zeros((6 * n, 6 * n))
    t = (6 * idx[:, None] + np.arange(3)).ravel()
    Mob[np.ix_(t, t)] = blk.transpose(0, 2, 1, 3).reshape(3 * n, 3 * n)
    rr = t + 3
    Mob[rr, rr] = np.repeat(1.0 / (8.0 * math.pi * mu * radius ** 3), 3)
    return Mob


def rpy_apply(pos, radius, F, mu=1.0):
    """U = Mob F for F [n][6], pair by pair (no dense matrix)."""
    pos = np.asarray(pos, dtype=np.float64)
    radius = np.asarray(radius, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    n = pos.shape[0]
    U = np.zeros((n, 6))
    for i in range(n):
        ai = radius[i]
        acc = F[i, :3] / (6.0 * math.pi * mu * ai)
        for j in range(n):
            if j != i:
                acc = acc + rpy_block(pos[i] - pos[j], ai, radius[j], mu) @ F[j, :3]
        U[i, :3] = acc
        U[i, 3:] = F[i, 3:] / (8.0 * math.pi * mu * ai ** 3)
    return U


def _rpy_coefficients(r, ai, aj, mu):
    """A, Bt and their derivatives in r for M = A I + Bt d d^T (d the
    unnormalised separation, r = |d|), per branch; arrays of pairs."""
    k8 = 1.0 / (8.0 * math.pi * mu)
    k6 = 1.0 / (6.0 * math.pi * mu)
    S = ai * ai + aj * aj
    far = r > ai + aj
    inside = r <= np.abs(ai - aj)
    rs = np.where(r > 0.0, r, 1.0)
    # separated: A = k8 (1/r + S/(3 r^3)), Bt = k8 (1/r^3 - S/r^5)
    A_f = k8 * (1.0 / rs + S / (3.0 * rs ** 3))
    dA_f = k8 * (-1.0 / rs ** 2 - S / rs ** 4)
    B_f = k8 * (1.0 / rs ** 3 - S / rs ** 5)
    dB_f = k8 * (-3.0 / rs ** 4 + 5.0 * S / rs ** 6)
    # overlapping: A = pre (sigma/2 - T^2/(32 r^3)), T = delta^2 + 3 r^2,
    # Bt = 3 pre (delta^2 - r^2)^2 / (32 r^5)
    pre = k6 / (ai * aj)
    d2 = (ai - aj) ** 2
    T = d2 + 3.0 * rs * rs
    A_o = pre * ((ai + aj) / 2.0 - T * T / (32.0 * rs ** 3))
    dA_o = -pre * 3.0 * T * (rs * rs - d2) / (32.0 * rs ** 4)
    B_o = pre * 3.0 * (d2 - rs * rs) ** 2 / (32.0 * rs ** 5)
    dB_o = pre * 3.0 * (d2 - rs * rs) * (rs * rs - 5.0 * d2) / (32.0 * rs ** 6)
    A = np.where(far, A_f, np.where(inside, k6 / np.maximum(ai, aj), A_o))
    dA = np.where(far, dA_f, np.where(inside, 0.0, dA_o))
    Bt = np.where(far, B_f, np.where(inside, 0.0, B_o))
    dB = np.where(far, dB_f, np.where(inside, 0.0, dB_o))
    return A, dA, Bt, dB


def rpy_grad(pos, radius, a, f, mu=1.0):
    """g[k] = d/dc_k of a^T Mob(c) f for the RPY mobility (a, f: [n][6];
    only the translational couplings depend on the centres). Each ordered
    pair (k, j), d = c_k - c_j, contributes the gradient in d of
    a_k^T M(d) f_j + a_j^T M(d) f_k."""
    pos = np.asarray(pos, dtype=np.float64)
    radius = np.asarray(radius, dtype=np.float64)
    at = np.asarray(a, dtype=np.float64)[:, :3]
    ft = np.asarray(f, dtype=np.float64)[:, :3]
    n = pos.shape[0]
    d = pos[:, None, :] - pos[None, :, :]
    r = np.sqrt(np.einsum("kjc,kjc->kj", d, d))
    ai = radius[:, None] * np.ones((1, n))
    aj = radius[None, :] * np.ones((n, 1))
    A, dA, Bt, dB = _rpy_coefficients(r, ai, aj, mu)
    rs = np.where(r > 0.0, r, 1.0)
    e = np.where((r > 0.0)[..., None], d / rs[..., None], 0.0)
    ak, fk = at[:, None, :], ft[:, None, :]
    aj_, fj = at[None, :, :], ft[None, :, :]
    P = np.einsum("kjc,kjc->kj", ak * np.ones_like(d), fj * np.ones_like(d)) + \
        np.einsum("kjc,kjc->kj", aj_ * np.ones_like(d), fk * np.ones_like(d))
    akd = np.einsum("kjc,kjc->kj", ak * np.ones_like(d), d)
    ajd = np.einsum("kjc,kjc->kj", aj_ * np.ones_like(d), d)
    fkd = np.einsum("kjc,kjc->kj", fk * np.ones_like(d), d)
    fjd = np.einsum("kjc,kjc->kj", fj * np.ones_like(d), d)
    Q = akd * fjd + ajd * fkd
    g = (dA * P + dB * Q)[..., None] * e + Bt[..., None] * (
        fjd[..., None] * ak + akd[..., None] * fj + fkd[..., None] * aj_ + ajd[..., None] * fk)
    idx = np.arange(n)
    g[idx, idx] = 0.0
    return g.sum(axis=1)


def adjoint_rpy(s, c, gamma, dL_dgamma=None, dL_dF=None, mu=1.0):
    """Implicit adjoint of the converged LCP with the RPY mobility (not in
    the paper; the dry-mobility derivation with Mob a function of the
    centres). With b = dL/dgamma + D^T dL/dF, M_AA w_A = b_A on A = {gamma >
    0}; dL/dq = -w; the centre gradient is the per-contact geometric part
    with V_w = Mob D w and U = Mob (F_ext + D gamma), minus
    d/dc [(D w)^T Mob(c) (D gamma + F_ext)]. Returns (dL_dq, dL_dpos, w)."""
    from . import D_apply, D_matrix, DT_apply, adjoint_positions
    n = s.n
    rad = s.radius if s.hydro_radius is None else s.hydro_radius
    gamma = np.asarray(gamma, dtype=np.float64)
    Mob = rpy_dense(s.pos, rad, mu)
    M = contact_matrix(D_matrix(n, c), Mob)
    b = np.zeros(c.nc) if dL_dgamma is None else np.asarray(dL_dgamma, dtype=np.float64).copy()
    if dL_dF is not None:
        b = b + DT_apply(c, dL_dF)
    act = gamma > 0.0
    idx = np.flatnonzero(act)
    w = np.zeros(c.nc)
    if idx.size:
        w[idx] = np.linalg.solve(M[np.ix_(idx, idx)], b[idx])
    Fc = D_apply(n, c, gamma)
    Fw = D_apply(n, c, w)
    Ftot = Fc + s.f_ext
    Vw = (Mob @ Fw.ravel()).reshape(n, 6)
    U = (Mob @ Ftot.ravel()).reshape(n, 6)
    out = adjoint_positions(s, c, gamma, w, dL_dF, Vw, U)
    out = out - rpy_grad(s.pos, rad, Fw, Ftot, mu)
    return -w, out, w


def contact_matrix(D, Mob):
    """M = D^T Mob D, dense (D: 6N x nc, sparse or dense)."""
    if hasattr(D, "toarray"):
        X = np.asarray(D.T @ Mob)          # nc x 6N
        return np.asarray((D.T @ X.T).T)   # (D^T (D^T Mob)^T)^T = D^T Mob D
    Dd = np.asarray(D)
    return Dd.T @ Mob @ Dd


@dataclasses.dataclass
class DenseStats:
    status: int          # 0 converged, 1 not within max_iter, 3 non-finite
    iters: int
    mvops: int
    res: float
    n_active: int
    n_degenerate: int
    alpha: float


def _res(gamma, g):
    m = np.minimum(gamma, g)
    return math.sqrt(float(m @ m))


def bbpgd_dense(M, q, diag, gamma0=None, tol=1e-6, max_iter=100000, bb=1):
    """Algorithm 1 with products by the explicit M. ``diag`` is the positive
    diagonal used by the fallback initial step. Returns (gamma, g, stats)."""
    M = np.asarray(M, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    nc = q.shape[0]
    gamma = np.zeros(nc) if gamma0 is None else np.asarray(gamma0, dtype=np.float64).copy()
    ndegen = 0
    alpha = 0.0
    iters = 0
    # g0 = M gamma0 + q
    g = M @ gamma + q
    mvops = 1
    res = _res(gamma, g)
    status = 0
    if not math.isfinite(res):
        status = 3
    elif res >= tol:
        # initial step size g0^T g0 / g0^T M g0
        t = M @ g
        mvops += 1
        num, den = float(g @ g), float(g @ t)
        if den > 0.0 and math.isfinite(den) and math.isfinite(num):
            alpha = num / den
        else:
            mx = float(np.max(diag)) if nc else 0.0
            alpha = 1.0 / mx if mx > 0.0 else 1.0
            ndegen += 1
        status = 1
        for j in range(1, max_iter + 1):
            gamma_prev, g_prev = gamma, g
            # projected descent step
            gamma = np.maximum(gamma_prev - alpha * g_prev, 0.0)
            # new gradient
            g = M @ gamma + q
            mvops += 1
            iters = j
            res = _res(gamma, g)
            if not math.isfinite(res):
                status = 3
                break
            if res < tol:
                status = 0
                break
            # BB step size
            s = gamma - gamma_prev
            y = g - g_prev
            ss, sy, yy = float(s @ s), float(s @ y), float(y @ y)
            use_bb2 = bb == 2 or (bb == 3 and j % 2 == 0)
            num, den = (sy, yy) if use_bb2 else (ss, sy)
            if den > 0.0 and num > 0.0 and math.isfinite(num) and math.isfinite(den):
                alpha = num / den
            else:
                ndegen += 1
    st = DenseStats(status, iters, mvops, res, int(np.count_nonzero(gamma > 0.0)), ndegen, alpha)
    return gamma, g, st


def polish_dense(M, q, gamma, max_pass=50):
    """Exact LCP solution near ``gamma`` on the explicit M: solve the active
    block, move violators, repeat. Returns (gamma, g, passes), passes = -1 if
    it did not settle."""
    act = np.asarray(gamma) > 0.0
    q = np.asarray(q, dtype=np.float64)
    gam = np.zeros(q.size)
    for p in range(max_pass):
        gam = np.zeros(q.size)
        idx = np.flatnonzero(act)
        if idx.size:
            gam[idx] = np.linalg.solve(M[np.ix_(idx, idx)], -q[idx])
        g = M @ gam + q
        leave = act & (gam < 0.0)
        join = (~act) & (g < 0.0)
        if not leave.any() and not join.any():
            return gam, g, p + 1
        act = (act & ~leave) | join
    return gam, M @ gam + q, -1


def self_diag(s, c):
    """Diagonal of D^T Mob_self D (the particles' own mobility blocks), used
    by the fallback initial step of a solve behind a general mobility."""
    from . import M_diag
    return M_diag(s, c)
