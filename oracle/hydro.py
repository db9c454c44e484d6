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
* ``bbpgd_dense``: Algorithm 1 on an explicit M, step for step as the C
  oracle's ``orc_bbpgd`` (BB1/BB2/alternating step sizes, a non-positive
  denominator keeps the previous step, a non-positive g0^T M g0 falls back
  to 1 / max of a given diagonal).

Pins (tests/test_oracle_hydro.py): the equal-radius Rotne-Prager closed
form (both branches), continuity at r = a_i + a_j and r = |a_i - a_j|, the
Oseen far field, positive definiteness, the two-sphere sedimentation
velocities, ``bbpgd_dense`` against the C oracle on the dry mobility, and
KKT plus brute-force active sets with the RPY mobility.
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


def self_diag(s, c):
    """Diagonal of D^T Mob_self D (the particles' own mobility blocks), used
    by the fallback initial step of a solve behind a general mobility."""
    from . import M_diag
    return M_diag(s, c)
