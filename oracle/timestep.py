"""First-order Euler time stepping of the collision-constrained suspension:
the outer loop of section 3.2 (test infrastructure: only the tests, the
smoke check and the benchmark's CPU leg use the oracle).

One step, in the paper's order:

1. U_nc = Mob F_ext at the current configuration (the dry mobility, or the
   RPY mobility of ``oracle.hydro``).
2. The close-pair set A(C^k, delta), its contact frames and q
   (``find_contacts``, ``build_q``; LCP LCPdef).
3. The LCP solved by Algorithm 1 (``bbpgd``), started from zero or, with
   ``warm``, from the previous step's gamma of the same pairs (0 for new
   pairs); then U_c = Mob D gamma.
4. C^{k+1} = C^k + dt G (U_nc + U_c) (Eq. time-step): centres move by U;
   the orientation quaternion theta = (s, p) moves by Psi(theta) Omega with
   Psi = 1/2 [-p^T; s I - [p]x] (the quaternion kinematics of section 2) and
   is then normalised (the paper's linear update leaves the norm free; a
   rotation needs a unit quaternion); a rod's axis is R(theta) e_z.

Pinned (tests/test_oracle_timestep.py): free translation; free rotation
about a fixed axis against the closed form (each step turns the axis by
2 atan(|Omega| dt / 2), the angle of the normalised quaternion update);
the quaternion/axis round trip; two spheres pushed head-on stop exactly
touching (Phi linear along the line of centres, so the converged LCP closes
the gap); two spheres dragged past each other (the paper's two-sphere
experiment, with the dry mobility) keep their centre of mass fixed and go
through its stages: a close pair with zero force, a positive force, then
zero force again while still close, then no pair.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import D_apply, bbpgd, build_q, find_contacts, mobility


def quat_from_axis(axis):
    """Unit quaternions (s, p) of the shortest rotations taking e_z to each
    unit axis (the half turn about x for -e_z)."""
    axis = np.asarray(axis, dtype=np.float64)
    q = np.empty((axis.shape[0], 4))
    for k, a in enumerate(axis):
        s = 1.0 + a[2]
        p = np.array([-a[1], a[0], 0.0])
        if s < 1e-12:
            s, p = 0.0, np.array([1.0, 0.0, 0.0])
        v = np.concatenate([[s], p])
        q[k] = v / np.sqrt(v @ v)
    return q


def rotation(q):
    """Rotation matrix of the unit quaternion q = (s, p):
    (s^2 - p.p) I + 2 p p^T + 2 s [p]x."""
    s, p = q[0], q[1:]
    px = np.array([[0.0, -p[2], p[1]], [p[2], 0.0, -p[0]], [-p[1], p[0], 0.0]])
    return (s * s - p @ p) * np.eye(3) + 2.0 * np.outer(p, p) + 2.0 * s * px


def quat_axis(quat):
    """Body axis e_z in space for each quaternion."""
    return np.array([rotation(q)[:, 2] for q in np.asarray(quat, dtype=np.float64)])


def psi(q):
    """Psi(theta) = 1/2 [-p^T; s I - [p]x], theta_dot = Psi Omega."""
    s, p = q[0], q[1:]
    px = np.array([[0.0, -p[2], p[1]], [p[2], 0.0, -p[0]], [-p[1], p[0], 0.0]])
    return 0.5 * np.vstack([-p[None, :], s * np.eye(3) - px])


def advance(pos, quat, U, dt):
    """Eq. time-step for centres and quaternions; returns (pos, quat, axis)."""
    pos = np.asarray(pos, dtype=np.float64) + dt * U[:, :3]
    qn = np.empty_like(quat)
    for k in range(quat.shape[0]):
        v = quat[k] + dt * (psi(quat[k]) @ U[k, 3:])
        qn[k] = v / np.sqrt(v @ v)
    return pos, qn, quat_axis(qn)


@dataclasses.dataclass
class StepRecord:
    i: np.ndarray          # contacts of the step (canonical order)
    j: np.ndarray
    phi: np.ndarray
    gamma: np.ndarray
    iters: int
    mvops: int
    status: int
    U: np.ndarray          # [n,6] U_nc + U_c used for the update


def step(s, quat, prev: StepRecord | None = None, warm=True, tol=None, hydro=None, mu=1.0):
    """One step from suspension ``s`` (its pos and axis) and quaternions
    ``quat``; returns (next suspension, next quaternions, record).
    ``hydro="rpy"``: the mobility is the RPY mobility of spheres of radii
    ``s.hydro_radius`` (else ``s.radius``) and viscosity ``mu``, and the LCP
    is solved on the explicit M = D^T Mob D (``bbpgd_dense``)."""
    c = find_contacts(s)
    gamma0 = None
    if warm and prev is not None and c.nc:
        old = {(int(a), int(b)): g for a, b, g in zip(prev.i, prev.j, prev.gamma)}
        gamma0 = np.array([old.get((int(a), int(b)), 0.0) for a, b in zip(c.i, c.j)])
    if hydro == "rpy":
        from . import D_matrix, M_diag
        from .hydro import bbpgd_dense, contact_matrix, rpy_dense
        rad = s.radius if s.hydro_radius is None else s.hydro_radius
        Mob = rpy_dense(s.pos, rad, mu)
        u_nc = (Mob @ s.f_ext.ravel()).reshape(s.n, 6)
        q = build_q(c, u_nc, s.dt)
        M = contact_matrix(D_matrix(s.n, c), Mob)
        gamma, g, st = bbpgd_dense(M, q, M_diag(s, c), gamma0=gamma0,
                                   tol=s.tol if tol is None else tol)
        u_c = (Mob @ D_apply(s.n, c, gamma).ravel()).reshape(s.n, 6)
    elif hydro is None:
        u_nc = mobility(s.axis, s.mob, s.f_ext)
        q = build_q(c, u_nc, s.dt)
        gamma, g, st = bbpgd(s, c, q, gamma0=gamma0, tol=tol)
        u_c = mobility(s.axis, s.mob, D_apply(s.n, c, gamma))
    else:
        raise ValueError(f"unknown mobility {hydro!r}")
    U = u_nc + u_c
    pos, qn, axis = advance(s.pos, quat, U, s.dt)
    rec = StepRecord(c.i.copy(), c.j.copy(), c.phi.copy(), gamma, st.iters, st.mvops,
                     st.status, U)
    return dataclasses.replace(s, pos=pos, axis=axis), qn, rec


def run(s, steps, warm=True, tol=None, quat=None, hydro=None, mu=1.0):
    """``steps`` steps from ``s``; returns (final suspension, quaternions,
    records)."""
    quat = quat_from_axis(s.axis) if quat is None else np.asarray(quat, dtype=np.float64)
    recs = []
    prev = None
    for _ in range(steps):
        s, quat, prev = step(s, quat, prev, warm, tol, hydro, mu)
        recs.append(prev)
    return s, quat, recs
