"""FP64 CPU oracle for the collision-resolution path (test infrastructure).

This package is the parity checker for the HIP path: a plain, serial, obviously
correct implementation of what the path computes, written from the paper
(Yan et al., arXiv:1909.06623, section 3). Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product library never
does, and the two share no code. The arithmetic lives in ``oracle.c`` (loops in
index order, no FMA contraction); this module marshals arrays and adds the
pieces that are plain linear algebra on top of it:

* ``polish``: the exact LCP solution on a fixed active set (a dense or sparse
  direct solve of the active block, with principal pivoting on violators);
* ``adjoint``: implicit differentiation through the converged LCP on its
  active set (not in the paper; derived from its LCP statement, LCP LCPdef).

Parity status of each function is recorded in its docstring. Functions pinned
only by the tests listed there are "parity unpinned by the paper" where the
paper defers the formula to other work (rod mobility, rod D entries, adjoint).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_long)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_pair_geometry.restype = ctypes.c_int
    lib.orc_pair_geometry.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double,
                                      _dp, _dp, ctypes.c_double, ctypes.c_double,
                                      _dp, ctypes.c_int, _dp]
    lib.orc_set_threads.restype = None
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_get_threads.restype = ctypes.c_int
    lib.orc_get_threads.argtypes = []
    lib.orc_find_contacts.restype = ctypes.c_long
    lib.orc_find_contacts.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp,
                                      _dp, _dp, _dp, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_double,
                                      ctypes.c_long, _ip, _ip, _dp, _dp, _dp, _dp,
                                      _dp, _lp]
    lib.orc_mobility.restype = None
    lib.orc_mobility.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp]
    lib.orc_D_apply.restype = None
    lib.orc_D_apply.argtypes = [ctypes.c_int, ctypes.c_long, _ip, _ip, _dp, _dp,
                                _dp, _dp, _dp]
    lib.orc_DT_apply.restype = None
    lib.orc_DT_apply.argtypes = [ctypes.c_long, _ip, _ip, _dp, _dp, _dp, _dp, _dp]
    lib.orc_build_q.restype = None
    lib.orc_build_q.argtypes = [ctypes.c_long, _ip, _ip, _dp, _dp, _dp, _dp, _dp,
                                ctypes.c_double, _dp]
    lib.orc_mvop.restype = None
    lib.orc_mvop.argtypes = [ctypes.c_int, ctypes.c_long, _ip, _ip, _dp, _dp, _dp,
                             _dp, _dp, _dp, _dp]
    lib.orc_M_diag.restype = None
    lib.orc_M_diag.argtypes = [ctypes.c_long, _ip, _ip, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_bbpgd.restype = ctypes.c_int
    lib.orc_bbpgd.argtypes = [ctypes.c_int, ctypes.c_long, _ip, _ip, _dp, _dp, _dp,
                              _dp, _dp, _dp, _dp, _dp, ctypes.c_double,
                              ctypes.c_int, ctypes.c_int, _dp]
    lib.orc_contact_grad.restype = None
    lib.orc_contact_grad.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double,
                                     _dp, _dp, ctypes.c_double, ctypes.c_double,
                                     _dp, ctypes.c_int, _dp, _dp, ctypes.c_double,
                                     _dp]
    lib.orc_adjoint_positions.restype = None
    lib.orc_adjoint_positions.argtypes = [ctypes.c_int, ctypes.c_long, _dp, _dp,
                                          _dp, _dp, _dp, ctypes.c_int, _ip, _ip,
                                          _dp, _dp, _dp, _dp, _dp, ctypes.c_double,
                                          _dp]
    _lib = lib
    return lib


def set_threads(t):
    """Threads of the close-pair search and of Algorithm 1 (default 1).
    With one thread every result is that of the plain serial loops; with
    more, the contact list and every product are the same and only the sums
    over contacts are added as per-thread partial sums in thread order."""
    _load().orc_set_threads(int(t))


def get_threads():
    return int(_load().orc_get_threads())


class threads:
    """Context manager: ``with threads(8): ...`` runs the oracle on 8 threads."""

    def __init__(self, t):
        self.t = int(t)

    def __enter__(self):
        self.prev = get_threads()
        set_threads(self.t)
        return self

    def __exit__(self, *exc):
        set_threads(self.prev)
        return False


def _d(a):
    """float64 C-contiguous array and its pointer (keeps the array alive via
    the caller's reference)."""
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ------------------------------------------------------------------ geometry

def pair_geometry(ci, pi, Ri, hi, cj, pj, Rj, hj, box=(0.0, 0.0, 0.0),
                  periodic=0):
    """Minimum separation of one pair (section 3.1) and its contact frame.

    Returns dict(phi, n, s, t, tau_i, tau_j, flags). Pinned by closed-form
    distances, brute-force parameter sampling and finite differences of Phi
    under rigid motions (Eq. Dtranspose)."""
    lib = _load()
    ci, pi, cj, pj, box = map(_f64, (ci, pi, cj, pj, box))
    out = np.zeros(12)
    fl = lib.orc_pair_geometry(_d(ci), _d(pi), float(Ri), float(hi), _d(cj),
                               _d(pj), float(Rj), float(hj), _d(box),
                               int(periodic), _d(out))
    return dict(phi=out[0], n=out[1:4].copy(), s=out[4], t=out[5],
                tau_i=out[6:9].copy(), tau_j=out[9:12].copy(), flags=fl)


@dataclasses.dataclass
class Contacts:
    """Close pairs in canonical order (by i, then j; i < j)."""
    i: np.ndarray        # [nc] int32
    j: np.ndarray        # [nc] int32
    phi: np.ndarray      # [nc]
    nrm: np.ndarray      # [nc,3], unit, from i to j
    tau_i: np.ndarray    # [nc,3] = (s p_i) x n
    tau_j: np.ndarray    # [nc,3] = (t p_j) x n
    st: np.ndarray       # [nc,2] closest-point parameters (s, t)
    n_parallel: int = 0
    n_zero: int = 0

    @property
    def nc(self) -> int:
        return int(self.i.shape[0])

    def keys(self):
        """Pairs as int64 keys i * 2^32 + j, for set comparisons."""
        return self.i.astype(np.int64) * (1 << 32) + self.j.astype(np.int64)


def find_contacts(s, method="cells", delta=None):
    """Close-pair set {l : Phi_l <= delta} (section 3.2) of suspension ``s``
    by brute force (``method='brute'``, every pair) or a cell list
    (``'cells'``). Pinned: both methods agree exactly (independent searches),
    and every pair is checked against ``pair_geometry``'s pins."""
    lib = _load()
    delta = s.delta if delta is None else float(delta)
    m = 0 if method == "brute" else 1
    pos, axis, rad, hl = map(_f64, (s.pos, s.axis, s.radius, s.half_len))
    lo, box = _f64(s.lo), _f64(s.box)
    cap = max(16, 8 * s.n)
    while True:
        ci = np.empty(cap, np.int32)
        cj = np.empty(cap, np.int32)
        phi = np.empty(cap)
        nrm = np.empty((cap, 3))
        ti = np.empty((cap, 3))
        tj = np.empty((cap, 3))
        st = np.empty((cap, 2))
        fl = np.zeros(2, dtype=np.int64)
        cnt = lib.orc_find_contacts(
            m, s.n, _d(pos), _d(axis), _d(rad), _d(hl), _d(lo), _d(box),
            int(s.periodic), int(getattr(s, "walls", 0)), delta, cap, ci.ctypes.data_as(_ip),
            cj.ctypes.data_as(_ip), _d(phi), _d(nrm), _d(ti), _d(tj), _d(st),
            fl.ctypes.data_as(_lp))
        if cnt <= cap:
            break
        cap = int(cnt)
    return Contacts(ci[:cnt].copy(), cj[:cnt].copy(), phi[:cnt].copy(),
                    nrm[:cnt].copy(), ti[:cnt].copy(), tj[:cnt].copy(),
                    st[:cnt].copy(), int(fl[0]), int(fl[1]))


# ------------------------------------------------------------------ operators

def mobility(axis, mob, F):
    """U = Mob F with the per-particle dry block diag(A, B)."""
    lib = _load()
    axis, mob, F = _f64(axis), _f64(mob), _f64(F)
    U = np.empty_like(F)
    lib.orc_mobility(axis.shape[0], _d(axis), _d(mob), _d(F), _d(U))
    return U


def _cptrs(c):
    return (_i32(c.i), _i32(c.j), _f64(c.nrm), _f64(c.tau_i), _f64(c.tau_j))


def D_apply(n, c, gamma):
    """F_c = D gamma (Eq. Dmatdef), [n,6]."""
    lib = _load()
    ci, cj, nrm, ti, tj = _cptrs(c)
    gamma = _f64(gamma)
    F = np.empty((n, 6))
    lib.orc_D_apply(n, c.nc, ci.ctypes.data_as(_ip), cj.ctypes.data_as(_ip),
                    _d(nrm), _d(ti), _d(tj), _d(gamma), _d(F))
    return F


def DT_apply(c, U):
    """(D^T U)_l, the rate of change of Phi_l under rigid velocities U."""
    lib = _load()
    ci, cj, nrm, ti, tj = _cptrs(c)
    U = _f64(U)
    out = np.empty(c.nc)
    lib.orc_DT_apply(c.nc, ci.ctypes.data_as(_ip), cj.ctypes.data_as(_ip),
                     _d(nrm), _d(ti), _d(tj), _d(U), _d(out))
    return out


def build_q(c, u_nc, dt):
    """q = Phi/dt + D^T U_nc (LCP LCPdef)."""
    lib = _load()
    ci, cj, nrm, ti, tj = _cptrs(c)
    phi, u_nc = _f64(c.phi), _f64(u_nc)
    q = np.empty(c.nc)
    lib.orc_build_q(c.nc, ci.ctypes.data_as(_ip), cj.ctypes.data_as(_ip),
                    _d(phi), _d(nrm), _d(ti), _d(tj), _d(u_nc), float(dt), _d(q))
    return q


def mvop(s, c, x):
    """M x = D^T Mob D x, one matrix-free product (LCP LCPdef)."""
    lib = _load()
    ci, cj, nrm, ti, tj = _cptrs(c)
    axis, mob, x = _f64(s.axis), _f64(s.mob), _f64(x)
    out = np.empty(c.nc)
    lib.orc_mvop(s.n, c.nc, ci.ctypes.data_as(_ip), cj.ctypes.data_as(_ip),
                 _d(nrm), _d(ti), _d(tj), _d(axis), _d(mob), _d(x), _d(out))
    return out


def M_diag(s, c):
    lib = _load()
    ci, cj, nrm, ti, tj = _cptrs(c)
    axis, mob = _f64(s.axis), _f64(s.mob)
    out = np.empty(c.nc)
    lib.orc_M_diag(c.nc, ci.ctypes.data_as(_ip), cj.ctypes.data_as(_ip),
                   _d(nrm), _d(ti), _d(tj), _d(axis), _d(mob), _d(out))
    return out


def D_matrix(n, c):
    """D as a scipy sparse matrix (6n x nc): column l holds (-n, -tau_i) in
    the rows of particle i and (+n, +tau_j) in the rows of particle j."""
    import scipy.sparse as sp
    nc = c.nc
    rows = np.empty((nc, 12), np.int64)
    vals = np.empty((nc, 12))
    for a in range(3):
        rows[:, a] = 6 * c.i + a
        rows[:, 3 + a] = 6 * c.i + 3 + a
        rows[:, 6 + a] = 6 * c.j + a
        rows[:, 9 + a] = 6 * c.j + 3 + a
        vals[:, a] = -c.nrm[:, a]
        vals[:, 3 + a] = -c.tau_i[:, a]
        vals[:, 6 + a] = c.nrm[:, a]
        vals[:, 9 + a] = c.tau_j[:, a]
    cols = np.repeat(np.arange(nc), 12)
    keep = np.ones((nc, 12), bool)
    keep[c.j < 0, 6:] = False   # a wall contact has the particle's entries only
    return sp.csc_matrix((vals[keep], (rows[keep], cols[keep.ravel()])), shape=(6 * n, nc))


def mobility_matrix(axis, mob):
    """Block-diagonal Mob as a scipy sparse matrix (6n x 6n)."""
    import scipy.sparse as sp
    n = axis.shape[0]
    blocks = np.zeros((n, 6, 6))
    pp = axis[:, :, None] * axis[:, None, :]
    eye = np.eye(3)[None]
    blocks[:, :3, :3] = mob[:, 0, None, None] * pp + mob[:, 1, None, None] * (eye - pp)
    blocks[:, 3:, 3:] = mob[:, 2, None, None] * pp + mob[:, 3, None, None] * (eye - pp)
    return sp.block_diag(list(blocks), format="csr") if n else sp.csr_matrix((0, 0))


def M_matrix(s, c):
    """M = D^T Mob D assembled as a sparse matrix (for small cases)."""
    D = D_matrix(s.n, c)
    K = mobility_matrix(_f64(s.axis), _f64(s.mob))
    return (D.T @ (K @ D)).tocsr()


# ------------------------------------------------------------------ solver

@dataclasses.dataclass
class SolveStats:
    status: int
    iters: int
    mvops: int
    residual: float
    n_active: int
    n_degenerate: int
    alpha: float


def bbpgd(s, c, q, gamma0=None, tol=None, max_iter=100000, bb=1):
    """Algorithm 1 (BBPGD) from gamma0 (zero by default), stopping when
    ||min(gamma, g)||_2 < tol. Returns (gamma, g, SolveStats).

    Pinned: the two-sphere head-on closed form, the scalar-LCP MVOP counts,
    independent pairs (diagonal M), brute-force active-set enumeration on
    small systems and the KKT invariants."""
    lib = _load()
    ci, cj, nrm, ti, tj = _cptrs(c)
    axis, mob, q = _f64(s.axis), _f64(s.mob), _f64(q)
    gamma = np.zeros(c.nc) if gamma0 is None else _f64(gamma0).copy()
    g = np.empty(c.nc)
    stats = np.zeros(8)
    tol = s.tol if tol is None else float(tol)
    lib.orc_bbpgd(s.n, c.nc, ci.ctypes.data_as(_ip), cj.ctypes.data_as(_ip),
                  _d(nrm), _d(ti), _d(tj), _d(axis), _d(mob), _d(q), _d(gamma),
                  _d(g), tol, int(max_iter), int(bb), _d(stats))
    st = SolveStats(int(stats[0]), int(stats[1]), int(stats[2]), float(stats[3]),
                    int(stats[4]), int(stats[5]), float(stats[6]))
    return gamma, g, st


def _cg(A, b, x0=None, rtol=1e-14, maxiter=200000):
    """Jacobi-preconditioned conjugate gradients on an SPD sparse A."""
    import scipy.sparse.linalg as spla
    d = A.diagonal()
    pre = spla.LinearOperator(A.shape, matvec=lambda v: v / d)
    x, info = spla.cg(A, b, x0=x0, rtol=rtol, atol=0.0, maxiter=maxiter, M=pre)
    if info != 0:
        raise RuntimeError(f"oracle CG did not converge ({info})")
    return x


def _solve_active(M, q, act, x0=None):
    """gamma_A solving M_AA gamma_A = -q_A (gamma_I = 0): a dense solve for
    small blocks, a sparse LU up to 20000 rows, Jacobi-preconditioned CG to a
    relative residual of 1e-14 beyond (started from x0 when given)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    gamma = np.zeros(q.shape[0])
    idx = np.flatnonzero(act)
    if idx.size == 0:
        return gamma
    Maa = M[idx][:, idx]
    if idx.size <= 3000:
        gamma[idx] = np.linalg.solve(Maa.toarray() if sp.issparse(Maa) else Maa,
                                     -q[idx])
    elif idx.size <= 20000:
        gamma[idx] = spla.splu(sp.csc_matrix(Maa)).solve(-q[idx])
    else:
        gamma[idx] = _cg(sp.csr_matrix(Maa), -q[idx],
                         None if x0 is None else np.asarray(x0, dtype=np.float64)[idx])
    return gamma


def polish(s, c, q, gamma, max_pass=50):
    """Exact LCP solution near ``gamma``: take A = {gamma > 0}, solve the
    active block M_AA gamma_A = -q_A, then move violators (gamma_A < 0 leaves
    A, g_I < 0 joins A) and repeat. Returns (gamma, g, passes); passes = -1
    if it did not settle within ``max_pass``."""
    M = M_matrix(s, c)
    q = _f64(q)
    act = np.asarray(gamma) > 0.0
    gam = np.asarray(gamma, dtype=np.float64)
    for p in range(max_pass):
        gam = _solve_active(M, q, act, gam)
        g = M @ gam + q
        leave = act & (gam < 0.0)
        join = (~act) & (g < 0.0)
        if not leave.any() and not join.any():
            return gam, g, p + 1
        act = (act & ~leave) | join
    return gam, g, -1


def adjoint(s, c, q, u_nc, gamma, dL_dgamma=None, dL_dF=None, method="direct"):
    """Implicit adjoint of the converged LCP on its active set
    A = {gamma > 0} (the active set of section 3.2; the derivation is not in
    the paper). With b = dL/dgamma + D^T dL/dF_c, solve M_AA w_A = b_A, w_I = 0.
    Returns (dL_dq, dL_dpos, w) with dL_dq = -w and dL_dpos[n,3] from the
    per-contact geometric derivatives (orientations, radii, Mob and U_nc held
    fixed). Pinned by central finite differences of polished solves and by
    the two-sphere closed form; parity unpinned by the paper."""
    import scipy.sparse as sp
    lib = _load()
    n = s.n
    gamma = _f64(gamma)
    b = np.zeros(c.nc) if dL_dgamma is None else _f64(dL_dgamma).copy()
    if dL_dF is not None:
        b = b + DT_apply(c, dL_dF)
    act = gamma > 0.0
    idx = np.flatnonzero(act)
    w = np.zeros(c.nc)
    if idx.size:
        M = M_matrix(s, c)
        Maa = M[idx][:, idx]
        if method == "direct":
            w = _solve_active(M, -b, act)
        else:
            w[idx] = _cg(sp.csr_matrix(Maa), b[idx])
    axis, mob = _f64(s.axis), _f64(s.mob)
    Uc = mobility(axis, mob, D_apply(n, c, gamma))
    Vw = mobility(axis, mob, D_apply(n, c, w))
    Utot = _f64(u_nc) + Uc
    out = adjoint_positions(s, c, gamma, w, dL_dF, Vw, Utot)
    return -w, out, w


def adjoint_positions(s, c, gamma, w, dL_dF, Vw, Utot):
    """The per-contact geometric part of the adjoint's centre gradient:
    sum_l dD_l^T [gamma_l (dL/dF - V_w) - w_l U] - sum_l w_l dPhi_l/dt over
    the centres, for given V_w = Mob D w and U = U_nc + U_c (any symmetric
    mobility; the mobility itself held fixed)."""
    lib = _load()
    n = s.n
    gamma, w, Vw, Utot = map(_f64, (gamma, w, Vw, Utot))
    dLdF = None if dL_dF is None else _f64(dL_dF)
    ci, cj = _i32(c.i), _i32(c.j)
    out = np.zeros((n, 3))
    pos, axis, rad, hl, box = map(_f64, (s.pos, s.axis, s.radius, s.half_len, s.box))
    lib.orc_adjoint_positions(
        n, c.nc, _d(pos), _d(axis), _d(rad), _d(hl), _d(box), int(s.periodic),
        ci.ctypes.data_as(_ip), cj.ctypes.data_as(_ip), _d(gamma), _d(w),
        None if dLdF is None else _d(dLdF), _d(Vw), _d(Utot), float(s.dt),
        _d(out))
    return out


def contact_grad(ci, pi, Ri, hi, cj, pj, Rj, hj, Ei, Ej, c_phi,
                 box=(0.0, 0.0, 0.0), periodic=0):
    """d/dr of D_l(r)^T [E_i; E_j] + c_phi Phi_l(r), r = c_j - c_i."""
    lib = _load()
    ci, pi, cj, pj, box, Ei, Ej = map(_f64, (ci, pi, cj, pj, box, Ei, Ej))
    out = np.zeros(3)
    lib.orc_contact_grad(_d(ci), _d(pi), float(Ri), float(hi), _d(cj), _d(pj),
                         float(Rj), float(hj), _d(box), int(periodic), _d(Ei),
                         _d(Ej), float(c_phi), _d(out))
    return out


def setup(s, method="cells"):
    """Contacts, U_nc = Mob F_ext and q for suspension ``s``."""
    c = find_contacts(s, method)
    u_nc = mobility(s.axis, s.mob, s.f_ext)
    q = build_q(c, u_nc, s.dt)
    return c, u_nc, q
