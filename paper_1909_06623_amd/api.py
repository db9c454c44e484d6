"""Python binding of the C ABI with the same names: build_contacts,
solve_lcp, solve_lcp_adjoint (plus apply_mobility and mvop).

Only argument marshalling happens here: PyTorch supplies device memory and the
current HIP stream; every step of the computation runs in the library's HIP
kernels. Inputs are float64 tensors on the GPU.
"""
from __future__ import annotations

import ctypes
import dataclasses
import sys
from typing import Optional

import torch

from . import _abi as A


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(fn, rc, allow=(A.SC_OK,)):
    if rc not in allow:
        raise A.ScError(fn, rc)
    return rc


def require_solution(fn, st):
    """Raise ScError unless a solve's status is SC_OK or SC_NOT_CONVERGED
    (the iteration cap: the outputs hold the last iterate). A timed-out
    barrier or a non-finite iterate leaves nothing fit to move particles
    with or to differentiate."""
    if st["status"] not in (A.SC_OK, A.SC_NOT_CONVERGED):
        raise A.ScError(fn, st["status"])
    return st


def _dev(t, dtype=torch.float64):
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    if not t.is_cuda:
        t = t.cuda()
    return t.to(dtype).contiguous()


@dataclasses.dataclass
class Particles:
    """Rigid particles: centres, unit axes, radii, half segment lengths
    (0 = sphere) and dry mobility coefficients (a_par, a_perp, b_par,
    b_perp), all float64 on the GPU."""
    pos: torch.Tensor
    axis: torch.Tensor
    radius: torch.Tensor
    half_len: torch.Tensor
    mob: torch.Tensor

    @property
    def n(self):
        return int(self.pos.shape[0])

    @classmethod
    def from_arrays(cls, pos, axis, radius, half_len, mob):
        return cls(_dev(pos), _dev(axis), _dev(radius), _dev(half_len), _dev(mob))

    @classmethod
    def from_suspension(cls, s):
        return cls.from_arrays(s.pos, s.axis, s.radius, s.half_len, s.mob)

    def c(self, pos=None):
        pos = self.pos if pos is None else pos
        return A.sc_particles(self.n, 0, pos.data_ptr(), self.axis.data_ptr(),
                              self.radius.data_ptr(), self.half_len.data_ptr(),
                              self.mob.data_ptr())


@dataclasses.dataclass
class Box:
    """Periodic box, or (periodic=False) free space with optional planar
    walls on its faces: bit 2a of ``walls`` closes x_a = lo_a, bit 2a + 1
    closes x_a = lo_a + len_a."""
    len: tuple
    lo: tuple = (0.0, 0.0, 0.0)
    periodic: bool = True
    walls: int = 0

    def c(self):
        b = A.sc_box()
        for k in range(3):
            b.lo[k] = float(self.lo[k])
            b.len[k] = float(self.len[k])
        b.periodic = 1 if self.periodic else 0
        b.walls = int(self.walls)
        return b


class Workspace:
    """Caller-owned scratch for the library (one device byte buffer, grown
    on demand, 256-byte aligned)."""

    def __init__(self):
        self.buf = None
        self.base = 0
        self.size = 0

    def get(self, n, capacity):
        need = int(A.lib().sc_workspace_bytes(int(n), int(capacity), A.SC_WS_ALL))
        if self.buf is None or self.size < need:
            self.buf = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
            addr = self.buf.data_ptr()
            self.base = (addr + 255) // 256 * 256
            self.size = need + 256 - (self.base - addr)
        return ctypes.c_void_p(self.base), ctypes.c_size_t(self.size)


_default_ws = {}


def default_workspace():
    dev = torch.cuda.current_device()
    if dev not in _default_ws:
        _default_ws[dev] = Workspace()
    return _default_ws[dev]


class Contacts:
    """Close pairs (i < j, solver order) with their frames and q, plus the
    library's private plan buffer, in caller-allocated device memory."""

    def __init__(self, n, capacity):
        self.n = int(n)
        self.capacity = int(capacity)
        cap = max(1, self.capacity)
        dev = "cuda"
        self.ci = torch.empty(cap, dtype=torch.int32, device=dev)
        self.cj = torch.empty(cap, dtype=torch.int32, device=dev)
        self.phi = torch.empty(cap, dtype=torch.float64, device=dev)
        self.q = torch.empty(cap, dtype=torch.float64, device=dev)
        self.frame = torch.empty((cap, 9), dtype=torch.float64, device=dev)
        pb = int(A.lib().sc_plan_bytes(self.n, self.capacity))
        self._plan = torch.empty(pb + 256, dtype=torch.uint8, device=dev)
        addr = self._plan.data_ptr()
        self.plan_ptr = (addr + 255) // 256 * 256
        self.plan_bytes = pb + 256 - (self.plan_ptr - addr)
        self.count = 0
        self.n_parallel = self.n_zero_dist = self.n_borderline = 0
        self.grid = (0, 0, 0)
        self.nnz = 0
        self._mat = None
        self.mat_ptr = 0
        self.mat_bytes = 0
        self.mat_ready = 0

    def c(self):
        s = A.sc_contacts()
        s.capacity = self.capacity
        s.count = self.count
        for name in ("ci", "cj", "phi", "q", "frame"):
            setattr(s, name, getattr(self, name).data_ptr())
        s.plan = self.plan_ptr
        s.plan_bytes = self.plan_bytes
        s.n_parallel = self.n_parallel
        s.n_zero_dist = self.n_zero_dist
        s.n_borderline = self.n_borderline
        s.nnz = self.nnz
        s.mat = self.mat_ptr
        s.mat_bytes = self.mat_bytes
        s.mat_ready = self.mat_ready
        return s

    def _take(self, s):
        self.count = int(s.count)
        self.n_parallel = int(s.n_parallel)
        self.n_zero_dist = int(s.n_zero_dist)
        self.n_borderline = int(s.n_borderline)
        self.grid = tuple(int(g) for g in s.grid)
        self.nnz = int(s.nnz)
        self.mat_ready = int(s.mat_ready)

    def assemble(self, particles):
        """Assemble M = D^T Mob D into a device buffer owned by this object."""
        mb = int(A.lib().sc_matrix_bytes(self.count, self.nnz))
        if mb == 0:
            raise RuntimeError(f"M with {self.nnz} nonzeros cannot be assembled")
        if self._mat is None or self.mat_bytes < mb:
            self._mat = torch.empty(mb + 256, dtype=torch.uint8, device="cuda")
            addr = self._mat.data_ptr()
            self.mat_ptr = (addr + 255) // 256 * 256
            self.mat_bytes = mb + 256 - (self.mat_ptr - addr)
        pc, cc = particles.c(), self.c()
        _check("sc_assemble_matrix",
               A.lib().sc_assemble_matrix(ctypes.byref(pc), ctypes.byref(cc), _stream()))
        self._take(cc)
        return self

    # views of the first `count` rows
    @property
    def i(self):
        return self.ci[: self.count]

    @property
    def j(self):
        return self.cj[: self.count]

    @property
    def nrm(self):
        return self.frame[: self.count, 0:3]

    @property
    def tau_i(self):
        return self.frame[: self.count, 3:6]

    @property
    def tau_j(self):
        return self.frame[: self.count, 6:9]

    def canonical_order(self, workspace: Optional["Workspace"] = None):
        """Permutation (int64 indices into the solver order) that lists the
        contacts by (ci, cj), the order of a plain enumeration of pairs
        i < j; computed by the library (sc_canonical_order)."""
        perm = torch.empty(max(1, self.count), dtype=torch.int32, device="cuda")
        ws = workspace or default_workspace()
        wsp, wsn = ws.get(self.n, self.capacity)
        cc = self.c()
        _check("sc_canonical_order",
               A.lib().sc_canonical_order(self.n, ctypes.byref(cc), _ptr(perm), wsp, wsn,
                                          _stream()))
        return perm[: self.count].to(torch.int64)


def release():
    """Wait for the device, then free the host resources the library keeps
    for this thread between calls (sc_release). Call before exiting."""
    _check("sc_release", A.lib().sc_release())


def apply_mobility(particles: Particles, f: torch.Tensor) -> torch.Tensor:
    """u = Mob f per particle (the dry block-diagonal mobility)."""
    f = _dev(f)
    u = torch.empty_like(f)
    pc = particles.c()
    _check("sc_apply_mobility",
           A.lib().sc_apply_mobility(ctypes.byref(pc), _ptr(f), _ptr(u), _stream()))
    return u


def build_contacts(particles: Particles, box: Box, delta: float, u_nc: torch.Tensor,
                   dt: float, capacity: Optional[int] = None,
                   workspace: Optional[Workspace] = None, assemble: bool = True) -> Contacts:
    """Close-pair set, contact frames, solver layout and q (grows the contact
    arrays and retries when the capacity is too small); with ``assemble``
    also forms the sparse M = D^T Mob D used by the one-pass solve."""
    u_nc = _dev(u_nc)
    ws = workspace or default_workspace()
    n = particles.n
    cap = int(capacity) if capacity is not None else max(64, 8 * n)
    pc, bc = particles.c(), box.c()
    while True:
        con = Contacts(n, cap)
        cc = con.c()
        wsp, wsn = ws.get(n, cap)
        rc = A.lib().sc_build_contacts(ctypes.byref(pc), ctypes.byref(bc), float(delta),
                                       _ptr(u_nc), float(dt), ctypes.byref(cc), wsp, wsn,
                                       _stream())
        con._take(cc)
        if rc == A.SC_ERR_CAPACITY:
            cap = int(cc.count)
            continue
        _check("sc_build_contacts", rc)
        if assemble:
            con.assemble(particles)
        return con


def mvop(particles: Particles, contacts: Contacts, x: torch.Tensor,
         workspace: Optional[Workspace] = None) -> torch.Tensor:
    """y = D^T Mob D x (one matrix-free product)."""
    x = _dev(x)
    y = torch.empty(max(1, contacts.count), dtype=torch.float64, device="cuda")
    ws = workspace or default_workspace()
    wsp, wsn = ws.get(particles.n, contacts.capacity)
    pc, cc = particles.c(), contacts.c()
    _check("sc_mvop", A.lib().sc_mvop(ctypes.byref(pc), ctypes.byref(cc), _ptr(x), _ptr(y),
                                      wsp, wsn, _stream()))
    return y[: contacts.count]


def solve_lcp(particles: Particles, contacts: Contacts, tol: float = 1e-6,
              max_iter: int = 100000, bb: int = 1, gamma0: Optional[torch.Tensor] = None,
              want_fc: bool = False, lanes_per_particle: int = 0, grid: int = 0,
              block: int = 0, op: int = 0, workspace: Optional[Workspace] = None,
              raise_on_nonconverged=False, slices_per_wave: int = 0,
              lds_entries_per_wave: int = 0, spin_limit: int = 0):
    """BBPGD (Algorithm 1). Returns (gamma, g, stats dict, f_c, u_c); f_c and
    u_c are None unless want_fc. ``spin_limit`` > 0 caps every barrier wait
    at that many polls (forces the SC_ERR_TIMEOUT path, for tests)."""
    nc = contacts.count
    gamma = torch.zeros(max(1, nc), dtype=torch.float64, device="cuda")
    if gamma0 is not None and nc:
        gamma[:nc] = _dev(gamma0)
    g = torch.empty(max(1, nc), dtype=torch.float64, device="cuda")
    f_c = u_c = None
    if want_fc:
        f_c = torch.empty((particles.n, 6), dtype=torch.float64, device="cuda")
        u_c = torch.empty((particles.n, 6), dtype=torch.float64, device="cuda")
    opts = A.sc_solve_opts(float(tol), int(max_iter), int(bb), 1 if gamma0 is not None else 0,
                           int(lanes_per_particle), int(grid), int(block), int(op),
                           int(slices_per_wave), int(lds_entries_per_wave), int(spin_limit))
    st = A.sc_stats()
    ws = workspace or default_workspace()
    wsp, wsn = ws.get(particles.n, contacts.capacity)
    pc, cc = particles.c(), contacts.c()
    rc = A.lib().sc_solve_lcp(ctypes.byref(pc), ctypes.byref(cc), ctypes.byref(opts),
                              _ptr(gamma), _ptr(g), _ptr(f_c), _ptr(u_c), ctypes.byref(st),
                              wsp, wsn, _stream())
    allow = (A.SC_OK,) if raise_on_nonconverged else (A.SC_OK, A.SC_NOT_CONVERGED,
                                                      A.SC_ERR_NONFINITE, A.SC_ERR_TIMEOUT)
    _check("sc_solve_lcp", rc, allow)
    return gamma[:nc], g[:nc], st.as_dict(), f_c, u_c


def solve_lcp_noalloc(particles: Particles, contacts: Contacts, gamma: torch.Tensor,
                      g: torch.Tensor, tol: float = 1e-6, max_iter: int = 100000, bb: int = 1,
                      warm_start: bool = False, f_c: Optional[torch.Tensor] = None,
                      u_c: Optional[torch.Tensor] = None, op: int = 0):
    """BBPGD as solve_lcp, through sc_solve_lcp_noalloc: the library's own
    device scratch array stands in for the workspace and nothing is
    allocated by the call. gamma and g (and f_c, u_c if given) are the
    caller's output buffers (gamma holds gamma_0 when ``warm_start``).
    Returns (return code, stats dict); the caller checks the code."""
    opts = A.sc_solve_opts(float(tol), int(max_iter), int(bb), 1 if warm_start else 0,
                           0, 0, 0, int(op), 0, 0, 0)
    st = A.sc_stats()
    pc, cc = particles.c(), contacts.c()
    rc = A.lib().sc_solve_lcp_noalloc(ctypes.byref(pc), ctypes.byref(cc), ctypes.byref(opts),
                                      _ptr(gamma), _ptr(g), _ptr(f_c), _ptr(u_c),
                                      ctypes.byref(st), _stream())
    return rc, st.as_dict()


STATS_BYTES = ctypes.sizeof(A.sc_stats)


def stats_from_device(buf: torch.Tensor) -> dict:
    """An sc_stats written to device memory (a uint8 tensor of STATS_BYTES),
    read back as a dict (synchronises with the copy)."""
    st = A.sc_stats.from_buffer_copy(bytes(buf.cpu().numpy().tobytes()))
    return st.as_dict()


def solve_lcp_async(particles: Particles, contacts: Contacts, gamma: torch.Tensor,
                    g: torch.Tensor, stats: torch.Tensor, tol: float = 1e-6,
                    max_iter: int = 100000, bb: int = 1, warm_start: bool = False,
                    f_c: Optional[torch.Tensor] = None, u_c: Optional[torch.Tensor] = None,
                    op: int = 0, spin_limit: int = 0, workspace: Optional[Workspace] = None):
    """BBPGD through sc_solve_lcp_async: enqueues the solve on the current
    stream and returns at once (capturable with torch.cuda.graph). gamma, g
    (and f_c, u_c) are the caller's buffers; ``stats`` is a device uint8
    tensor of STATS_BYTES that receives the sc_stats (``stats_from_device``).
    Raises only on argument or launch errors."""
    opts = A.sc_solve_opts(float(tol), int(max_iter), int(bb), 1 if warm_start else 0,
                           0, 0, 0, int(op), 0, 0, int(spin_limit))
    ws = workspace or default_workspace()
    wsp, wsn = ws.get(particles.n, contacts.capacity)
    pc, cc = particles.c(), contacts.c()
    _check("sc_solve_lcp_async",
           A.lib().sc_solve_lcp_async(ctypes.byref(pc), ctypes.byref(cc), ctypes.byref(opts),
                                      _ptr(gamma), _ptr(g), _ptr(f_c), _ptr(u_c), _ptr(stats),
                                      wsp, wsn, _stream()))


def solve_lcp_adjoint(particles: Particles, box: Box, contacts: Contacts,
                      u_nc: torch.Tensor, dt: float, gamma: torch.Tensor,
                      dL_dgamma: Optional[torch.Tensor] = None,
                      dL_df: Optional[torch.Tensor] = None, tol: float = 1e-10,
                      max_iter: int = 100000, lanes_per_particle: int = 0, grid: int = 0,
                      block: int = 0, op: int = 0, workspace: Optional[Workspace] = None,
                      slices_per_wave: int = 0, lds_entries_per_wave: int = 0):
    """Implicit adjoint of a converged solve: returns (dL_dq, dL_dpos, stats)."""
    nc = contacts.count
    u_nc = _dev(u_nc)
    gamma = _dev(gamma)
    dLg = None if dL_dgamma is None else _dev(dL_dgamma)
    dLf = None if dL_df is None else _dev(dL_df)
    dq = torch.empty(max(1, nc), dtype=torch.float64, device="cuda")
    dpos = torch.empty((particles.n, 3), dtype=torch.float64, device="cuda")
    opts = A.sc_adjoint_opts(float(tol), int(max_iter), int(lanes_per_particle), int(grid),
                             int(block), int(op), int(slices_per_wave),
                             int(lds_entries_per_wave))
    st = A.sc_stats()
    ws = workspace or default_workspace()
    wsp, wsn = ws.get(particles.n, contacts.capacity)
    pc, bc, cc = particles.c(), box.c(), contacts.c()
    rc = A.lib().sc_solve_lcp_adjoint(ctypes.byref(pc), ctypes.byref(bc), ctypes.byref(cc),
                                      _ptr(u_nc), float(dt), _ptr(gamma), _ptr(dLg),
                                      _ptr(dLf), _ptr(dq), _ptr(dpos), ctypes.byref(opts),
                                      ctypes.byref(st), wsp, wsn, _stream())
    _check("sc_solve_lcp_adjoint", rc, (A.SC_OK, A.SC_NOT_CONVERGED))
    return dq[:nc], dpos, st.as_dict()


def polish_lcp(particles: Particles, contacts: Contacts, gamma: torch.Tensor,
               tol: float = 1e-12, max_iter: int = 100000, max_pass: int = 0,
               want_fc: bool = False, op: int = 0, workspace: Optional[Workspace] = None):
    """Active-set polish of a solve (sc_polish_lcp): the exact LCP solution
    on the active set of ``gamma`` (solved by conjugate gradients to ``tol``),
    violators moved between passes. Returns (gamma, g, stats, f_c, u_c): the
    polished point and M gamma + q if stats["status"] is SC_OK, else the input
    and its g; f_c and u_c are None unless want_fc."""
    nc, n = contacts.count, particles.n
    gam = torch.empty(max(1, nc), dtype=torch.float64, device="cuda")
    if nc:
        gam[:nc] = _dev(gamma)[:nc]
    g = torch.empty(max(1, nc), dtype=torch.float64, device="cuda")
    f_c = torch.empty((n, 6), dtype=torch.float64, device="cuda") if want_fc else None
    u_c = torch.empty((n, 6), dtype=torch.float64, device="cuda") if want_fc else None
    opts = A.sc_adjoint_opts(float(tol), int(max_iter), 0, 0, 0, int(op), 0, 0)
    st = A.sc_stats()
    ws = workspace or default_workspace()
    wsp, wsn = ws.get(n, contacts.capacity)
    pc, cc = particles.c(), contacts.c()
    rc = A.lib().sc_polish_lcp(ctypes.byref(pc), ctypes.byref(cc), _ptr(gam), _ptr(g),
                               _ptr(f_c), _ptr(u_c), ctypes.byref(opts), int(max_pass),
                               ctypes.byref(st), wsp, wsn, _stream())
    _check("sc_polish_lcp", rc, (A.SC_OK, A.SC_NOT_CONVERGED))
    return gam[:nc], g[:nc], st.as_dict(), f_c, u_c


class RPY:
    """Rotne-Prager-Yamakawa mobility of spheres in unbounded fluid
    (``sc_rpy``): translational pair couplings for unequal radii with the
    overlap forms, single-sphere rotational mobility, evaluated directly on
    the GPU. ``pos`` is read at every product, so it may be updated in
    place between solves; ``radius`` are hydrodynamic radii."""

    def __init__(self, pos: torch.Tensor, radius: torch.Tensor, mu: float = 1.0):
        self.pos = _dev(pos)
        self.radius = _dev(radius)
        self.mu = float(mu)
        n = int(self.pos.shape[0])
        wb = int(A.lib().sc_rpy_work_bytes(n))
        self._work = torch.empty(wb + 256, dtype=torch.uint8, device="cuda")
        addr = self._work.data_ptr()
        self._wp = (addr + 255) // 256 * 256
        self._ctx = A.sc_rpy(n, 0, self.pos.data_ptr(), self.radius.data_ptr(), self.mu,
                             self._wp, wb + 256 - (self._wp - addr))

    @property
    def n(self):
        return int(self._ctx.n)

    def fn_ctx(self):
        """(function address, context address) for sc_solve_lcp_mob."""
        return (ctypes.cast(A.lib().sc_rpy_apply, ctypes.c_void_p).value,
                ctypes.addressof(self._ctx))

    def apply(self, f: torch.Tensor) -> torch.Tensor:
        """u = Mob f for f [n][6]."""
        f = _dev(f)
        u = torch.empty_like(f)
        _check("sc_rpy_apply", A.lib().sc_rpy_apply(ctypes.addressof(self._ctx), self.n,
                                                    _ptr(f), _ptr(u), _stream()))
        return u

    def grad_fn_ctx(self):
        """(gradient function address, context address) for the adjoint."""
        return (ctypes.cast(A.lib().sc_rpy_grad, ctypes.c_void_p).value,
                ctypes.addressof(self._ctx))

    def grad(self, a: torch.Tensor, f: torch.Tensor) -> torch.Tensor:
        """g[k] = d/dc_k (a^T Mob f) for a, f [n][6]."""
        a, f = _dev(a), _dev(f)
        g = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
        _check("sc_rpy_grad", A.lib().sc_rpy_grad(ctypes.addressof(self._ctx), self.n, _ptr(a),
                                                  _ptr(f), _ptr(g), _stream()))
        return g


class DryMobility:
    """The dry block-diagonal mobility of ``particles`` as a mobility
    function (``sc_dry_apply``)."""

    def __init__(self, particles: Particles):
        self.P = particles
        self._ctx = particles.c()

    def fn_ctx(self):
        return (ctypes.cast(A.lib().sc_dry_apply, ctypes.c_void_p).value,
                ctypes.addressof(self._ctx))

    def grad_fn_ctx(self):
        """The dry mobility does not depend on the centres."""
        return None

    def apply(self, f: torch.Tensor) -> torch.Tensor:
        return apply_mobility(self.P, f)


class _DevView:
    """A [shape] float64 view of device memory the library hands to a
    mobility function (no copy; valid during the call)."""

    def __init__(self, ptr, shape):
        self.__cuda_array_interface__ = {"shape": shape, "typestr": "<f8", "data": (ptr, False),
                                         "version": 2, "strides": None}


def _view(ptr, shape):
    return torch.as_tensor(_DevView(ptr, shape), device="cuda")


class FnMobility:
    """A mobility written in Python, for solve_lcp_mob and
    solve_lcp_adjoint_mob: ``apply(f, u)`` writes u = Mob f into the [n, 6]
    tensor u (f and u are views of the solver's buffers; the work goes on
    the current stream), and the optional ``grad(a, f, g)`` writes
    g = d/dc (a^T Mob f) into the [n, 3] tensor g. Mob must be symmetric
    positive definite. The solver calls them through ctypes from the calling
    thread; an exception raised inside is re-raised by the solve."""

    def __init__(self, apply, grad=None):
        self._apply, self._grad = apply, grad
        self._error = None

        def cb(ctx, n, f, u, stream):
            try:
                self._apply(_view(f, (n, 6)), _view(u, (n, 6)))
                return A.SC_OK
            except BaseException as e:  # handed back to the caller of the solve
                self._error = e
                return A.SC_ERR_INVALID

        def gcb(ctx, n, a, f, g, stream):
            try:
                self._grad(_view(a, (n, 6)), _view(f, (n, 6)), _view(g, (n, 3)))
                return A.SC_OK
            except BaseException as e:
                self._error = e
                return A.SC_ERR_INVALID

        self._cb = A.MOBILITY_FN(cb)
        self._gcb = A.MOBILITY_GRAD_FN(gcb) if grad is not None else None

    def apply(self, f: torch.Tensor) -> torch.Tensor:
        """u = Mob f for f [n][6] (the Python function called directly)."""
        f = _dev(f)
        u = torch.empty_like(f)
        self._apply(f, u)
        return u

    def fn_ctx(self):
        return (ctypes.cast(self._cb, ctypes.c_void_p).value, None)

    def grad_fn_ctx(self):
        if self._gcb is None:
            return None
        return (ctypes.cast(self._gcb, ctypes.c_void_p).value, None)

    def take_error(self):
        e, self._error = self._error, None
        return e


def _raise_mobility_error(mobility):
    take = getattr(mobility, "take_error", None)
    e = take() if take is not None else None
    if e is not None:
        raise e


def solve_lcp_mob(particles: Particles, contacts: Contacts, mobility, tol: float = 1e-6,
                  max_iter: int = 100000, bb: int = 1, gamma0: Optional[torch.Tensor] = None,
                  want_fc: bool = False, check_every: int = 0,
                  raise_on_nonconverged: bool = False):
    """Algorithm 1 with every product D^T Mob D x taking Mob from
    ``mobility`` (an RPY or DryMobility object, or anything with
    ``fn_ctx()`` returning an sc_mobility_fn address and its context).
    Returns (gamma, g, stats dict, f_c, u_c) like solve_lcp."""
    nc = contacts.count
    n = particles.n
    gamma = torch.zeros(max(1, nc), dtype=torch.float64, device="cuda")
    if gamma0 is not None and nc:
        gamma[:nc] = _dev(gamma0)
    g = torch.empty(max(1, nc), dtype=torch.float64, device="cuda")
    f_c = u_c = None
    if want_fc:
        f_c = torch.empty((n, 6), dtype=torch.float64, device="cuda")
        u_c = torch.empty((n, 6), dtype=torch.float64, device="cuda")
    opts = A.sc_solve_opts(float(tol), int(max_iter), int(bb), 1 if gamma0 is not None else 0,
                           0, 0, 0, 0, 0, 0, 0)
    st = A.sc_stats()
    wb = int(A.lib().sc_solve_mob_work_bytes(n, contacts.capacity))
    work = torch.empty(wb + 256, dtype=torch.uint8, device="cuda")
    wp = (work.data_ptr() + 255) // 256 * 256
    fn, ctx = mobility.fn_ctx()
    pc, cc = particles.c(), contacts.c()
    ctx = None if ctx is None else ctypes.c_void_p(ctx)
    rc = A.lib().sc_solve_lcp_mob(ctypes.byref(pc), ctypes.byref(cc), ctypes.byref(opts),
                                  ctypes.c_void_p(fn), ctx, int(check_every),
                                  _ptr(gamma), _ptr(g), _ptr(f_c), _ptr(u_c), ctypes.byref(st),
                                  ctypes.c_void_p(wp), wb + 256 - (wp - work.data_ptr()),
                                  _stream())
    _raise_mobility_error(mobility)
    allow = (A.SC_OK,) if raise_on_nonconverged else (A.SC_OK, A.SC_NOT_CONVERGED,
                                                      A.SC_ERR_NONFINITE)
    _check("sc_solve_lcp_mob", rc, allow)
    return gamma[:nc], g[:nc], st.as_dict(), f_c, u_c


def solve_lcp_rpy(particles: Particles, contacts: Contacts, rpy: RPY, tol: float = 1e-6,
                  max_iter: int = 100000, bb: int = 1, gamma0: Optional[torch.Tensor] = None,
                  want_fc: bool = False, grid: int = 0, spin_limit: int = 0,
                  raise_on_nonconverged: bool = False):
    """Algorithm 1 with the RPY mobility ``rpy`` in one persistent launch
    (sc_solve_lcp_rpy): the same arithmetic definition as solve_lcp_mob(...,
    rpy), without a launch per phase; for small systems. Returns (gamma, g,
    stats dict, f_c, u_c)."""
    nc, n = contacts.count, particles.n
    gamma = torch.zeros(max(1, nc), dtype=torch.float64, device="cuda")
    if gamma0 is not None and nc:
        gamma[:nc] = _dev(gamma0)
    g = torch.empty(max(1, nc), dtype=torch.float64, device="cuda")
    f_c = u_c = None
    if want_fc:
        f_c = torch.empty((n, 6), dtype=torch.float64, device="cuda")
        u_c = torch.empty((n, 6), dtype=torch.float64, device="cuda")
    opts = A.sc_solve_opts(float(tol), int(max_iter), int(bb), 1 if gamma0 is not None else 0,
                           0, int(grid), 0, 0, 0, 0, int(spin_limit))
    st = A.sc_stats()
    wb = int(A.lib().sc_solve_rpy_work_bytes(n, contacts.capacity))
    work = torch.empty(wb + 256, dtype=torch.uint8, device="cuda")
    wp = (work.data_ptr() + 255) // 256 * 256
    pc, cc = particles.c(), contacts.c()
    rc = A.lib().sc_solve_lcp_rpy(ctypes.byref(pc), ctypes.byref(cc),
                                  ctypes.c_void_p(ctypes.addressof(rpy._ctx)), ctypes.byref(opts),
                                  _ptr(gamma), _ptr(g), _ptr(f_c), _ptr(u_c), ctypes.byref(st),
                                  ctypes.c_void_p(wp), wb + 256 - (wp - work.data_ptr()),
                                  _stream())
    allow = (A.SC_OK,) if raise_on_nonconverged else (A.SC_OK, A.SC_NOT_CONVERGED,
                                                      A.SC_ERR_NONFINITE, A.SC_ERR_TIMEOUT)
    _check("sc_solve_lcp_rpy", rc, allow)
    return gamma[:nc], g[:nc], st.as_dict(), f_c, u_c


def solve_lcp_adjoint_mob(particles: Particles, box: Box, contacts: Contacts,
                          u_nc: torch.Tensor, dt: float, gamma: torch.Tensor, mobility,
                          f_ext: Optional[torch.Tensor] = None,
                          dL_dgamma: Optional[torch.Tensor] = None,
                          dL_df: Optional[torch.Tensor] = None, tol: float = 1e-10,
                          max_iter: int = 100000, check_every: int = 0):
    """Implicit adjoint of a solve behind ``mobility`` (see solve_lcp_mob):
    returns (dL_dq, dL_dpos, stats). A mobility that depends on the centres
    (``grad_fn_ctx()`` not None, e.g. RPY) needs ``f_ext``."""
    nc, n = contacts.count, particles.n
    u_nc = _dev(u_nc)
    gamma = _dev(gamma)
    fe = None if f_ext is None else _dev(f_ext)
    dLg = None if dL_dgamma is None else _dev(dL_dgamma)
    dLf = None if dL_df is None else _dev(dL_df)
    dq = torch.empty(max(1, nc), dtype=torch.float64, device="cuda")
    dpos = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    opts = A.sc_adjoint_opts(float(tol), int(max_iter), 0, 0, 0, 0, 0, 0)
    st = A.sc_stats()
    wb = int(A.lib().sc_adjoint_mob_work_bytes(n, contacts.capacity))
    work = torch.empty(wb + 256, dtype=torch.uint8, device="cuda")
    wp = (work.data_ptr() + 255) // 256 * 256
    fn, ctx = mobility.fn_ctx()
    ctx = None if ctx is None else ctypes.c_void_p(ctx)
    gfc = mobility.grad_fn_ctx()
    gfn, gctx = (None, None) if gfc is None else gfc
    pc, bc, cc = particles.c(), box.c(), contacts.c()
    rc = A.lib().sc_solve_lcp_adjoint_mob(
        ctypes.byref(pc), ctypes.byref(bc), ctypes.byref(cc), _ptr(u_nc), _ptr(fe), float(dt),
        _ptr(gamma), _ptr(dLg), _ptr(dLf), ctypes.c_void_p(fn), ctx,
        None if gfn is None else ctypes.c_void_p(gfn),
        None if gctx is None else ctypes.c_void_p(gctx), ctypes.byref(opts), int(check_every),
        _ptr(dq), _ptr(dpos), ctypes.byref(st), ctypes.c_void_p(wp),
        wb + 256 - (wp - work.data_ptr()), _stream())
    _raise_mobility_error(mobility)
    _check("sc_solve_lcp_adjoint_mob", rc, (A.SC_OK, A.SC_NOT_CONVERGED))
    return dq[:nc], dpos, st.as_dict()


class Batch:
    """Many independent LCPs solved in one persistent launch (one team of
    workgroups per instance at a time, instances taken largest first).

    ``items``: list of (Particles, Contacts) with assembled M, or, with
    ``adjoint``, (Particles, Contacts, Box, u_nc, dt). ``team`` > 0 runs
    every instance on that many workgroups; with ``team`` = 0 each instance
    gets the smallest power of two t with t * ``nnz_per_workgroup`` >= its
    nonzeros of M (at most 32), and with both 0 the target is autotuned.
    ``adjoint_team`` / ``adjoint_nnz_per_workgroup`` do the same for the
    adjoint launch (both 0: the forward's policy, tuned on its own when the
    forward's is). ``block`` / ``adjoint_block``: threads per workgroup of
    each launch (0: 1024 and 512). After ``solve()`` /
    ``graph_solve()``, ``gamma[k]`` and ``g[k]`` hold each solution and, with
    ``adjoint`` (1: loss 1/2 ||D gamma||^2 + dL_dgamma . gamma, 2: the linear
    term only), ``dL_dq[k]`` and ``dL_dpos[k]`` its gradients.

    With ``build=True`` the items are (Particles, Box, delta, u_nc, dt) and
    every solve first builds all contacts and M on the device from the
    particles' current positions (so ``graph_solve`` replays build, solves
    and adjoints as one graph). ``capacity`` / ``nnz_capacity`` (lists) bound
    each instance's contacts and nonzeros; by default they are measured by
    one build per instance with headroom. Then ``contacts[k]`` holds the
    contact arrays, ``gamma[k]``, ``g[k]`` and ``dL_dq[k]`` have capacity
    rows, and ``counts()`` gives the rows in use."""

    def __init__(self, items, tol=1e-6, max_iter=100000, bb=1, team=0, block=0,
                 gamma0=None, adjoint=0, dL_dgamma=None, adjoint_tol=1e-10,
                 adjoint_max_iter=100000, build=False, capacity=None, nnz_capacity=None,
                 adjoint_team=0, nnz_per_workgroup=0, adjoint_nnz_per_workgroup=0,
                 adjoint_block=0):
        self._keep = []
        self.gamma, self.g, self.dL_dq, self.dL_dpos = [], [], [], []
        self.build = bool(build)
        self.contacts = []
        arr = (A.sc_batch_item * max(1, len(items)))()
        for k, it in enumerate(items):
            if self.build:
                P, box, delta, u_nc, dt = it[0], it[1], float(it[2]), _dev(it[3]), float(it[4])
                cap, nnzc = self._capacities(k, P, box, delta, u_nc, dt, capacity, nnz_capacity)
                con = Contacts(P.n, cap)
                con.nnz = nnzc
                mb = int(A.lib().sc_matrix_bytes(cap, nnzc))
                if mb == 0:
                    raise RuntimeError(f"M with {nnzc} nonzeros cannot be assembled")
                con._mat = torch.empty(mb + 256, dtype=torch.uint8, device="cuda")
                con.mat_ptr = (con._mat.data_ptr() + 255) // 256 * 256
                con.mat_bytes = mb + 256 - (con.mat_ptr - con._mat.data_ptr())
                self.contacts.append(con)
                rows = cap
                arr[k].box = box.c()
                arr[k].u_nc = u_nc.data_ptr()
                arr[k].dt = dt
                arr[k].delta = delta
                self._keep += [u_nc]
            else:
                P, con = it[0], it[1]
                if not con.mat_ready:
                    con.assemble(P)
                rows = con.count
            gm = torch.zeros(max(1, rows), dtype=torch.float64, device="cuda")
            if gamma0 is not None and rows:
                g0 = _dev(gamma0[k])
                gm[: g0.numel()] = g0
            g = torch.empty(max(1, rows), dtype=torch.float64, device="cuda")
            self.gamma.append(gm[:rows])
            self.g.append(g[:rows])
            arr[k].p = P.c()
            arr[k].c = con.c()
            arr[k].gamma = gm.data_ptr()
            arr[k].g = g.data_ptr()
            self._keep += [P, con, gm, g]
            if adjoint:
                if not self.build:
                    box, u_nc, dt = it[2], _dev(it[3]), float(it[4])
                    arr[k].box = box.c()
                    arr[k].u_nc = u_nc.data_ptr()
                    arr[k].dt = dt
                    self._keep.append(u_nc)
                dq = torch.empty(max(1, rows), dtype=torch.float64, device="cuda")
                dpos = torch.empty((max(1, P.n), 3), dtype=torch.float64, device="cuda")
                arr[k].dL_dq = dq.data_ptr()
                arr[k].dL_dpos = dpos.data_ptr()
                if dL_dgamma is not None and dL_dgamma[k] is not None:
                    dg = _dev(dL_dgamma[k])
                    arr[k].dL_dgamma = dg.data_ptr()
                    self._keep.append(dg)
                self.dL_dq.append(dq[:rows])
                self.dL_dpos.append(dpos[: P.n])
                self._keep += [dq, dpos]
        self.count = len(items)
        self.adjoint = int(adjoint)
        opts = A.sc_batch_opts(float(tol), int(max_iter), int(bb),
                               1 if gamma0 is not None else 0, int(team), int(block),
                               self.adjoint, float(adjoint_tol), int(adjoint_max_iter),
                               1 if self.build else 0, int(adjoint_team),
                               int(nnz_per_workgroup), int(adjoint_nnz_per_workgroup),
                               int(adjoint_block))
        need = int(A.lib().sc_batch_workspace_bytes(self.count, arr, ctypes.byref(opts)))
        if need == 0:
            raise RuntimeError("sc_batch_workspace_bytes: invalid arguments")
        self._ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
        base = (self._ws.data_ptr() + 255) // 256 * 256
        size = need + 256 - (base - self._ws.data_ptr())
        h = ctypes.c_void_p()
        _check("sc_batch_create",
               A.lib().sc_batch_create(self.count, arr, ctypes.byref(opts), ctypes.c_void_p(base),
                                       ctypes.c_size_t(size), _stream(), ctypes.byref(h)))
        self._items = arr
        self._h = h

    @staticmethod
    def _capacities(k, P, box, delta, u_nc, dt, capacity, nnz_capacity):
        if capacity is not None and nnz_capacity is not None:
            return int(capacity[k]), int(nnz_capacity[k])
        c0 = build_contacts(P, box, delta, u_nc, dt)
        cap = int(capacity[k]) if capacity is not None else int(1.25 * c0.count) + 64
        nnzc = (int(nnz_capacity[k]) if nnz_capacity is not None
                else int(1.5 * c0.nnz) + 16 * (cap - c0.count) + 1024)
        return cap, nnzc

    @staticmethod
    def tuned_policy(info):
        """The keyword arguments that recreate the team policies an autotuned
        batch picked (from ``stats()``'s info): size classes (team 0 and a
        nonzeros-per-workgroup target) or one team size, for each launch."""
        f, a = info["nnz_per_workgroup"], info["adjoint_nnz_per_workgroup"]
        return {"team": 0 if f > 0 else info["team"], "nnz_per_workgroup": f,
                "adjoint_team": 0 if a > 0 else info["team_adjoint"],
                "adjoint_nnz_per_workgroup": a}

    def counts(self):
        """Build mode: (contacts, nonzeros of M, build status) per instance for
        the last solve; also sets ``contacts[k].count``."""
        if not self.build:
            raise RuntimeError("counts() needs a batch created with build=True")
        n = max(1, self.count)
        cnt = (ctypes.c_int32 * n)()
        nnz = (ctypes.c_int64 * n)()
        st = (ctypes.c_int32 * n)()
        _check("sc_batch_contacts", A.lib().sc_batch_contacts(self._h, cnt, nnz, st, _stream()))
        out = [(int(cnt[k]), int(nnz[k]), int(st[k])) for k in range(self.count)]
        for con, (c, z, s) in zip(self.contacts, out):
            con.count = c if s == A.SC_OK else 0
            con.nnz = z
        return out

    def solve(self):
        _check("sc_batch_solve", A.lib().sc_batch_solve(self._h, _stream()))

    def graph_solve(self):
        _check("sc_batch_graph_launch", A.lib().sc_batch_graph_launch(self._h, _stream()))

    def stats(self):
        """(per-instance solve stats, per-instance adjoint stats or None, launch info)."""
        st = (A.sc_stats * max(1, self.count))()
        adj = (A.sc_stats * max(1, self.count))()
        info = A.sc_batch_info()
        _check("sc_batch_stats", A.lib().sc_batch_stats(self._h, st, adj, ctypes.byref(info),
                                                        _stream()))
        inf = {"team": info.team, "block": info.block, "grid": info.grid,
               "lds_entries_per_wave": info.lds_entries_per_wave,
               "tune_ms": list(info.tune_ms), "team_adjoint": info.team_adjoint,
               "tune_adjoint_ms": list(info.tune_adjoint_ms),
               "nnz_per_workgroup": info.nnz_per_workgroup,
               "adjoint_nnz_per_workgroup": info.adjoint_nnz_per_workgroup,
               "adjoint_block": info.adjoint_block}
        sts = [st[k].as_dict() for k in range(self.count)]
        adjs = [adj[k].as_dict() for k in range(self.count)] if self.adjoint else None
        return sts, adjs, inf

    def close(self):
        if self._h:
            A.lib().sc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        # at interpreter shutdown the HIP runtime may already be gone: leave
        # the plan to the process's end instead of calling into it
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
