"""Time stepping of a collision-constrained suspension (section 3.2's outer
loop): per step the contacts are rebuilt, the LCP is solved (warm-started
from the previous step's collision forces of the same pairs) and the
configuration advances by first-order Euler (Eq. time-step) with the
quaternion kinematics of section 2. Every step runs in the library's HIP
kernels; this module marshals arguments and keeps the state between steps."""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import torch

from . import _abi as A
from .api import (RPY, Box, Contacts, Particles, Workspace, _check, _dev, _ptr, _stream,
                  apply_mobility, build_contacts, require_solution, solve_lcp, solve_lcp_mob,
                  solve_lcp_rpy)


def quat_from_axis(axis: torch.Tensor) -> torch.Tensor:
    """[n][4] unit quaternions (s, p) of the shortest rotations e_z -> axis."""
    axis = _dev(axis)
    n = int(axis.shape[0])
    quat = torch.empty((max(1, n), 4), dtype=torch.float64, device="cuda")
    _check("sc_quat_from_axis", A.lib().sc_quat_from_axis(n, _ptr(axis), _ptr(quat), _stream()))
    return quat[:n]


def advance(particles: Particles, quat: torch.Tensor, u_nc: torch.Tensor,
            u_c: Optional[torch.Tensor], dt: float) -> None:
    """In place: centres += dt U, quaternions by dt Psi Omega (normalised),
    axes = R(quat) e_z, with U = u_nc + u_c."""
    _check("sc_advance", A.lib().sc_advance(particles.n, _ptr(particles.pos), _ptr(quat),
                                            _ptr(particles.axis), _ptr(u_nc), _ptr(u_c),
                                            float(dt), _stream()))


def map_gamma(n: int, prev: Contacts, gamma_prev: torch.Tensor, cur: Contacts) -> torch.Tensor:
    """gamma_0 of ``cur``: the previous gamma of the same pair, 0 for new pairs."""
    gamma0 = torch.empty(max(1, cur.count), dtype=torch.float64, device="cuda")
    pc, cc = prev.c(), cur.c()
    _check("sc_map_gamma", A.lib().sc_map_gamma(int(n), ctypes.byref(pc), _ptr(gamma_prev),
                                                ctypes.byref(cc), _ptr(gamma0), _stream()))
    return gamma0[: cur.count]


@dataclasses.dataclass
class StepInfo:
    contacts: Contacts
    gamma: torch.Tensor
    stats: dict
    u_c: torch.Tensor


class TimeStepper:
    """Euler steps of ``particles`` (whose pos and axis tensors are updated in
    place) under external forces ``f_ext`` [n][6] with time step ``dt`` and
    pair threshold ``delta``. ``warm_start``: gamma_0 of each step from the
    previous step's solution. ``hydro_radius``: the mobility is the RPY
    mobility of spheres of these hydrodynamic radii and viscosity ``mu``
    (every product through ``solve_lcp_mob``) instead of the dry mobility.
    ``mobility``: any mobility object with ``apply(f)`` and ``fn_ctx()``
    (RPY, DryMobility, FnMobility); it must follow the particles' centres,
    which the steps update in place. ``persistent``: with an RPY mobility,
    solve in one persistent launch (solve_lcp_rpy) instead of a launch per
    phase; None chooses by size: persistent up to PERSISTENT_RPY_MAX_N
    particles (measured faster there, slower beyond). ``spin_limit`` is
    passed to the persistent solves (> 0 forces their barrier time-out, for
    tests). A step whose solve ends with an error status (a barrier time-out,
    a non-finite iterate) raises ScError before anything moves."""

    PERSISTENT_RPY_MAX_N = 2048

    def __init__(self, particles: Particles, box: Box, delta: float, dt: float,
                 f_ext: torch.Tensor, tol: float = 1e-6, warm_start: bool = True,
                 max_iter: int = 100000, hydro_radius: Optional[torch.Tensor] = None,
                 mu: float = 1.0, mobility=None, persistent: Optional[bool] = None,
                 spin_limit: int = 0):
        self.P = particles
        self.box = box
        self.delta = float(delta)
        self.dt = float(dt)
        self.f_ext = _dev(f_ext)
        self.tol = float(tol)
        self.warm = bool(warm_start)
        self.max_iter = int(max_iter)
        self.quat = quat_from_axis(particles.axis).clone()
        self.ws = Workspace()
        self.prev: Optional[Contacts] = None
        self.prev_gamma: Optional[torch.Tensor] = None
        # reads particles.pos at every product, which the steps update in place
        if mobility is not None and hydro_radius is not None:
            raise ValueError("give either hydro_radius or mobility")
        self.rpy = mobility if mobility is not None else (
            None if hydro_radius is None else RPY(particles.pos, hydro_radius, mu))
        if persistent is None:
            persistent = particles.n <= self.PERSISTENT_RPY_MAX_N
        self.persistent = bool(persistent) and isinstance(self.rpy, RPY)
        self.spin_limit = int(spin_limit)

    def step(self) -> StepInfo:
        P = self.P
        u_nc = apply_mobility(P, self.f_ext) if self.rpy is None else self.rpy.apply(self.f_ext)
        con = build_contacts(P, self.box, self.delta, u_nc, self.dt, workspace=self.ws,
                             assemble=self.rpy is None)
        gamma0 = None
        if self.warm and self.prev is not None and con.count:
            gamma0 = map_gamma(P.n, self.prev, self.prev_gamma, con)
        if self.rpy is None:
            gamma, g, st, f_c, u_c = solve_lcp(P, con, tol=self.tol, max_iter=self.max_iter,
                                               gamma0=gamma0, want_fc=True, workspace=self.ws,
                                               spin_limit=self.spin_limit)
            solver = "sc_solve_lcp"
        elif self.persistent:
            gamma, g, st, f_c, u_c = solve_lcp_rpy(P, con, self.rpy, tol=self.tol,
                                                   max_iter=self.max_iter, gamma0=gamma0,
                                                   want_fc=True, spin_limit=self.spin_limit)
            solver = "sc_solve_lcp_rpy"
        else:
            gamma, g, st, f_c, u_c = solve_lcp_mob(P, con, self.rpy, tol=self.tol,
                                                   max_iter=self.max_iter, gamma0=gamma0,
                                                   want_fc=True)
            solver = "sc_solve_lcp_mob"
        require_solution(solver, st)
        advance(P, self.quat, u_nc, u_c, self.dt)
        self.prev, self.prev_gamma = con, gamma
        return StepInfo(con, gamma, st, u_c)
