"""torch.autograd bindings of the collision solve.

Two functions, both thin wrappers of the C ABI (every step runs in the HIP
library):

* ``collision_solve(pos, ...)``: close pairs, D, q and the BBPGD solve of
  the collision LCP (section 3.2, Algorithm 1) as a function of the particle
  centres. Returns (gamma, F_c = D gamma). Its backward is the implicit
  adjoint through the converged solution on its active set (not in the
  paper; the derivation is in ``sc_solve_lcp_adjoint``'s header comment):
  it returns dL/d(centres) and stores dL/dq in the ``SolveInfo``.
* ``lcp_solve(q, ...)``: the solve on a fixed contact set as a function of q,
  returning gamma; its backward returns dL/dq = -w with M_AA w_A = dL/dgamma_A.
* ``hydro_collision_solve(pos, ...)``: as ``collision_solve`` with the RPY
  mobility of spheres: U_nc = Mob(c) F_ext and every product of the solve go
  through it, and the backward includes the mobility's dependence on the
  centres (``sc_solve_lcp_adjoint_mob``).

Orientations, radii and mobility coefficients receive no gradient, and U_nc
none in ``collision_solve`` (the dry mobility does not depend on the
centres). The contact set is piecewise constant in the centres; the
gradient is that of the active branch.

A forward solve that ends with an error status (a barrier time-out, a
non-finite iterate) raises ScError before anything is saved for backward,
and so does a backward whose conjugate-gradient solve misses its tolerance.
"""
from __future__ import annotations

import copy
import dataclasses
from typing import Optional

import torch
from torch.autograd.function import once_differentiable

from . import _abi as A
from .api import (RPY, Box, Contacts, Particles, build_contacts, polish_lcp, require_solution,
                  solve_lcp, solve_lcp_adjoint, solve_lcp_adjoint_mob, solve_lcp_mob,
                  solve_lcp_rpy)


# Largest system whose RPY solve runs as one persistent launch.
PERSISTENT_RPY_MAX_N = 2048


@dataclasses.dataclass
class SolveInfo:
    """Side results of a differentiable solve."""
    contacts: Optional[Contacts] = None
    stats: Optional[dict] = None
    dL_dq: Optional[torch.Tensor] = None          # filled by backward
    adjoint_stats: Optional[dict] = None          # filled by backward
    polish_stats: Optional[dict] = None           # with polish=True


class _CollisionSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, particles, box, u_nc, dt, delta, tol, adjoint_tol, info, kw, polish):
        P = dataclasses.replace(particles, pos=pos.detach().to(torch.float64).contiguous())
        con = build_contacts(P, box, delta, u_nc, dt)
        gamma, g, st, f_c, u_c = solve_lcp(P, con, tol=tol, want_fc=True, **kw)
        info.contacts, info.stats = con, st
        require_solution("sc_solve_lcp", st)
        if polish:
            # the exact LCP solution on the solve's active set (the input
            # itself if no pass settles: info.polish_stats["status"] says which)
            gamma, g, info.polish_stats, f_c, u_c = polish_lcp(P, con, gamma, tol=adjoint_tol,
                                                               want_fc=True)
        ctx.state = (P, box, con, u_nc, dt, adjoint_tol, info, kw)
        ctx.save_for_backward(gamma)
        return gamma, f_c

    @staticmethod
    @once_differentiable
    def backward(ctx, dL_dgamma, dL_df):
        (gamma,) = ctx.saved_tensors
        P, box, con, u_nc, dt, adjoint_tol, info, kw = ctx.state
        dq, dpos, sta = solve_lcp_adjoint(P, box, con, u_nc, dt, gamma, dL_dgamma=dL_dgamma,
                                          dL_df=dL_df, tol=adjoint_tol,
                                          **_adjoint_kw(kw))
        info.dL_dq, info.adjoint_stats = dq, sta
        _require_adjoint("sc_solve_lcp_adjoint", sta)
        return dpos, None, None, None, None, None, None, None, None, None, None


class _LcpSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, particles, box, contacts, u_nc, dt, tol, adjoint_tol, info, kw):
        con = copy.copy(contacts)
        con.q = contacts.q.clone()
        con.q[: con.count] = q.detach().to(torch.float64)
        gamma, g, st, _, _ = solve_lcp(particles, con, tol=tol, **kw)
        info.contacts, info.stats = con, st
        require_solution("sc_solve_lcp", st)
        ctx.state = (particles, box, con, u_nc, dt, adjoint_tol, info, kw)
        ctx.save_for_backward(gamma)
        return gamma

    @staticmethod
    @once_differentiable
    def backward(ctx, dL_dgamma):
        (gamma,) = ctx.saved_tensors
        P, box, con, u_nc, dt, adjoint_tol, info, kw = ctx.state
        dq, dpos, sta = solve_lcp_adjoint(P, box, con, u_nc, dt, gamma, dL_dgamma=dL_dgamma,
                                          tol=adjoint_tol, **_adjoint_kw(kw))
        info.dL_dq, info.adjoint_stats = dq, sta
        _require_adjoint("sc_solve_lcp_adjoint", sta)
        return dq, None, None, None, None, None, None, None, None, None


class _HydroCollisionSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, particles, box, f_ext, hydro_radius, mu, dt, delta, tol, adjoint_tol,
                info):
        P = dataclasses.replace(particles, pos=pos.detach().to(torch.float64).contiguous())
        R = RPY(P.pos, hydro_radius, mu)
        u_nc = R.apply(f_ext)
        con = build_contacts(P, box, delta, u_nc, dt, assemble=False)
        # one persistent launch for small systems, a launch per phase beyond
        # (the same solve; measured faster on each side of this size)
        solve = solve_lcp_rpy if P.n <= PERSISTENT_RPY_MAX_N else solve_lcp_mob
        gamma, g, st, f_c, u_c = solve(P, con, R, tol=tol, want_fc=True)
        info.contacts, info.stats = con, st
        require_solution(solve.__name__, st)
        ctx.state = (P, box, con, R, f_ext, u_nc, dt, adjoint_tol, info)
        ctx.save_for_backward(gamma)
        return gamma, f_c

    @staticmethod
    @once_differentiable
    def backward(ctx, dL_dgamma, dL_df):
        (gamma,) = ctx.saved_tensors
        P, box, con, R, f_ext, u_nc, dt, adjoint_tol, info = ctx.state
        dq, dpos, sta = solve_lcp_adjoint_mob(P, box, con, u_nc, dt, gamma, R, f_ext=f_ext,
                                              dL_dgamma=dL_dgamma, dL_df=dL_df,
                                              tol=adjoint_tol)
        info.dL_dq, info.adjoint_stats = dq, sta
        _require_adjoint("sc_solve_lcp_adjoint_mob", sta)
        return dpos, None, None, None, None, None, None, None, None, None, None


def _require_adjoint(fn, st):
    """The gradient is only that of the solve when the adjoint's CG met its
    tolerance: any other status (the iteration cap included) raises."""
    if st["status"] != A.SC_OK:
        raise A.ScError(fn, st["status"])


def _adjoint_kw(kw):
    keep = ("lanes_per_particle", "grid", "block", "op", "slices_per_wave",
            "lds_entries_per_wave", "workspace")
    return {k: v for k, v in kw.items() if k in keep}


def collision_solve(pos: torch.Tensor, particles: Particles, box: Box, u_nc: torch.Tensor,
                    dt: float, delta: float, tol: float = 1e-6, adjoint_tol: float = 1e-10,
                    info: Optional[SolveInfo] = None, polish: bool = False, **solve_kw):
    """(gamma, F_c, info) for centres ``pos`` [n, 3] (float64, CUDA). The
    other particle properties come from ``particles``; gamma is in the
    library's contact order (``info.contacts``). ``polish``: replace the
    solve's iterate by the exact solution on its active set (sc_polish_lcp,
    to ``adjoint_tol``) before returning and differentiating."""
    info = SolveInfo() if info is None else info
    gamma, f_c = _CollisionSolve.apply(pos, particles, box, u_nc, float(dt), float(delta),
                                       float(tol), float(adjoint_tol), info, solve_kw,
                                       bool(polish))
    return gamma, f_c, info


def lcp_solve(q: torch.Tensor, particles: Particles, box: Box, contacts: Contacts,
              u_nc: torch.Tensor, dt: float, tol: float = 1e-6, adjoint_tol: float = 1e-10,
              info: Optional[SolveInfo] = None, **solve_kw):
    """(gamma, info) of the LCP on ``contacts`` with the given q (library
    contact order); differentiable in q."""
    info = SolveInfo() if info is None else info
    gamma = _LcpSolve.apply(q, particles, box, contacts, u_nc, float(dt), float(tol),
                            float(adjoint_tol), info, solve_kw)
    return gamma, info


def hydro_collision_solve(pos: torch.Tensor, particles: Particles, box: Box,
                          f_ext: torch.Tensor, dt: float, delta: float,
                          hydro_radius: Optional[torch.Tensor] = None, mu: float = 1.0,
                          tol: float = 1e-6, adjoint_tol: float = 1e-10,
                          info: Optional[SolveInfo] = None):
    """(gamma, F_c, info) for sphere centres ``pos`` [n, 3] with the RPY
    mobility (hydrodynamic radii default to the collision radii), external
    forces and torques ``f_ext`` [n, 6]; differentiable in ``pos``. The
    forward solve is one persistent launch up to PERSISTENT_RPY_MAX_N spheres
    (solve_lcp_rpy) and a launch per phase beyond (solve_lcp_mob); the
    backward is the adjoint behind the RPY mobility."""
    info = SolveInfo() if info is None else info
    hr = particles.radius if hydro_radius is None else hydro_radius
    f_ext = f_ext.to(device="cuda", dtype=torch.float64).contiguous()
    hr = hr.to(device="cuda", dtype=torch.float64).contiguous()
    gamma, f_c = _HydroCollisionSolve.apply(pos, particles, box, f_ext, hr, float(mu), float(dt),
                                            float(delta), float(tol), float(adjoint_tol), info)
    return gamma, f_c, info
