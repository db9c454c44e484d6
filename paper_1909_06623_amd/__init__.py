"""MI355X-native collision resolution for rigid-particle suspensions.

Contact detection and Barzilai-Borwein projected gradient descent for the
collision LCP of Yan et al. (arXiv:1909.06623, section 3), as hand-written HIP
kernels for gfx950 behind a C ABI (include/sc_api.h). This package is the thin
Python binding: PyTorch provides device memory and streams only.
"""
from ._abi import ScError, LIB_PATH  # noqa: F401
from .api import (RPY, Batch, Box, Contacts, DryMobility, FnMobility, Particles,  # noqa: F401
                  Workspace, apply_mobility, release, build_contacts, mvop, polish_lcp, solve_lcp,
                  solve_lcp_adjoint, solve_lcp_adjoint_mob, solve_lcp_mob, solve_lcp_noalloc,
                  solve_lcp_rpy, solve_lcp_async, stats_from_device, STATS_BYTES)
from .autograd import SolveInfo, collision_solve, hydro_collision_solve, lcp_solve  # noqa: F401

__all__ = ["Batch", "Box", "Contacts", "DryMobility", "FnMobility", "Particles", "RPY",
           "Workspace", "apply_mobility", "release", "build_contacts", "mvop", "polish_lcp",
           "solve_lcp", "solve_lcp_adjoint",
           "solve_lcp_adjoint_mob", "solve_lcp_mob", "solve_lcp_noalloc", "solve_lcp_rpy", "solve_lcp_async",
           "stats_from_device", "STATS_BYTES", "ScError",
           "SolveInfo", "collision_solve", "hydro_collision_solve", "lcp_solve"]
