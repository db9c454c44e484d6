"""ctypes view of the C ABI declared in include/sc_api.h (structs, codes,
function signatures). Loading fails loudly if the HIP library is not built:
there is no fallback implementation."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libscgpu.so")

SC_OK = 0
SC_NOT_CONVERGED = 1
SC_ERR_INVALID = -1
SC_ERR_CAPACITY = -2
SC_ERR_NONFINITE = -3
SC_ERR_BOX = -4
SC_ERR_HIP = -5
SC_ERR_WORKSPACE = -6
SC_ERR_TIMEOUT = -7

SC_NOALLOC_SCRATCH_BYTES = 64 << 20

SC_WS_ALL = 0
SC_WS_BUILD = 1
SC_WS_SOLVE = 2
SC_WS_ADJOINT = 3

SC_OP_AUTO = 0
SC_OP_CHAIN = 1
SC_OP_MATRIX = 2
SC_OP_CALLBACK = 3
SC_OP_RPY = 4

c_dp = ctypes.c_void_p  # device pointers travel as plain addresses


class sc_particles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("pos", c_dp), ("axis", c_dp), ("radius", c_dp),
                ("half_len", c_dp), ("mob", c_dp)]


class sc_box(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("len", ctypes.c_double * 3),
                ("periodic", ctypes.c_int32), ("walls", ctypes.c_int32)]


class sc_contacts(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int32), ("count", ctypes.c_int32),
                ("ci", c_dp), ("cj", c_dp), ("phi", c_dp), ("q", c_dp),
                ("frame", c_dp), ("plan", c_dp), ("plan_bytes", ctypes.c_size_t),
                ("n_parallel", ctypes.c_int32), ("n_zero_dist", ctypes.c_int32),
                ("n_borderline", ctypes.c_int32), ("grid", ctypes.c_int32 * 3),
                ("nnz", ctypes.c_int64), ("mat", c_dp), ("mat_bytes", ctypes.c_size_t),
                ("mat_ready", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class sc_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("bb", ctypes.c_int32), ("warm_start", ctypes.c_int32),
                ("lanes_per_particle", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("block", ctypes.c_int32), ("op", ctypes.c_int32),
                ("slices_per_wave", ctypes.c_int32), ("lds_entries_per_wave", ctypes.c_int32),
                ("spin_limit", ctypes.c_int32)]


class sc_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("mvops", ctypes.c_int32), ("n_active", ctypes.c_int32),
                ("residual", ctypes.c_double), ("alpha", ctypes.c_double),
                ("n_degenerate", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("kernel_ms", ctypes.c_double), ("lanes_per_particle", ctypes.c_int32),
                ("block", ctypes.c_int32), ("op", ctypes.c_int32),
                ("slices_per_wave", ctypes.c_int32), ("lds_entries_per_wave", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("reserved")}


class sc_adjoint_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("lanes_per_particle", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("block", ctypes.c_int32), ("op", ctypes.c_int32),
                ("slices_per_wave", ctypes.c_int32), ("lds_entries_per_wave", ctypes.c_int32)]


class sc_batch_item(ctypes.Structure):
    _fields_ = [("p", sc_particles), ("c", sc_contacts), ("gamma", c_dp), ("g", c_dp),
                ("box", sc_box), ("u_nc", c_dp), ("dt", ctypes.c_double),
                ("delta", ctypes.c_double), ("dL_dgamma", c_dp), ("dL_dq", c_dp),
                ("dL_dpos", c_dp)]


class sc_batch_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("bb", ctypes.c_int32), ("warm_start", ctypes.c_int32),
                ("team", ctypes.c_int32), ("block", ctypes.c_int32),
                ("adjoint", ctypes.c_int32), ("adjoint_tol", ctypes.c_double),
                ("adjoint_max_iter", ctypes.c_int32), ("build", ctypes.c_int32),
                ("adjoint_team", ctypes.c_int32), ("nnz_per_workgroup", ctypes.c_int32),
                ("adjoint_nnz_per_workgroup", ctypes.c_int32), ("adjoint_block", ctypes.c_int32)]


class sc_batch_info(ctypes.Structure):
    _fields_ = [("team", ctypes.c_int32), ("block", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("lds_entries_per_wave", ctypes.c_int32),
                ("tune_ms", ctypes.c_float * 12), ("team_adjoint", ctypes.c_int32),
                ("tune_adjoint_ms", ctypes.c_float * 12),
                ("nnz_per_workgroup", ctypes.c_int32),
                ("adjoint_nnz_per_workgroup", ctypes.c_int32),
                ("adjoint_block", ctypes.c_int32)]


class sc_rpy(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved", ctypes.c_int32), ("pos", c_dp),
                ("radius", c_dp), ("mu", ctypes.c_double), ("work", c_dp),
                ("work_bytes", ctypes.c_size_t)]


# int (*)(void *ctx, int32_t n, const double *f, double *u, void *stream)
MOBILITY_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p)

# int (*)(void *ctx, int32_t n, const double *a, const double *f, double *g, void *stream)
MOBILITY_GRAD_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p)

P = ctypes.POINTER
SIGNATURES = {
    "sc_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "sc_plan_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "sc_matrix_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int64]),
    "sc_assemble_matrix": (ctypes.c_int, [P(sc_particles), P(sc_contacts), c_dp]),
    "sc_apply_mobility": (ctypes.c_int, [P(sc_particles), c_dp, c_dp, c_dp]),
    "sc_build_contacts": (ctypes.c_int, [P(sc_particles), P(sc_box), ctypes.c_double,
                                         c_dp, ctypes.c_double, P(sc_contacts), c_dp,
                                         ctypes.c_size_t, c_dp]),
    "sc_canonical_order": (ctypes.c_int, [ctypes.c_int32, P(sc_contacts), c_dp, c_dp,
                                          ctypes.c_size_t, c_dp]),
    "sc_mvop": (ctypes.c_int, [P(sc_particles), P(sc_contacts), c_dp, c_dp, c_dp,
                               ctypes.c_size_t, c_dp]),
    "sc_solve_lcp": (ctypes.c_int, [P(sc_particles), P(sc_contacts), P(sc_solve_opts),
                                    c_dp, c_dp, c_dp, c_dp, P(sc_stats), c_dp,
                                    ctypes.c_size_t, c_dp]),
    "sc_solve_lcp_noalloc": (ctypes.c_int, [P(sc_particles), P(sc_contacts),
                                            P(sc_solve_opts), c_dp, c_dp, c_dp, c_dp,
                                            P(sc_stats), c_dp]),
    "sc_solve_lcp_async": (ctypes.c_int, [P(sc_particles), P(sc_contacts),
                                          P(sc_solve_opts), c_dp, c_dp, c_dp, c_dp, c_dp,
                                          c_dp, ctypes.c_size_t, c_dp]),
    "sc_solve_lcp_adjoint": (ctypes.c_int, [P(sc_particles), P(sc_box), P(sc_contacts),
                                            c_dp, ctypes.c_double, c_dp, c_dp, c_dp,
                                            c_dp, c_dp, P(sc_adjoint_opts), P(sc_stats),
                                            c_dp, ctypes.c_size_t, c_dp]),
    "sc_polish_lcp": (ctypes.c_int, [P(sc_particles), P(sc_contacts), c_dp, c_dp, c_dp, c_dp,
                                     P(sc_adjoint_opts), ctypes.c_int32, P(sc_stats), c_dp,
                                     ctypes.c_size_t, c_dp]),
    "sc_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, P(sc_batch_item),
                                                   P(sc_batch_opts)]),
    "sc_batch_create": (ctypes.c_int, [ctypes.c_int32, P(sc_batch_item), P(sc_batch_opts),
                                       c_dp, ctypes.c_size_t, c_dp, P(ctypes.c_void_p)]),
    "sc_batch_solve": (ctypes.c_int, [c_dp, c_dp]),
    "sc_batch_graph_launch": (ctypes.c_int, [c_dp, c_dp]),
    "sc_batch_stats": (ctypes.c_int, [c_dp, P(sc_stats), P(sc_stats), P(sc_batch_info), c_dp]),
    "sc_batch_contacts": (ctypes.c_int, [c_dp, P(ctypes.c_int32), P(ctypes.c_int64),
                                         P(ctypes.c_int32), c_dp]),
    "sc_batch_destroy": (None, [c_dp]),
    "sc_advance": (ctypes.c_int, [ctypes.c_int32, c_dp, c_dp, c_dp, c_dp, c_dp,
                                  ctypes.c_double, c_dp]),
    "sc_quat_from_axis": (ctypes.c_int, [ctypes.c_int32, c_dp, c_dp, c_dp]),
    "sc_map_gamma": (ctypes.c_int, [ctypes.c_int32, P(sc_contacts), c_dp, P(sc_contacts),
                                    c_dp, c_dp]),
    "sc_rpy_work_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "sc_rpy_apply": (ctypes.c_int, [c_dp, ctypes.c_int32, c_dp, c_dp, c_dp]),
    "sc_dry_apply": (ctypes.c_int, [c_dp, ctypes.c_int32, c_dp, c_dp, c_dp]),
    "sc_solve_mob_work_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "sc_solve_lcp_mob": (ctypes.c_int, [P(sc_particles), P(sc_contacts), P(sc_solve_opts),
                                        c_dp, c_dp, ctypes.c_int32, c_dp, c_dp, c_dp, c_dp,
                                        P(sc_stats), c_dp, ctypes.c_size_t, c_dp]),
    "sc_rpy_grad": (ctypes.c_int, [c_dp, ctypes.c_int32, c_dp, c_dp, c_dp, c_dp]),
    "sc_adjoint_mob_work_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "sc_solve_lcp_adjoint_mob": (ctypes.c_int, [P(sc_particles), P(sc_box), P(sc_contacts),
                                                c_dp, c_dp, ctypes.c_double, c_dp, c_dp, c_dp,
                                                c_dp, c_dp, c_dp, c_dp, P(sc_adjoint_opts),
                                                ctypes.c_int32, c_dp, c_dp, P(sc_stats), c_dp,
                                                ctypes.c_size_t, c_dp]),
    "sc_solve_rpy_work_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "sc_solve_lcp_rpy": (ctypes.c_int, [P(sc_particles), P(sc_contacts), c_dp,
                                        P(sc_solve_opts), c_dp, c_dp, c_dp, c_dp, P(sc_stats),
                                        c_dp, ctypes.c_size_t, c_dp]),
    "sc_release": (ctypes.c_int, []),
    "sc_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "sc_version": (ctypes.c_int, []),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library {LIB_PATH} is not built; run "
                "`python -c 'import __graft_entry__ as g; g.build()'` first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class ScError(RuntimeError):
    def __init__(self, fn, code):
        self.code = code
        msg = lib().sc_strerror(code).decode()
        super().__init__(f"{fn} failed with code {code}: {msg}")
