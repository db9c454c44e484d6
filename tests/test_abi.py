"""Host-side checks of the C ABI (no GPU needed): the library loads, every
function declared in include/sc_api.h is exported, and argument validation
rejects bad calls before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sc_api.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for fn in ("sc_build_contacts", "sc_solve_lcp", "sc_solve_lcp_adjoint",
               "sc_workspace_bytes", "sc_strerror"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    from paper_1909_06623_amd import _abi as A
    L = A.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) == set(A.SIGNATURES)


def test_strerror_and_version():
    from paper_1909_06623_amd import _abi as A
    L = A.lib()
    assert L.sc_version() >= 100
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert L.sc_strerror(code) != b"unknown status code"
    assert L.sc_strerror(42) == b"unknown status code"


def test_workspace_bytes_monotone():
    from paper_1909_06623_amd import _abi as A
    L = A.lib()
    a = L.sc_workspace_bytes(1000, 5000, A.SC_WS_ALL)
    b = L.sc_workspace_bytes(2000, 5000, A.SC_WS_ALL)
    c = L.sc_workspace_bytes(2000, 10000, A.SC_WS_ALL)
    assert 0 < a < b < c
    assert L.sc_workspace_bytes(-1, 10, A.SC_WS_ALL) == 0
    # per purpose: each no larger than the whole, the whole the largest of them
    parts = [L.sc_workspace_bytes(2000, 10000, w)
             for w in (A.SC_WS_BUILD, A.SC_WS_SOLVE, A.SC_WS_ADJOINT)]
    assert all(0 < x <= c for x in parts) and max(parts) == c
    assert L.sc_workspace_bytes(2000, 10000, 9) == 0


def test_invalid_arguments_rejected_without_device_work():
    from paper_1909_06623_amd import _abi as A
    L = A.lib()
    assert L.sc_build_contacts(None, None, 0.1, None, 1e-3, None, None, 0, None) == A.SC_ERR_INVALID
    p = A.sc_particles(-5, 0, 0, 0, 0, 0, 0)
    assert L.sc_apply_mobility(ctypes.byref(p), None, None, None) == A.SC_ERR_INVALID
    p0 = A.sc_particles(0, 0, 0, 0, 0, 0, 0)
    assert L.sc_apply_mobility(ctypes.byref(p0), None, None, None) == A.SC_OK
    c = A.sc_contacts()
    c.capacity, c.count = 5, 10  # count beyond capacity
    opts = A.sc_solve_opts(1e-6, 100, 1, 0, 0)
    st = A.sc_stats()
    assert L.sc_solve_lcp(ctypes.byref(p0), ctypes.byref(c), ctypes.byref(opts), None, None,
                          None, None, ctypes.byref(st), None, 0, None) == A.SC_ERR_INVALID
    c.count = 0
    bad = A.sc_solve_opts(-1.0, 100, 1, 0, 0)
    assert L.sc_solve_lcp(ctypes.byref(p0), ctypes.byref(c), ctypes.byref(bad), None, None,
                          None, None, ctypes.byref(st), None, 0, None) == A.SC_ERR_INVALID
    bad = A.sc_solve_opts(1e-6, 100, 7, 0, 0)
    assert L.sc_solve_lcp(ctypes.byref(p0), ctypes.byref(c), ctypes.byref(bad), None, None,
                          None, None, ctypes.byref(st), None, 0, None) == A.SC_ERR_INVALID
    for field, value in (("slices_per_wave", 3), ("lds_entries_per_wave", -2),
                         ("lanes_per_particle", 16), ("block", 768), ("op", 3),
                         ("spin_limit", -1)):
        bad = A.sc_solve_opts(1e-6, 100, 1, 0, 0)
        setattr(bad, field, value)
        assert L.sc_solve_lcp(ctypes.byref(p0), ctypes.byref(c), ctypes.byref(bad), None, None,
                              None, None, ctypes.byref(st), None, 0, None) == A.SC_ERR_INVALID
    box = A.sc_box()
    assert L.sc_build_contacts(ctypes.byref(p0), ctypes.byref(box), 0.1, None, 1e-3,
                               ctypes.byref(c), None, 0, None) == A.SC_ERR_INVALID
    # time stepping and batch queries reject bad arguments before any launch
    assert L.sc_advance(-1, None, None, None, None, None, 0.1, None) == A.SC_ERR_INVALID
    assert L.sc_advance(4, None, None, None, None, None, 0.0, None) == A.SC_ERR_INVALID
    assert L.sc_advance(4, None, None, None, None, None, 0.1, None) == A.SC_ERR_INVALID
    assert L.sc_advance(0, None, None, None, None, None, 0.1, None) == A.SC_OK
    assert L.sc_quat_from_axis(-1, None, None, None) == A.SC_ERR_INVALID
    assert L.sc_map_gamma(3, None, None, None, None, None) == A.SC_ERR_INVALID
    assert L.sc_batch_contacts(None, None, None, None, None) == A.SC_ERR_INVALID
    assert L.sc_batch_workspace_bytes(1, None, None) == 0


def test_product_path_has_no_cpu_fallback():
    """The binding raises when the HIP library is missing instead of
    computing anything on the CPU, and never imports the oracle."""
    import paper_1909_06623_amd._abi as A
    import paper_1909_06623_amd.api as api
    import paper_1909_06623_amd.autograd as AG
    import paper_1909_06623_amd.timestep as TS
    src = (open(api.__file__).read() + open(A.__file__).read() + open(AG.__file__).read()
           + open(TS.__file__).read())
    assert "oracle" not in src.replace("oracle.", "")
    saved = A._lib, A.LIB_PATH
    try:
        A._lib = None
        A.LIB_PATH = "/nonexistent/libscgpu.so"
        with pytest.raises(RuntimeError):
            A.lib()
    finally:
        A._lib, A.LIB_PATH = saved


def test_mobility_entry_points_reject_bad_arguments_without_device_work():
    """The solve and adjoint behind a mobility function, the persistent RPY
    solve and the RPY functions validate their arguments before touching the
    device."""
    from paper_1909_06623_amd import _abi as A
    L = A.lib()
    rpy_fn = ctypes.cast(L.sc_rpy_apply, ctypes.c_void_p)
    p0 = A.sc_particles(0, 0, 0, 0, 0, 0, 0)
    c = A.sc_contacts()
    c.capacity, c.count = 0, 0
    st = A.sc_stats()
    opts = A.sc_solve_opts(1e-6, 100, 1, 0, 0)
    # no mobility function; bad options; count beyond capacity
    assert L.sc_solve_lcp_mob(ctypes.byref(p0), ctypes.byref(c), ctypes.byref(opts), None,
                              None, 0, None, None, None, None, ctypes.byref(st), None, 0,
                              None) == A.SC_ERR_INVALID
    for bad in (A.sc_solve_opts(0.0, 100, 1, 0, 0), A.sc_solve_opts(1e-6, -1, 1, 0, 0),
                A.sc_solve_opts(1e-6, 100, 4, 0, 0)):
        assert L.sc_solve_lcp_mob(ctypes.byref(p0), ctypes.byref(c), ctypes.byref(bad), rpy_fn,
                                  None, 0, None, None, None, None, ctypes.byref(st), None, 0,
                                  None) == A.SC_ERR_INVALID
    assert L.sc_solve_lcp_mob(ctypes.byref(p0), ctypes.byref(c), ctypes.byref(opts), rpy_fn,
                              None, -1, None, None, None, None, ctypes.byref(st), None, 0,
                              None) == A.SC_ERR_INVALID
    c.capacity, c.count = 2, 3
    assert L.sc_solve_lcp_mob(ctypes.byref(p0), ctypes.byref(c), ctypes.byref(opts), rpy_fn,
                              None, 0, None, None, None, None, ctypes.byref(st), None, 0,
                              None) == A.SC_ERR_INVALID
    c.capacity, c.count = 0, 0
    # the adjoint: no mobility, dt <= 0, tol <= 0
    box = A.sc_box()
    aopts = A.sc_adjoint_opts(1e-10, 100)
    args = lambda dt, o, fn: (ctypes.byref(p0), ctypes.byref(box), ctypes.byref(c), None, None,
                              dt, None, None, None, fn, None, None, None, ctypes.byref(o), 0,
                              None, None, ctypes.byref(st), None, 0, None)
    assert L.sc_solve_lcp_adjoint_mob(*args(1e-3, aopts, None)) == A.SC_ERR_INVALID
    assert L.sc_solve_lcp_adjoint_mob(*args(0.0, aopts, rpy_fn)) == A.SC_ERR_INVALID
    assert L.sc_solve_lcp_adjoint_mob(*args(1e-3, A.sc_adjoint_opts(0.0, 100), rpy_fn)) == \
        A.SC_ERR_INVALID
    # RPY: n mismatch, mu <= 0, no work buffer; n = 0 is a no-op
    R = A.sc_rpy(4, 0, 0, 0, 1.0, 0, 0)
    assert L.sc_rpy_apply(ctypes.addressof(R), 3, None, None, None) == A.SC_ERR_INVALID
    assert L.sc_rpy_grad(ctypes.addressof(R), 3, None, None, None, None) == A.SC_ERR_INVALID
    R.mu = 0.0
    assert L.sc_rpy_apply(ctypes.addressof(R), 4, None, None, None) == A.SC_ERR_INVALID
    R.mu = 1.0
    R.pos, R.radius = 256, 256
    assert L.sc_rpy_apply(ctypes.addressof(R), 4, 256, 256, None) == A.SC_ERR_WORKSPACE
    R0 = A.sc_rpy(0, 0, 0, 0, 1.0, 0, 0)
    assert L.sc_rpy_apply(ctypes.addressof(R0), 0, None, None, None) == A.SC_OK
    assert L.sc_rpy_work_bytes(1000) >= 3 * 8 * 1000
    assert L.sc_solve_mob_work_bytes(-1, 10) == 0 and L.sc_adjoint_mob_work_bytes(10, -1) == 0
    # the persistent RPY solve: missing RPY, bad options, particle counts that
    # differ, mu <= 0, count beyond capacity
    Rp = A.sc_rpy(0, 0, 0, 0, 1.0, 0, 0)
    pers = lambda r, o: L.sc_solve_lcp_rpy(ctypes.byref(p0), ctypes.byref(c), r, ctypes.byref(o),
                                           None, None, None, None, ctypes.byref(st), None, 0,
                                           None)
    assert pers(None, opts) == A.SC_ERR_INVALID
    for bad in (A.sc_solve_opts(0.0, 100, 1, 0, 0), A.sc_solve_opts(1e-6, -1, 1, 0, 0),
                A.sc_solve_opts(1e-6, 100, 0, 0, 0), A.sc_solve_opts(1e-6, 100, 1, 0, 0, -1),
                A.sc_solve_opts(1e-6, 100, 1, 0, 0, 0, 0, 0, 0, 0, -1)):
        assert pers(ctypes.addressof(Rp), bad) == A.SC_ERR_INVALID
    Rp.n = 4
    assert pers(ctypes.addressof(Rp), opts) == A.SC_ERR_INVALID
    Rp.n, Rp.mu = 0, -1.0
    assert pers(ctypes.addressof(Rp), opts) == A.SC_ERR_INVALID
    Rp.mu = 1.0
    c.capacity, c.count = 2, 3
    assert pers(ctypes.addressof(Rp), opts) == A.SC_ERR_INVALID
    c.capacity, c.count = 0, 0
    assert L.sc_solve_rpy_work_bytes(-1, 10) == 0 and L.sc_solve_rpy_work_bytes(10, -1) == 0
    assert L.sc_solve_rpy_work_bytes(1000, 3000) >= 2 * 8 * 3000 + 6 * 8 * 1000


def test_stream_ordered_entry_points_reject_bad_calls_without_device_work():
    """sc_canonical_order and sc_solve_lcp_async check their arguments on
    the host before anything is enqueued."""
    from paper_1909_06623_amd import _abi as A
    L = A.lib()
    assert L.sc_canonical_order(3, None, None, None, 0, None) == A.SC_ERR_INVALID
    c = A.sc_contacts()
    c.capacity, c.count = 5, 10
    assert L.sc_canonical_order(3, ctypes.byref(c), None, None, 0, None) == A.SC_ERR_INVALID
    c.count = 2  # no plan buffer
    assert L.sc_canonical_order(3, ctypes.byref(c), None, None, 0, None) == A.SC_ERR_INVALID
    assert L.sc_canonical_order(-1, ctypes.byref(c), None, None, 0, None) == A.SC_ERR_INVALID
    p0 = A.sc_particles(0, 0, 0, 0, 0, 0, 0)
    c.count = 0
    opts = A.sc_solve_opts(1e-6, 100, 1, 0, 0)
    # no device stats record
    assert L.sc_solve_lcp_async(ctypes.byref(p0), ctypes.byref(c), ctypes.byref(opts), None,
                                None, None, None, None, None, 0, None) == A.SC_ERR_INVALID
    bad = A.sc_solve_opts(0.0, 100, 1, 0, 0)
    assert L.sc_solve_lcp_async(ctypes.byref(p0), ctypes.byref(c), ctypes.byref(bad), None,
                                None, None, None, ctypes.c_void_p(256), None, 0,
                                None) == A.SC_ERR_INVALID
    bad = A.sc_solve_opts(1e-6, 100, 4, 0, 0)
    assert L.sc_solve_lcp_async(ctypes.byref(p0), ctypes.byref(c), ctypes.byref(bad), None,
                                None, None, None, ctypes.c_void_p(256), None, 0,
                                None) == A.SC_ERR_INVALID


def test_noalloc_solve_rejects_oversized_systems_on_the_host():
    """The allocation-free solve refuses, before any device work, a system
    whose workspace exceeds its static scratch array."""
    from paper_1909_06623_amd import _abi as A
    L = A.lib()
    p = A.sc_particles(100000, 0, 0, 0, 0, 0, 0)
    c = A.sc_contacts()
    c.capacity, c.count = 4_000_000, 0
    opts = A.sc_solve_opts(1e-6, 100, 1, 0, 0)
    st = A.sc_stats()
    assert L.sc_solve_lcp_noalloc(ctypes.byref(p), ctypes.byref(c), ctypes.byref(opts), None,
                                  None, None, None, ctypes.byref(st), None) == A.SC_ERR_WORKSPACE
    assert L.sc_solve_lcp_noalloc(None, ctypes.byref(c), ctypes.byref(opts), None, None, None,
                                  None, ctypes.byref(st), None) == A.SC_ERR_INVALID


def test_batch_options_rejected_on_the_host():
    """sc_batch_create checks its team policy options before any device work:
    a team size and a size-class target for the same launch, negative
    targets, team and block sizes outside their sets."""
    from paper_1909_06623_amd import _abi as A
    L = A.lib()

    def opts(**kw):
        o = A.sc_batch_opts()
        o.tol, o.max_iter, o.bb = 1e-6, 100, 1
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    out = ctypes.c_void_p(1)
    for bad in (dict(team=4, nnz_per_workgroup=1000),
                dict(adjoint_team=2, adjoint_nnz_per_workgroup=10),
                dict(nnz_per_workgroup=-1), dict(adjoint_nnz_per_workgroup=-5), dict(team=3),
                dict(adjoint_team=64), dict(block=300), dict(adjoint_block=768), dict(bb=4),
                dict(tol=0.0)):
        o = opts(**bad)
        assert L.sc_batch_create(0, None, ctypes.byref(o), None, 0, None,
                                 ctypes.byref(out)) == A.SC_ERR_INVALID, bad
        assert out.value is None, bad


def test_tuned_policy_recreates_each_launch():
    """Batch.tuned_policy turns an autotuned batch's info into the options
    that recreate it: size classes when a target was picked, else the team."""
    from paper_1909_06623_amd.api import Batch
    info = {"team": 32, "nnz_per_workgroup": 32768, "team_adjoint": 8,
            "adjoint_nnz_per_workgroup": 0}
    assert Batch.tuned_policy(info) == {"team": 0, "nnz_per_workgroup": 32768,
                                        "adjoint_team": 8, "adjoint_nnz_per_workgroup": 0}
    info = {"team": 16, "nnz_per_workgroup": 0, "team_adjoint": 32,
            "adjoint_nnz_per_workgroup": 16384}
    assert Batch.tuned_policy(info) == {"team": 16, "nnz_per_workgroup": 0,
                                        "adjoint_team": 0, "adjoint_nnz_per_workgroup": 16384}


def test_polish_rejects_bad_arguments_without_device_work():
    """sc_polish_lcp checks its arguments on the host before any launch."""
    from paper_1909_06623_amd import _abi as A
    L = A.lib()
    p0 = A.sc_particles(0, 0, 0, 0, 0, 0, 0)
    c = A.sc_contacts()
    c.capacity, c.count = 5, 10  # count beyond capacity
    o = A.sc_adjoint_opts(1e-12, 100, 0, 0, 0, 0, 0, 0)
    st = A.sc_stats()
    args = lambda pp, cc, oo, mp, ss: L.sc_polish_lcp(pp, cc, None, None, None, None, oo, mp,
                                                      ss, None, 0, None)
    assert args(ctypes.byref(p0), ctypes.byref(c), ctypes.byref(o), 0,
                ctypes.byref(st)) == A.SC_ERR_INVALID
    c.count = 0
    assert args(None, ctypes.byref(c), ctypes.byref(o), 0, ctypes.byref(st)) == A.SC_ERR_INVALID
    assert args(ctypes.byref(p0), ctypes.byref(c), None, 0, ctypes.byref(st)) == A.SC_ERR_INVALID
    assert args(ctypes.byref(p0), ctypes.byref(c), ctypes.byref(o), -1,
                ctypes.byref(st)) == A.SC_ERR_INVALID
    assert args(ctypes.byref(p0), ctypes.byref(c), ctypes.byref(o), 0, None) == A.SC_ERR_INVALID
    for field, value in (("tol", 0.0), ("max_iter", -1), ("block", 300), ("op", 3),
                         ("lanes_per_particle", 3)):
        bad = A.sc_adjoint_opts(1e-12, 100, 0, 0, 0, 0, 0, 0)
        setattr(bad, field, value)
        assert args(ctypes.byref(p0), ctypes.byref(c), ctypes.byref(bad), 0,
                    ctypes.byref(st)) == A.SC_ERR_INVALID, field
