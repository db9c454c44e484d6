"""Benchmark: contact detection + BBPGD solve to ||min(gamma, g)|| < 1e-6 on
100,000 spherocylinders (length 1, diameter 0.05, ~6 close pairs per rod,
isotropic, periodic box), FP64, one MI355X.

One step = build_contacts (cell binning, pairs, D, q, assembled M) +
solve_lcp on the resident synthetic inputs. Prints one JSON line: whole-job
throughput in rods/s, the HBM roofline of the persistent BBPGD kernel
(algorithmic bytes of the method's iterations over the kernel's HIP-event
time), the adjoint/forward time ratio (loss 1/2 ||D gamma||^2), and the FP64
oracle timed on the host for comparison.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Counter summary of the solve kernel on this workload (rocprofv3 FETCH_SIZE
# and WRITE_SIZE passes, scaled by a plain-copy calibration).
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_bbpgd_mat_rods100k_traffic.json")
TRAFFIC_FILE_LARGE = os.path.join(ROOT, "profiles", "k_bbpgd_mat_rods1M_spheres100k_traffic.json")
# Sources that define the persistent matrix solve kernel.
KERNEL_SOURCES = ["sc_matrix.hip", "sc_matrix.hpp", "sc_matrix_pass.hpp", "sc_chain.hpp", "sc_sync.hpp",
                  "sc_common.hpp"]


def iteration_bytes(nc, n, rods=True):
    """Algorithmic bytes of one BBPGD iteration (one product M gamma = D^T Mob
    D gamma with the BB step and reductions), with D kept compact and read
    twice. Rods: per contact an 80-byte D record read twice, 8 bytes of
    incidence and 48 bytes of gamma/g/q traffic; per particle U written and
    read (96) and the axis (24). Spheres: 32-byte records, U of 3 entries."""
    return 216 * nc + 120 * n if rods else 120 * nc + 56 * n


def mixed_iteration_bytes(nc_rod, nc_sph, n_rod, n_sph):
    """iteration_bytes for a mixture: contacts that involve a rod and rods
    priced as rods, sphere-sphere contacts and spheres as spheres."""
    return 216 * nc_rod + 120 * nc_sph + 120 * n_rod + 56 * n_sph


def large(sc, W, torch, np, steps=3):
    """Forward solve of the 1,000,000-rod + 100,000-sphere suspension (aligned
    rods, Watson kappa 5): the largest single-GPU configuration, whose
    iterate records and operator (about 0.7 GB per product) do not fit the
    caches, so its roofline is the HBM one. One warm-up solve, then `steps`
    timed solves (HIP events of the persistent kernel on its stream)."""
    s = W.workload(3)
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box))
    u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    con = sc.build_contacts(P, box, s.delta, u_nc, s.dt)
    torch.cuda.synchronize()
    build_ms = 1e3 * (time.perf_counter() - t0)
    sts = [sc.solve_lcp(P, con, tol=s.tol)[2] for _ in range(steps + 1)][1:]
    st = sts[-1]
    ci = con.i.cpu().numpy()
    cj = con.j.cpu().numpy()
    sph = s.half_len == 0
    nc_sph = int(np.count_nonzero(sph[ci] & sph[cj]))
    n_sph = int(np.count_nonzero(sph))
    bytes_iter = mixed_iteration_bytes(con.count - nc_sph, nc_sph, s.n - n_sph, n_sph)
    products = st["iters"] + 2
    kernel_ms = float(np.mean([x["kernel_ms"] for x in sts]))
    achieved = bytes_iter * products / (kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic(st["iters"], TRAFFIC_FILE_LARGE)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "algorithmic_frac": achieved / HBM_PEAK_GBS,
            "hbm_frac": (None if traffic is None
                         else traffic / (kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS),
            "kernel": "k_bbpgd_mat (persistent BBPGD solve, one launch per solve)",
            "bytes_model": "216 n_c,rod + 120 n_c,sph + 120 N_rod + 56 N_sph bytes per "
                           "product (contacts touching a rod priced as rods), (iterations "
                           "+ 2) products per launch",
            "bytes_per_product": bytes_iter, "products_per_launch": products,
            "bytes_per_launch": bytes_iter * products, "launch_ms": kernel_ms,
            "us_per_product": 1e3 * kernel_ms / products, "grid": st["grid"],
            "lds_entries_per_wave": st["lds_entries_per_wave"]}
    return {"workload": "1,000,000 spherocylinders (Watson-aligned, kappa 5) + 100,000 "
                        "spheres D=0.1, periodic box 27.864, delta 0.015, BBPGD (BB1) to 1e-6",
            "n": s.n, "n_contacts": con.count, "nnz_M": con.nnz, "iters": st["iters"],
            "status": st["status"], "build_ms": build_ms, "solve_ms": kernel_ms,
            "rods_per_s": s.n / (kernel_ms * 1e-3), "roofline": roof}


def chain_roofline(st, bytes_iter):
    """Roofline of the matrix-free two-pass solve (k_bbpgd) under the same
    model as the main leg; its counter bytes are in profiles/k_bbpgd_rods100k.md."""
    products = st["iters"] + 2
    gbs = bytes_iter * products / (st["kernel_ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": None,
            "kernel": "k_bbpgd (persistent BBPGD, matrix-free two-pass product)",
            "bytes_per_product": bytes_iter, "products_per_launch": products,
            "launch_ms": st["kernel_ms"], "lds_entries_per_wave": st["lds_entries_per_wave"]}


def spheres1000(sc, W, torch, np, steps):
    """The 1000-sphere suspension (radius 0.5, volume fraction 0.3, delta
    0.1, dt 1e-3): contact build + BBPGD to 1e-6 per step, as the main leg;
    latency-bound at this size (a few hundred contacts per workgroup)."""
    s = W.workload(1)
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box))
    u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
    ws = sc.Workspace()
    con = sc.build_contacts(P, box, s.delta, u_nc, s.dt, workspace=ws)
    cap = con.capacity
    for _ in range(3):
        sc.build_contacts(P, box, s.delta, u_nc, s.dt, capacity=cap, workspace=ws)
        sc.solve_lcp(P, con, tol=s.tol, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts = []
    for _ in range(steps):
        con = sc.build_contacts(P, box, s.delta, u_nc, s.dt, capacity=cap, workspace=ws)
        sts.append(sc.solve_lcp(P, con, tol=s.tol, workspace=ws)[2])
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    st = sts[-1]
    products = st["iters"] + 2
    kernel_ms = float(np.mean([x["kernel_ms"] for x in sts]))
    bytes_iter = iteration_bytes(con.count, s.n, rods=False)
    gbs = bytes_iter * products / (kernel_ms * 1e-3) / 1e9
    # the same step with no host synchronisation: a batch of this one system
    # built on the device, replayed as one HIP graph (build, M, solve), on a
    # team of workgroups that share one XCD
    graph = {}
    for team in (4, 8):
        b = sc.Batch([(P, box, s.delta, u_nc, s.dt)], tol=s.tol, team=team, build=True)
        for _ in range(3):
            b.graph_solve()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            b.graph_solve()
        torch.cuda.synchronize()
        gms = 1e3 * (time.perf_counter() - t1) / steps
        bst, _, _ = b.stats()
        (gnc, _, gstatus), = b.counts()
        graph[f"team{team}"] = {"ms_per_step": gms, "iters": bst[0]["iters"],
                                "status": max(bst[0]["status"], gstatus), "n_contacts": gnc}
        b.close()
    return {"workload": "1000 spheres R=0.5, volume fraction 0.3, periodic box 12.04, delta 0.1, "
                        "dt 1e-3, BBPGD (BB1) to 1e-6",
            "graph_step": dict(graph, note="one-system batch with build=True replayed as a HIP "
                                           "graph: contact build, M and the solve with no host "
                                           "synchronisation, on one XCD's team"),
            "n": s.n, "n_contacts": con.count, "iters": st["iters"], "status": st["status"],
            "ms_per_step": ms, "particles_per_s": s.n / (ms * 1e-3), "solve_kernel_ms": kernel_ms,
            "us_per_product": 1e3 * kernel_ms / products, "grid": st["grid"],
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k_bbpgd_mat (persistent BBPGD solve)",
                         "bytes_model": "120 n_c + 56 N bytes per product (spheres), (iterations "
                                        "+ 2) products per launch",
                         "bytes_per_product": bytes_iter, "launch_ms": kernel_ms,
                         "note": "0.25 MB per product: bound by the per-iteration latency "
                                 "(gathers, barrier, reduction), not by memory; the grid is "
                                 "chosen from nnz(M)"}}


def timestepping(sc, W, torch, np, steps):
    """Euler time steps (contacts rebuilt, LCP solved, centres and
    quaternions advanced) of the 100,000-rod suspension, with and without
    warm-starting each LCP from the previous step's forces."""
    from paper_1909_06623_amd import timestep as ts
    out = {"steps": steps}
    for warm in (True, False):
        s = W.workload(2)
        P = sc.Particles.from_suspension(s)
        stp = ts.TimeStepper(P, sc.Box(tuple(s.box)), s.delta, s.dt,
                             torch.from_numpy(s.f_ext).cuda(), tol=s.tol, warm_start=warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = [stp.step() for _ in range(steps)]
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        key = "warm" if warm else "cold"
        out[key] = {"ms_per_step": ms, "iters": [x.stats["iters"] for x in infos],
                    "contacts": [x.contacts.count for x in infos],
                    "all_converged": all(x.stats["status"] == 0 for x in infos)}
    return out


# FP64 operations of one ordered pair of the RPY sum as the kernel evaluates
# the far-field branch (every add, multiply and the square-root estimate
# counted once, a fused multiply-add as two): difference 3, r^2 5, radius
# test 2, 1/r with two Newton steps 10, coefficients 12, d.F 5, update 13.
RPY_FLOPS_PER_PAIR = 50
FP64_VECTOR_PEAK_TFLOPS = 78.6


def hydro(sc, W, torch, np, steps):
    """The solve behind a non-diagonal mobility (RPY): the RPY product on a
    20,000-sphere cluster (ALU roofline of the pair kernel), a solve through
    RPY of 20,000 overlapping spheres in free space, and time steps of the
    1000-sphere sedimenting cluster of section 6.3 (and of a 20,000-sphere
    one)."""
    from paper_1909_06623_amd import timestep as ts
    out = {}
    s = W.sphere_cluster(20000, W.SEED_BASE + 901)
    R = sc.RPY(torch.from_numpy(s.pos).cuda(), torch.from_numpy(s.hydro_radius).cuda())
    F = torch.from_numpy(np.random.default_rng(1).standard_normal((s.n, 6))).cuda()
    # one product captured in a HIP graph (its two kernels, no memset) and
    # replayed, so that host-side call overhead stays out of the timing
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(3):
            R.apply(F)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        U_g = R.apply(F)
    U_e = R.apply(F)
    graph.replay()
    torch.cuda.synchronize()
    if not torch.equal(U_g, U_e):
        raise RuntimeError("graph replay of the RPY product differs from the eager call")
    # warm replays first (about 20 ms of FP64 work: the first products after
    # the memory-bound legs run at lower clocks), then the timed ones
    for _ in range(40):
        graph.replay()
    reps = 50
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = RPY_FLOPS_PER_PAIR * s.n * (s.n - 1)
    tf = flops / (ms * 1e-3) / 1e12
    out["rpy_product"] = {
        "workload": "20000-sphere cluster (section 6.3 recipe), random forces",
        "n": s.n, "ms": ms, "pairs_per_s": s.n * (s.n - 1) / (ms * 1e-3),
        "roofline": {"bound": "alu", "achieved": tf, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": tf / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_rpy_pairs + k_rpy_finish (one sc_rpy_apply, HIP graph "
                               "replays)",
                     "flops_model": f"{RPY_FLOPS_PER_PAIR} FP64 flops per ordered pair"}}

    s = W.spheres(20000, 0.3, W.SEED_BASE + 909)
    s.periodic = 0
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box), periodic=False)
    R = sc.RPY(P.pos, P.radius)
    u_nc = R.apply(torch.from_numpy(s.f_ext).cuda())
    con = sc.build_contacts(P, box, s.delta, u_nc, s.dt, assemble=False)
    sc.solve_lcp_mob(P, con, R, tol=s.tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gam, g, st, _, _ = sc.solve_lcp_mob(P, con, R, tol=s.tol)
    wall = 1e3 * (time.perf_counter() - t0)
    out["solve_rpy"] = {
        "workload": "20000 overlapping spheres (phi 0.3, uniform centres) in free space, "
                    "RPY mobility, BB1 to 1e-6",
        "n": s.n, "n_contacts": con.count, "status": st["status"], "iters": st["iters"],
        "mvops": st["mvops"], "n_active": st["n_active"], "solve_ms": wall,
        "gpu_ms": st["kernel_ms"], "ms_per_product": st["kernel_ms"] / max(1, st["mvops"]),
        "rpy_share": min(1.0, ms * st["mvops"] / max(1e-9, st["kernel_ms"]))}
    # the adjoint of L = 1/2 ||D gamma||^2 through RPY (CG, geometric terms and
    # the RPY centre gradient)
    fe = torch.from_numpy(s.f_ext).cuda()
    gam, _, _, f_c, _ = sc.solve_lcp_mob(P, con, R, tol=s.tol, want_fc=True)
    sc.solve_lcp_adjoint_mob(P, box, con, u_nc, s.dt, gam, R, f_ext=fe, dL_df=f_c, tol=1e-10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, sta = sc.solve_lcp_adjoint_mob(P, box, con, u_nc, s.dt, gam, R, f_ext=fe, dL_df=f_c,
                                         tol=1e-10)
    adj_ms = 1e3 * (time.perf_counter() - t0)
    out["solve_rpy"]["adjoint"] = {"ms": adj_ms, "status": sta["status"], "cg_iters": sta["iters"],
                                   "adjoint_forward_ratio": adj_ms / wall}

    # cold solves of the 1000-sphere cluster: one persistent launch against a
    # launch per phase (the same iteration; host wall clock over 20 solves
    # after a synchronisation)
    s = W.sphere_cluster(1000, W.SEED_BASE + 900)
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box), lo=tuple(s.lo), periodic=False)
    R = sc.RPY(P.pos, torch.from_numpy(s.hydro_radius).cuda())
    con = sc.build_contacts(P, box, s.delta, R.apply(torch.from_numpy(s.f_ext).cuda()), s.dt,
                            assemble=False)
    small = {"workload": "1000-sphere cluster (section 6.3 recipe), cold solve to its tolerance",
             "n_contacts": con.count}
    for name, fn in (("persistent", sc.solve_lcp_rpy), ("per_phase", sc.solve_lcp_mob)):
        fn(P, con, R, tol=s.tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 20
        for _ in range(reps):
            _, _, st, _, _ = fn(P, con, R, tol=s.tol)
        torch.cuda.synchronize()
        small[name] = {"ms": 1e3 * (time.perf_counter() - t0) / reps, "mvops": st["mvops"],
                       "status": st["status"]}
    out["solve_rpy_small"] = small

    for n, nsteps in ((1000, steps), (20000, max(2, steps // 4))):
        s = W.sphere_cluster(n, W.SEED_BASE + 900 + (n == 20000))
        P = sc.Particles.from_suspension(s)
        box = sc.Box(tuple(s.box), lo=tuple(s.lo), periodic=False)
        stp = ts.TimeStepper(P, box, s.delta, s.dt, torch.from_numpy(s.f_ext).cuda(), tol=s.tol,
                             hydro_radius=torch.from_numpy(s.hydro_radius).cuda())
        stp.step()
        z0 = float(P.pos[:, 2].mean())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = [stp.step() for _ in range(nsteps)]
        torch.cuda.synchronize()
        z1 = float(P.pos[:, 2].mean())
        out[f"cluster{n}_steps"] = {
            "steps": nsteps, "ms_per_step": 1e3 * (time.perf_counter() - t0) / nsteps,
            "iters": [x.stats["iters"] for x in infos],
            "contacts": [x.contacts.count for x in infos],
            "active": [x.stats["n_active"] for x in infos],
            "mean_fall_speed": (z0 - z1) / (nsteps * s.dt),
            "all_converged": all(x.stats["status"] == 0 for x in infos),
            "solver": "persistent" if stp.persistent else "per-phase"}
        if stp.persistent:
            # the same steps with a launch per phase, for comparison
            P2 = sc.Particles.from_suspension(s)
            stp2 = ts.TimeStepper(P2, box, s.delta, s.dt, torch.from_numpy(s.f_ext).cuda(),
                                  tol=s.tol, hydro_radius=torch.from_numpy(s.hydro_radius).cuda(),
                                  persistent=False)
            stp2.step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(nsteps):
                stp2.step()
            torch.cuda.synchronize()
            out[f"cluster{n}_steps"]["ms_per_step_per_phase"] = \
                1e3 * (time.perf_counter() - t0) / nsteps
    return out


def operator_bytes(nc, nnz):
    """Bytes the assembled-M product itself streams per iteration: each
    nonzero's column and value (12), and per row its length (4), q (8) and
    gamma, g read and written (32)."""
    return 12 * nnz + 44 * nc


def kernel_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1909_06623_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(iters, path=TRAFFIC_FILE):
    """HBM bytes per launch from the stored counter summary, or None if the
    kernel sources or the launch (iteration count) changed since."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256") != kernel_digest() or t.get("iters") != iters:
        return None
    return t.get("bytes_per_launch")


def batched(sc, W, torch, np, count):
    """512 independent suspensions (N log-uniform in [200, 20000], spheres or
    rods): contact build with assembly of M, forward solve and adjoint of
    L = 1/2 ||D gamma||^2 each, as one HIP graph replayed (the batch builds
    its contacts on the device), against the same work done one instance at
    a time (build_contacts + solve_lcp + solve_lcp_adjoint) on the same GPU.
    The solve + adjoint part alone (contacts prebuilt) is timed both ways
    too."""
    sus, _ = W.batched_instances(count=count)
    inst = []
    for s in sus:
        P = sc.Particles.from_suspension(s)
        box = sc.Box(tuple(s.box))
        u_nc = sc.apply_mobility(P, torch.from_numpy(s.f_ext).cuda())
        inst.append((s, P, box, u_nc))
    tol, atol = 1e-6, 1e-8
    ws = sc.Workspace()

    def graph_ms(b, reps=3):
        b.graph_solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            b.graph_solve()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    # whole pipeline: build + solve + adjoint in one graph
    t0 = time.perf_counter()
    bb = sc.Batch([(P, box, s.delta, u_nc, s.dt) for s, P, box, u_nc in inst], tol=tol, team=0,
                  adjoint=1, adjoint_tol=atol, build=True)
    tune_s = time.perf_counter() - t0
    full_ms = graph_ms(bb)
    st, adj, info = bb.stats()
    cnt = bb.counts()

    def one(s, P, box, u_nc):
        con = sc.build_contacts(P, box, s.delta, u_nc, s.dt, workspace=ws)
        gam, g, s1, f_c, _ = sc.solve_lcp(P, con, tol=tol, want_fc=True, workspace=ws)
        sc.solve_lcp_adjoint(P, box, con, u_nc, s.dt, gam, dL_df=f_c, tol=atol, workspace=ws)
        return con, s1["iters"]

    for it in inst[:4]:  # warm the single-instance path
        one(*it)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    singles = [one(*it) for it in inst]
    torch.cuda.synchronize()
    single_ms = 1e3 * (time.perf_counter() - t0)

    # solve + adjoint only, contacts prebuilt
    items = [(P, con, box, u_nc, s.dt) for (s, P, box, u_nc), (con, _) in zip(inst, singles)]
    pol = sc.Batch.tuned_policy(info)
    bs = sc.Batch(items, tol=tol, adjoint=1, adjoint_tol=atol, **pol)
    solve_ms = graph_ms(bs)

    def solve_one(P, con, box, u_nc, dt):
        gam, g, s1, f_c, _ = sc.solve_lcp(P, con, tol=tol, want_fc=True, workspace=ws)
        sc.solve_lcp_adjoint(P, box, con, u_nc, dt, gam, dL_df=f_c, tol=atol, workspace=ws)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in items:
        solve_one(*it)
    torch.cuda.synchronize()
    single_solve_ms = 1e3 * (time.perf_counter() - t0)

    # kernel times of the persistent batched kernels: eager solves on the
    # current stream bracketed by HIP events, forward alone (a batch without
    # the adjoint) and forward + adjoint; the difference is the adjoint launch
    bf = sc.Batch([(P, con) for P, con, _, _, _ in items], tol=tol, team=pol["team"],
                  nnz_per_workgroup=pol["nnz_per_workgroup"])

    def event_ms(b, reps=3):
        b.solve()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            b.solve()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    fwd_ms = event_ms(bf)
    fwd_adj_ms = event_ms(bs)
    sf, _, _ = bf.stats()
    sfa, adj2, _ = bs.stats()
    bf.close()
    bs.close()
    bb.close()
    fwd_bytes = adj_bytes = 0
    for s, (P, con, _, _, _), x, a in zip(sus, items, sf, adj2):
        rods = bool(np.all(s.half_len > 0))
        fwd_bytes += (x["iters"] + 2) * iteration_bytes(con.count, s.n, rods)
        adj_bytes += a["iters"] * iteration_bytes(a["n_active"], s.n, rods)
    adj_ms = max(1e-9, fwd_adj_ms - fwd_ms)

    def roof(nbytes, ms, kernel, model):
        gbs = nbytes / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel": kernel,
                "bytes_model": model, "bytes_per_launch": nbytes, "launch_ms": ms}

    kernels = {
        "forward": roof(fwd_bytes, fwd_ms, "k_bbpgd_batch (every instance's Algorithm 1, one "
                        "cooperative launch; eager, HIP events)",
                        "per instance (iterations + 2) x (216 n_c + 120 N) bytes for rods, "
                        "(120 n_c + 56 N) for spheres, summed"),
        "adjoint": roof(adj_bytes, adj_ms, "k_bbpgd_batch adjoint instantiation (every "
                        "instance's masked CG; forward + adjoint time minus forward)",
                        "per instance CG iterations x (216 |A| + 120 N) bytes for rods, "
                        "(120 |A| + 56 N) for spheres, summed"),
        "forward_iters_match": [x["iters"] for x in sf] == [x["iters"] for x in sfa]}
    n_tot = sum(s.n for s in sus)
    return {"instances": count, "particles": n_tot,
            "contacts": sum(c for c, _, _ in cnt),
            "contacts_match_single_builds": [c for c, _, _ in cnt] == [c.count for c, _ in singles],
            "nnz_M": sum(z for _, z, _ in cnt),
            "batch_ms": full_ms, "one_at_a_time_ms": single_ms,
            "speedup": single_ms / full_ms,
            "batch_particles_per_s": n_tot / (full_ms * 1e-3),
            "solve_adjoint_batch_ms": solve_ms,
            "solve_adjoint_one_at_a_time_ms": single_solve_ms,
            "solve_adjoint_speedup": single_solve_ms / solve_ms,
            "policy": pol,
            "team_sizes": {str(t): sum(1 for x in st if x["grid"] == t) for t in (1, 2, 4, 8, 16, 32)},
            "adjoint_team_sizes": {str(t): sum(1 for x in adj if x["grid"] == t)
                                   for t in (1, 2, 4, 8, 16, 32)},
            "tune_policies": [f"classes nnz/workgroup {4096 << i}" for i in range(6)]
            + [f"team {1 << i}" for i in range(6)], "tune_ms": info["tune_ms"],
            "tune_adjoint_ms": info["tune_adjoint_ms"], "tune_s": tune_s,
            "all_converged": all(x["status"] == 0 for x in st),
            "adjoint_all_converged": all(x["status"] == 0 for x in adj),
            "adjoint_cg_iters_sum": sum(x["iters"] for x in adj),
            "iters_max": max(x["iters"] for x in st),
            "iters_sum": sum(x["iters"] for x in st),
            "single_iters_sum": int(sum(i for _, i in singles)),
            "tol": tol, "adjoint_tol": atol,
            "kernels": kernels,
            "work": "contact build with assembly of M + forward BBPGD + adjoint (CG, geometric "
                    "gradient) per instance",
            "launch": "batched build kernels + reset + cooperative persistent forward and "
                      "adjoint kernels, one HIP graph replay"}


def host_cpu():
    """(CPU model, logical CPUs of the host, CPUs this process may run on)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def cpu_baseline(s, W, no_hydro):
    """The oracle (plain FP64 C) on the same workload: cell-list contacts, q
    and Algorithm 1 to 1e-6, once on one core and once on all the cores this
    process may use (OpenMP; the same contact list and products, the sums of
    Algorithm 1 added per thread in thread order). `value` is the all-cores
    leg."""
    import oracle as O
    model, nproc, usable = host_cpu()
    env = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    nt = max(1, min(usable, env) if env else usable)
    legs = {}
    for name, t in (("one_core", 1), ("all_cores", nt)):
        with O.threads(t):
            t1 = time.perf_counter()
            c, u_o, q_o = O.setup(s)
            tc = time.perf_counter() - t1
            t1 = time.perf_counter()
            go, gg, sto = O.bbpgd(s, c, q_o)
            ts = time.perf_counter() - t1
        legs[name] = {"value": s.n / (tc + ts), "unit": "rods/s", "cores": t,
                      "contacts_s": tc, "bbpgd_s": ts, "iters": sto.iters,
                      "solve_only_rods_per_s": s.n / ts}
    a = legs["all_cores"]
    cpu = {"value": a["value"], "unit": "rods/s", "cores": a["cores"], "kind": "oracle",
           "sample": (f"the full 100k-rod workload once per leg: cell-list contacts + q + "
                      f"BBPGD to 1e-6 (serial FP64 C; all cores: OpenMP over particles and "
                      f"contacts): {a['contacts_s']:.1f} s + {a['bbpgd_s']:.1f} s on "
                      f"{a['cores']} threads, {legs['one_core']['contacts_s']:.1f} s + "
                      f"{legs['one_core']['bbpgd_s']:.1f} s on one"),
           "one_core": legs["one_core"], "all_cores": a, "cpu_model": model, "nproc": nproc,
           "usable_cpus": usable}
    if not no_hydro:
        # the oracle's time step behind the RPY mobility (dense NumPy on one
        # thread) on the 1000-sphere cluster, beside the GPU's in `hydro`
        import oracle.timestep as OT
        from threadpoolctl import threadpool_limits
        cl = W.sphere_cluster(1000, W.SEED_BASE + 900)
        with threadpool_limits(1):
            t1 = time.perf_counter()
            OT.step(cl, OT.quat_from_axis(cl.axis), None, hydro="rpy")
            tr = time.perf_counter() - t1
        cpu["rpy_cluster1000_step_ms"] = 1e3 * tr
        cpu["rpy_sample"] = ("one time step of the 1000-sphere cluster with the RPY mobility: "
                             "contacts, dense Mob and M, Algorithm 1, update; one thread")
    return cpu


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=float, default=1.0, help="particle-count scale (tests)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--no-timestep", action="store_true")
    ap.add_argument("--no-hydro", action="store_true",
                    help="skip the RPY-mobility leg")
    ap.add_argument("--hydro-steps", type=int, default=20)
    ap.add_argument("--timestep-steps", type=int, default=8)
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 1.1M-particle forward solve")
    ap.add_argument("--only-large", action="store_true",
                    help="run only the 1.1M-particle forward solve (for profiling)")
    ap.add_argument("--large-steps", type=int, default=3)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (to scale HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1909_06623_amd as sc
    import workloads as W

    torch.cuda.set_device(0)
    if args.only_large:
        big = large(sc, W, torch, np, args.large_steps)
        torch.cuda.synchronize()
        sc.release()
        print(json.dumps({"large": big}), flush=True)
        return
    if args.calibrate_copy:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8,
                          "launches": 5}), flush=True)
        return
    s = W.workload(2, scale=args.scale)
    print(f"[bench] workload {s.name}: N={s.n}, box {s.box[0]:.4f}", file=sys.stderr, flush=True)
    P = sc.Particles.from_suspension(s)
    box = sc.Box(tuple(s.box))
    f_ext = torch.from_numpy(s.f_ext).cuda()
    u_nc = sc.apply_mobility(P, f_ext)
    ws = sc.Workspace()
    cap = None

    def step():
        con = sc.build_contacts(P, box, s.delta, u_nc, s.dt, capacity=cap, workspace=ws)
        out = sc.solve_lcp(P, con, tol=s.tol, workspace=ws)
        return con, out

    con, out = step()
    cap = con.capacity
    for _ in range(max(0, args.warmup - 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        con, out = step()
        stats.append(out[2])
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    ms_step = 1e3 * t_total / args.steps

    # phase split: contacts alone and solve alone
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        sc.build_contacts(P, box, s.delta, u_nc, s.dt, capacity=cap, workspace=ws)
    torch.cuda.synchronize()
    build_ms = 1e3 * (time.perf_counter() - t1) / args.steps
    t1 = time.perf_counter()
    for _ in range(args.steps):
        g_out = sc.solve_lcp(P, con, tol=s.tol, workspace=ws)
    torch.cuda.synchronize()
    solve_ms = 1e3 * (time.perf_counter() - t1) / args.steps
    # the matrix-free two-pass product on the same contacts, for comparison
    chain = sc.solve_lcp(P, con, tol=s.tol, workspace=ws, op=1)[2]

    st = stats[-1]
    iters = st["iters"]
    used_matrix = st["op"] == 2
    rods = bool(np.all(s.half_len > 0))
    bytes_iter = iteration_bytes(con.count, s.n, rods)
    products = iters + 2  # Algorithm 1: g_0, g_0^T M g_0, then one per step
    bytes_launch = bytes_iter * products
    # mean HIP-event time of the persistent kernel over the timed steps
    kernel_ms = float(np.mean([x["kernel_ms"] for x in stats]))
    achieved = bytes_launch / (kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic(iters) if used_matrix else None

    adj = None
    if not args.no_adjoint:
        gam, g, st2, f_c, u_c = sc.solve_lcp(P, con, tol=s.tol, want_fc=True, workspace=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dq, dpos, sta = sc.solve_lcp_adjoint(P, box, con, u_nc, s.dt, gam, dL_df=f_c,
                                             tol=1e-8, workspace=ws)
        torch.cuda.synchronize()
        adj_ms = 1e3 * (time.perf_counter() - t1)
        cg_bytes = sta["iters"] * iteration_bytes(sta["n_active"], s.n, rods)
        cg_gbs = cg_bytes / (sta["kernel_ms"] * 1e-3) / 1e9
        adj = {"adjoint_ms": adj_ms, "forward_solve_ms": solve_ms,
               "ratio": adj_ms / solve_ms, "cg_iters": sta["iters"],
               "cg_rel_residual": sta["residual"], "n_active": sta["n_active"],
               "cg_kernel_ms": sta["kernel_ms"],
               "roofline": {"bound": "hbm", "achieved": cg_gbs, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": cg_gbs / HBM_PEAK_GBS, "traffic": None,
                            "kernel": "k_cg_mat (persistent masked CG on M_AA, one launch)",
                            "bytes_model": "216 |A| + 120 N bytes per CG iteration (one "
                                           "masked product on the active set)",
                            "bytes_per_launch": cg_bytes, "launch_ms": sta["kernel_ms"],
                            "us_per_iteration": 1e3 * sta["kernel_ms"] / max(1, sta["iters"])}}
        # the active-set polish of the same solve (exact on its active set)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        gpol, gpg, stp, _, _ = sc.polish_lcp(P, con, gam, tol=1e-13, workspace=ws)
        torch.cuda.synchronize()
        adj["polish"] = {"ms": 1e3 * (time.perf_counter() - t2), "status": stp["status"],
                         "passes": stp["mvops"], "cg_iters": stp["iters"],
                         "cg_kernel_ms": stp["kernel_ms"], "residual_before": st2["residual"],
                         "residual_after": stp["residual"],
                         "rel_gamma_change": float(torch.linalg.norm(gpol - gam)
                                                   / torch.linalg.norm(gpol))}

    batch = None if args.no_batch else batched(sc, W, torch, np, args.batch_count)
    big = None if args.no_large else large(sc, W, torch, np, args.large_steps)
    sph = spheres1000(sc, W, torch, np, 20)
    tsl = None if args.no_timestep else timestepping(sc, W, torch, np, args.timestep_steps)
    hyd = None if args.no_hydro else hydro(sc, W, torch, np, args.hydro_steps)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(s, W, args.no_hydro)
    line = {
        "metric": "BBPGD solve time to res 1e-6 (rods/s), HBM GB/s; adjoint/forward time ratio",
        "value": s.n / (ms_step * 1e-3),
        "unit": "rods/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "100000 spherocylinders L=1 D=0.05, isotropic, ~6 close "
                               "pairs per rod, periodic box, delta 0.015, dt 1e-4, "
                               "BBPGD (BB1) to ||min(gamma,g)||_2 < 1e-6",
                   "n": s.n, "n_contacts": con.count, "iters": iters,
                   "mvops": st["mvops"], "n_active": st["n_active"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_frac": achieved / HBM_PEAK_GBS,
                     "hbm_frac": (None if traffic is None
                                  else traffic / (kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS),
                     "note": ("frac and achieved count the method's algorithmic bytes; the "
                              "77 MB per product stays in LDS (most of M) and the 256 MB "
                              "Infinity Cache, so hbm_frac (measured HBM bytes, traffic) is "
                              "far lower and the kernel is bound by its per-iteration "
                              "latency; the 1.1M-particle leg (large.roofline) is the one "
                              "that streams from HBM"),
                     "kernel": ("k_bbpgd_mat" if used_matrix else "k_bbpgd")
                               + " (persistent BBPGD solve, one launch per solve)",
                     "bytes_model": ("216 n_c + 120 N" if rods else "120 n_c + 56 N")
                                    + " bytes per product, (iterations + 2) products "
                                      "per launch",
                     "bytes_per_product": bytes_iter, "products_per_launch": products,
                     "bytes_per_launch": bytes_launch, "launch_ms": kernel_ms,
                     "us_per_product": 1e3 * kernel_ms / products,
                     "operator_bytes_per_product": (operator_bytes(con.count, con.nnz)
                                                    if used_matrix else None),
                     "grid": st["grid"], "block": st["block"],
                     "slices_per_wave": st["slices_per_wave"],
                     "lds_entries_per_wave": st["lds_entries_per_wave"],
                     "lanes_per_particle": st["lanes_per_particle"]},
        "cpu_baseline": cpu,
        "chain_solve": {"iters": chain["iters"], "kernel_ms": chain["kernel_ms"],
                        "us_per_iter": 1e3 * chain["kernel_ms"] / (chain["iters"] + 2),
                        "roofline": chain_roofline(chain, bytes_iter)},
        "operator": "assembled M" if st["op"] == 2 else "matrix-free chain",
        "nnz_M": con.nnz,
        "build_ms": build_ms,
        "solve_ms": solve_ms,
        "solve_only_rods_per_s": s.n / (solve_ms * 1e-3),
        "adjoint": adj,
        "adjoint_forward_ratio": None if adj is None else adj["ratio"],
        "batched": batch,
        "large": big,
        "spheres1000": sph,
        "timestep": tsl,
        "hydro": hyd,
    }
    # everything the library keeps between calls is released before exit
    torch.cuda.synchronize()
    sc.release()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
