"""Benchmark: contact detection + BBPGD solve to ||min(gamma, g)|| < 1e-6 on
100,000 spherocylinders (length 1, diameter 0.05, ~6 close pairs per rod,
isotropic, periodic box), FP64, one MI355X.

One step = build_contacts + solve_lcp on the resident synthetic inputs.
Prints one JSON line: whole-job throughput in rods/s, the HBM roofline of the
BBPGD iteration (algorithmic bytes per iteration over the measured GPU time of
the iteration loop), the adjoint/forward time ratio (loss 1/2 ||D gamma||^2),
and the FP64 oracle timed on the host for comparison.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def rod_iteration_bytes(nc, n):
    """Algorithmic bytes of one matrix-free BBPGD iteration on a rod system:
    per contact the 80-byte frame record read in both passes, 8 bytes of
    incidence and 48 bytes of gamma/g/q traffic; per particle U written and
    read (96) and the axis (24)."""
    return 216 * nc + 120 * n


def matrix_iteration_bytes(nc, nnz):
    """Algorithmic bytes of one BBPGD iteration on the assembled M: each
    nonzero's column index and value (12), and per row its offset (4), q (8)
    and gamma, g read and written (32). Column gathers of gamma and g are
    reuse of rows already counted."""
    return 12 * nnz + 44 * nc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=float, default=1.0, help="particle-count scale (tests)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
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
    bytes_iter = (matrix_iteration_bytes(con.count, con.nnz) if used_matrix
                  else rod_iteration_bytes(con.count, s.n))
    kernel_ms = float(np.median([x["kernel_ms"] for x in stats]))
    per_iter_s = kernel_ms * 1e-3 / max(1, iters + 2)
    achieved = bytes_iter / per_iter_s / 1e9

    adj = None
    if not args.no_adjoint:
        gam, g, st2, f_c, u_c = sc.solve_lcp(P, con, tol=s.tol, want_fc=True, workspace=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dq, dpos, sta = sc.solve_lcp_adjoint(P, box, con, u_nc, s.dt, gam, dL_df=f_c,
                                             tol=1e-8, workspace=ws)
        torch.cuda.synchronize()
        adj_ms = 1e3 * (time.perf_counter() - t1)
        adj = {"adjoint_ms": adj_ms, "forward_solve_ms": solve_ms,
               "ratio": adj_ms / solve_ms, "cg_iters": sta["iters"],
               "cg_rel_residual": sta["residual"], "n_active": sta["n_active"]}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        t1 = time.perf_counter()
        c, u_o, q_o = O.setup(s)
        tc = time.perf_counter() - t1
        t1 = time.perf_counter()
        go, gg, sto = O.bbpgd(s, c, q_o)
        ts = time.perf_counter() - t1
        cpu = {"value": s.n / (tc + ts), "unit": "rods/s", "cores": 1, "kind": "oracle",
               "sample": f"the full workload once: cell-list contacts {tc:.1f} s + "
                         f"BBPGD {ts:.1f} s ({sto.iters} iterations), serial FP64 C",
               "solve_only_rods_per_s": s.n / ts, "iters": sto.iters}

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
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": ("k_bbpgd_mat" if used_matrix else "k_bbpgd")
                               + " (persistent BBPGD solve; per launch = iterations + 2 "
                               "products)",
                     "bytes_model": ("12 nnz + 44 n_c" if used_matrix
                                     else "216 n_c + 120 N"),
                     "bytes_per_iter": bytes_iter, "us_per_iter": per_iter_s * 1e6,
                     "kernel_ms": kernel_ms, "grid": st["grid"], "block": st["block"],
                     "lanes_per_particle": st["lanes_per_particle"]},
        "cpu_baseline": cpu,
        "chain_solve": {"iters": chain["iters"], "kernel_ms": chain["kernel_ms"],
                        "us_per_iter": 1e3 * chain["kernel_ms"] / (chain["iters"] + 2)},
        "operator": "assembled M" if st["op"] == 2 else "matrix-free chain",
        "nnz_M": con.nnz,
        "build_ms": build_ms,
        "solve_ms": solve_ms,
        "solve_only_rods_per_s": s.n / (solve_ms * 1e-3),
        "adjoint": adj,
        "adjoint_forward_ratio": None if adj is None else adj["ratio"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
