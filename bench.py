"""Benchmark: Schur matvecs/s and time-to-1e-10 residual, FP64 vs FP32-refined,
on one MI355X.

Default workload (c2): the long-domain 2-D Poisson-Neumann problem on
[0, 64] x [0, 1], 128 x 8 elements, polynomial order 16 (17 x 17 GLL points),
manufactured solution plus seeded zero-mean Gaussian forcing.  One step is one
full solve (Algorithm 2: right-hand side and null-space projection,
element-interior elimination, Schur right-hand side, DBJ-GMRES to 1e-10,
solution assembly and recovery) with the inputs resident in HBM.

Other workloads (--config c3 | c4 | c5) time the same path on the stretched
256 x 16 grid with distinct strips, the 65 Fourier modes x (Re, Im) of the
64 x 8 grid, and the uneven 32-problem batch.

Prints one JSON line.  --matvec-only runs just the Schur matvec kernel (used
for the hardware-counter passes).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np

WORKLOADS = {
    "c2": "2-D Poisson-Neumann [0,64]x[0,1], 128x8 elements, order 16, manufactured + seeded Gaussian "
          "forcing, DBJ-GMRES to 1e-10",
    "c3": "2-D stretched grid 256x16 elements, order 12, geometric z-stretch, seeded distinct strip widths, "
          "f ~ U[0,1], DBJ-GMRES to 1e-10",
    "c4": "3-D via Fourier in y: 64x8 elements, order 12, 128 y-points -> 65 Helmholtz modes x (Re, Im) = "
          "130 batched Schur solves, DBJ-GMRES to 1e-10",
    "c5": "uneven batch of 32 seeded 2-D Poisson/Helmholtz problems, 16x2..256x16 elements, orders 8-16, "
          "DBJ-GMRES to 1e-10",
}


def gpu_events_time(fn, reps, stream):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(reps):
        fn()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / reps   # ms


def make_solver(cfg, precision, inner_tol=0.0, zlabel=0, setup="auto"):
    import paper_1512_01756_amd as P
    from paper_1512_01756_amd import workloads
    kw = {"precision": precision, "inner_tol": inner_tol, "zlabel": zlabel, "setup": setup}
    if cfg in ("c2", "c3"):
        p = workloads.c2() if cfg == "c2" else workloads.c3()
        return P.Solver(p.xb, p.zb, p.n - 1, **kw), p.f.reshape(-1)
    if cfg == "c4":
        p = workloads.c4()
        return P.Solver(p.xb, p.zb, p.n - 1, kwaves=p.kwaves, nrhs=2, **kw), p.f.reshape(-1)
    probs = workloads.c5()
    grids = [(p.xb, p.zb, p.n - 1, float(p.kwaves[0])) for p in probs]
    return P.Solver(grids=grids, **kw), np.concatenate([p.f.reshape(-1) for p in probs])


def matvec_bytes(solver, s_op, s_vec):
    """Algorithmic bytes of one batched Schur matvec: every distinct N x 2N
    half block once, the input and output interface vectors of every
    instance."""
    tot = 0
    for info in solver.info:
        N = info["n"] * info["mz"]
        tot += info["unique_W"] * N * 2 * N * s_op
        tot += 2 * info["kS"] * s_vec * info["nrhs"]
    return tot


def matvec_flops(solver):
    """Algorithmic flops of one batched Schur matvec: y_h = x_h + W_h x_win
    for every half of every instance (2 N x 2N per half, plus the identity)."""
    tot = 0
    for info in solver.info:
        N = info["n"] * info["mz"]
        nh = 2 * (info["mx"] - 1)
        tot += (2 * nh * N * 2 * N + info["kS"]) * info["nrhs"]
    return tot


GEMM_KERNELS = {0: "k_half_gemm<double, 16> (split-K, 16 waves)", 1: "k_half_gemm<double, 8> (split-K, 8 waves)",
                2: "k_half_gemm_t<double> (LDS-staged, XCD-ordered)", 3: "k_half_gemm_t<double> (LDS-staged)",
                4: "k_half_gemm_t<double> (LDS-staged, XCD-ordered, 64-value chunks)",
                5: "k_half_gemm_t<double> (LDS-staged, 64-value chunks)"}


def matvec_kernel_name(solver):
    """The kernel the FP64 matvec runs: the MFMA GEMM schedule the setup timed
    fastest where strips share blocks, the streaming GEMV where they do not."""
    names = set()
    for info in solver.info:
        if info["unique_W"] < 2 * (info["mx"] - 1):
            names.add(GEMM_KERNELS.get(info["gemm_sched"][0], "k_half_gemm<double>"))
        else:
            names.add("k_half_gemv_stream<double> (distinct blocks)")
    return " + ".join(sorted(names))


# HBM-side bytes per launch of the FP64 batched Schur matvec, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) over `bench.py --matvec-only`,
# each scaled by the counter's reading for a 256 MiB device copy (fetch x2.000,
# write x1.000); see profiles/c2_schur_matvec_hbm_counters.txt.  Valid only for
# the kernel version the passes measured (c2: the split-K k_half_gemm<double>
# with paired K-steps, 16 waves; c3: the streaming
# k_half_gemv_stream<double>, profiles/c3_schur_matvec_hbm_counters.txt); a run
# whose tuner picked another kernel reports no traffic.
MATVEC_TRAFFIC = {"c2": (GEMM_KERNELS[0], 6.482e6), "c3": ("k_half_gemv_stream<double> (distinct blocks)", 3.568e8)}

PEAK_HBM_GBPS = 8000.0
PEAK_FP64_MFMA_TFLOPS = 78.6


def cpu_baseline(budget_s=25.0):
    """The oracle as it stands, timed on the host: setup once (reported, not
    part of the sample), then DBJ solves of the same c2 problem until ~budget_s
    of solve time."""
    from oracle import schur, smpm, solve
    from paper_1512_01756_amd import workloads
    prob = workloads.c2()
    grid = smpm.Grid(prob.xb, prob.zb, prob.n)
    t0 = time.perf_counter()
    o = schur.build(grid)
    setup_s = time.perf_counter() - t0
    F = smpm.rhs(grid, o.tau, prob.f[0, 0])
    times, mv = [], []
    while sum(times) < budget_s and len(times) < 10:
        t0 = time.perf_counter()
        r = solve.dbj_solve(o, F)
        times.append(time.perf_counter() - t0)
        mv.append(r.iters + 2)     # one S per iteration, one in Q, one residual check
    solve_s = float(np.median(times))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": float(np.mean(mv) / solve_s), "unit": "matvecs/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(times)} full DBJ solves of the c2 workload after a {setup_s:.1f} s oracle setup "
                      f"(setup not in the sample); median solve {solve_s * 1e3:.1f} ms, {r.iters} GMRES iterations",
            "time_to_1e-10_ms": solve_s * 1e3, "setup_s": setup_s}, r.u


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--matvec-reps", type=int, default=200)
    ap.add_argument("--matvec-only", action="store_true")
    ap.add_argument("--zlabel", type=int, default=0, choices=(0, 1),
                    help="deflation space: 0 one column per interface (the paper's), 1 per element segment")
    ap.add_argument("--setup", default="auto", choices=("auto", "host", "device"),
                    help="where the large dense setup steps run (setup is not timed)")
    ap.add_argument("--inner-tol", type=float, default=0.0,
                    help="FP32-IR inner tolerance floor (0: the library default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the 2-D path would shard its strips across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1512_01756_amd as P

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)

    if args.matvec_only:
        # The Schur matvec alone, plus a plain device copy of known size that
        # calibrates the HBM byte counters (FETCH_SIZE / WRITE_SIZE).
        s, _ = make_solver(args.config, P.FP64, setup=args.setup)
        x = torch.randn(s.total_kS, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        ms = gpu_events_time(lambda: s.schur_apply_all(x, y, P.FP64), args.matvec_reps, stream)
        cbytes = 256 << 20
        a = torch.ones(cbytes // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        cms = gpu_events_time(lambda: b.copy_(a), 5, stream)
        print(json.dumps({"config": args.config, "matvec_fp64_us": ms * 1e3,
                          "algorithmic_bytes": matvec_bytes(s, 8, 8),
                          "copy_bytes_each_way": cbytes, "copy_us": cms * 1e3}), flush=True)
        s.close()
        return

    forms = {}
    fvec = None
    for name, prec in (("fp64", P.FP64), ("fp32_ir", P.FP32_IR), ("fp16s_ir", P.FP16S_IR)):
        t0 = time.perf_counter()
        s, fh = make_solver(args.config, prec, args.inner_tol, args.zlabel, args.setup)
        setup_s = time.perf_counter() - t0
        if fvec is None:
            fvec = torch.as_tensor(fh).to(dev)
            u = torch.empty_like(fvec)
        for _ in range(args.warmup):
            s.solve(fvec, None, u, check=False)
        torch.cuda.synchronize()
        stats_list = []
        status_list = []

        def step():
            _, st, status = s.solve(fvec, None, u, check=(prec != P.FP16S_IR))
            stats_list.append(st)
            status_list.append(status)

        ms = gpu_events_time(step, args.steps, stream)
        forms[name] = {"solver": s, "ms": ms, "stats": stats_list[-1], "setup_s": setup_s,
                       "status": "ok" if status_list[-1] == 0 else f"status {status_list[-1]}",
                       "u": u.cpu().numpy().copy()}

    # c4 also end to end from the physical 3-D field: transform in y, the
    # batched mode solves, inverse transform (Sec. 5).
    physical = None
    if args.config == "c4":
        from paper_1512_01756_amd import workloads
        p4 = workloads.c4()
        my, ly = 128, 8.0
        fphys = torch.as_tensor(workloads.fourier_field(0, p4.r, my)).to(dev)
        uphys = torch.empty_like(fphys)
        physical = {}
        for name, prec, one in (("fp64", P.FP64, False), ("fp32_ir", P.FP32_IR, False),
                                ("fp64_one_krylov", P.FP64, True)):
            sf = P.Solver(p4.xb, p4.zb, p4.n - 1, fourier=(my, ly), precision=prec, inner_tol=args.inner_tol,
                          one_krylov=one)
            for _ in range(args.warmup):
                sf.solve_fourier(fphys, None, uphys)
            physical[name] = gpu_events_time(lambda: sf.solve_fourier(fphys, None, uphys), args.steps, stream)
            if one:
                _, st1, _ = sf.solve_fourier(fphys, None, uphys)
                physical["one_krylov_iterations"] = st1["iters_max"]
                physical["one_krylov_rel_residual_max"] = st1["rel_residual_max"]
            sf.close()

    # The Schur matvec kernel alone (batched half-interface GEMV), both precisions.
    s64 = forms["fp64"]["solver"]
    x = torch.randn(s64.total_kS, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    x32, y32 = x.float(), y.float()
    for _ in range(10):
        s64.schur_apply_all(x, y)
    mv64_ms = gpu_events_time(lambda: s64.schur_apply_all(x, y, P.FP64), args.matvec_reps, stream)
    mv32_ms = gpu_events_time(lambda: s64.schur_apply_all(x32, y32, P.FP32_IR), args.matvec_reps, stream)
    bytes64 = matvec_bytes(s64, 8, 8)
    bytes32 = matvec_bytes(s64, 4, 4)
    gbs64 = bytes64 / (mv64_ms * 1e-3) / 1e9
    gbs32 = bytes32 / (mv32_ms * 1e-3) / 1e9

    # Roofline of the dominant kernel (the FP64 batched Schur matvec): the
    # binding roof is the one with the longer ideal time for this launch.
    flops64 = matvec_flops(s64)
    t_hbm = bytes64 / (PEAK_HBM_GBPS * 1e9)
    t_mfma = flops64 / (PEAK_FP64_MFMA_TFLOPS * 1e12)
    tflops64 = flops64 / (mv64_ms * 1e-3) / 1e12
    if t_mfma > t_hbm:
        roofline = {"bound": "mfma", "achieved": tflops64, "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                    "frac": tflops64 / PEAK_FP64_MFMA_TFLOPS}
    else:
        roofline = {"bound": "hbm", "achieved": gbs64, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                    "frac": gbs64 / PEAK_HBM_GBPS}
    kname = matvec_kernel_name(s64)
    measured = MATVEC_TRAFFIC.get(args.config)
    roofline.update({"traffic": measured[1] if measured and measured[0] == kname else None, "kernel": kname,
                     "launch_us": mv64_ms * 1e3, "algorithmic_bytes_per_launch": bytes64,
                     "algorithmic_flops_per_launch": flops64, "achieved_GBps": gbs64,
                     "achieved_TFLOPs": tflops64})

    fp64, ir, ir16 = forms["fp64"], forms["fp32_ir"], forms["fp16s_ir"]
    s16 = ir16["solver"]
    mv16_ms = gpu_events_time(lambda: s16.schur_apply_all(x32, y32, P.FP16S_IR), args.matvec_reps, stream)
    bytes16 = matvec_bytes(s64, 2, 4)
    value = fp64["stats"]["schur_matvecs"] / (fp64["ms"] * 1e-3)
    i0 = s64.info[0]
    line = {
        "metric": "Schur matvecs/s + time-to-1e-10 residual, FP64 vs FP32-refined, 1 GPU",
        "value": value,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp64["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "systems": s64.nsys,
                   "deflation": "per element segment" if args.zlabel else "per interface",
                   "instances": fp64["stats"]["instances"], "k_S_total": s64.total_kS, "r_total": s64.total_r,
                   "first_system": {"mx": i0["mx"], "mz": i0["mz"], "n": i0["n"], "d": i0["d"]}},
        "value_definition": "Schur matvecs performed by one full FP64 DBJ solve divided by its wall time",
        "time_to_1e-10_ms": {"fp64": fp64["ms"], "fp32_ir": ir["ms"], "fp16s_ir": ir16["ms"]},
        "time_to_1e-10_ms_from_physical_field": physical,
        "iterations": {"fp64_max": fp64["stats"]["iters_max"], "fp64_total": fp64["stats"]["iters_total"],
                       "fp32_ir_inner_max": ir["stats"]["iters_max"], "fp32_ir_inner_total": ir["stats"]["iters_total"],
                       "fp32_ir_sweeps": ir["stats"]["sweeps_max"],
                       "fp16s_ir_inner_max": ir16["stats"]["iters_max"], "fp16s_ir_inner_total": ir16["stats"]["iters_total"],
                       "fp16s_ir_sweeps": ir16["stats"]["sweeps_max"], "fp16s_ir_status": ir16["status"]},
        "rel_residual_max": {"fp64": fp64["stats"]["rel_residual_max"], "fp32_ir": ir["stats"]["rel_residual_max"],
                             "fp16s_ir": ir16["stats"]["rel_residual_max"]},
        "setup_s": {"fp64": fp64["setup_s"], "fp32_ir": ir["setup_s"], "fp16s_ir": ir16["setup_s"]},
        "gemm_schedules": {"matvec_S64_S32_M64_M32": i0["gemm_sched"], "element": i0["elem_sched"],
                           "fused_S_Minv_fp64_fp32": [fp64["solver"].info[0]["fused_op"][0],
                                                      ir["solver"].info[0]["fused_op"][1]],
                           "legend": "0 split-K 16 waves, 1 split-K 8 waves, 2 LDS-staged XCD-ordered, "
                                     "3 LDS-staged plain; matvec lists: 4 / 5 = 2 / 3 with 64-value chunks; "
                                     "element lists: 4 / 5 LDS-staged 32- / 16-row tiles with K split over "
                                     "the waves; -1 unused; picked by timing at setup"},
        "matvec_kernel": {"fp64_us": mv64_ms * 1e3, "fp32_us": mv32_ms * 1e3,
                          "fp64_matvecs_per_s": 1e3 / mv64_ms, "fp32_matvecs_per_s": 1e3 / mv32_ms,
                          "fp64_GBps": gbs64, "fp32_GBps": gbs32, "fp16s_us": mv16_ms * 1e3,
                          "fp16s_GBps": bytes16 / (mv16_ms * 1e-3) / 1e9},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline and args.config == "c2":
        line["cpu_baseline"], u_oracle = cpu_baseline()
        # the same right-hand side on both sides: each form's solution against
        # the oracle's (max abs difference over max |u|, after both gauges)
        scale = float(np.abs(u_oracle).max())
        line["error_vs_oracle"] = {k: float(np.abs(v["u"] - u_oracle).max() / scale) for k, v in forms.items()}
    for v in forms.values():
        v["solver"].close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
