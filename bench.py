"""Benchmark: Schur matvecs/s and time-to-1e-10 residual, FP64 vs FP32-refined,
on one MI355X.

Headline workload (c2): the long-domain 2-D Poisson-Neumann problem on
[0, 64] x [0, 1], 128 x 8 elements, polynomial order 16 (17 x 17 GLL points),
manufactured solution plus seeded zero-mean Gaussian forcing.  One step is one
full solve (Algorithm 2: right-hand side and null-space projection,
element-interior elimination, Schur right-hand side, DBJ-GMRES to a 1e-10
relative Schur residual, solution assembly and recovery) with the inputs
resident in HBM.  Step i solves the forcing of seed i mod 10, so consecutive
solves never repeat a right-hand side; the time to 1e-10 is the median over
the timed solves, each bracketed by HIP events on the solve's stream, and the
headline value is the Schur matvecs of all timed solves over their total
time.

The same line carries the other workloads, each in FP64 and with the FP32
inner solve inside FP64 refinement, over three right-hand-side seeds: the
stretched 256 x 16 grid with distinct strips (c3), the 65 Fourier modes x
(Re, Im) of the 64 x 8 grid (c4) and the uneven 32-problem batch (c5); and
the four methods of the paper's Table 2 over m_x = 64 .. 1024 (iterations and
solve times of Schur, BJ, DBJ and 2LAS GMRES on m_x x 10 grids of order 9).

Rooflines: each kernel the FP64 solve runs per iteration (the S M^-1 GEMM or
its two parts), the standalone Schur matvec and the element-interior
elimination, timed alone with HIP events on the stream they run on, against
the algorithmic flops and bytes of the method (nonzero operator entries,
distinct blocks once, vectors in and out).

Prints one JSON line.  --kernel-only runs one kernel alone (for the
hardware-counter passes), --solve-only the FP64 solves alone (for a
solve-only kernel trace).
"""
import argparse
import json
import os
import subprocess
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

PEAK_HBM_GBPS = 8000.0
PEAK_MFMA_TFLOPS = {"fp64": 78.6, "fp32": 157.3}
# MI355X's last-level (Infinity) cache: working sets below it can be served
# faster than HBM, so HBM claims use operators above it.
MALL_BYTES = 256 << 20


# ---------------------------------------------------------------------------
# Inputs

def workload_rhs(cfg, seed):
    """Right-hand side of `seed` on the workload's fixed (seed 0) grid."""
    from paper_1512_01756_amd import workloads
    if cfg == "c2":
        return workloads.c2(seed=seed).f.reshape(-1)
    if cfg == "c3":
        return workloads.c3(seed=0, rhs_seed=seed).f.reshape(-1)
    if cfg == "c4":
        return workloads.c4(seed=seed).f.reshape(-1)
    return np.concatenate([p.f.reshape(-1) for p in workloads.c5(seed=0, rhs_seed=seed)])


def make_solver(cfg, precision, inner_tol=0.0, zlabel=0, setup="auto", tol=1e-10):
    import paper_1512_01756_amd as P
    from paper_1512_01756_amd import workloads
    kw = {"precision": precision, "inner_tol": inner_tol, "zlabel": zlabel, "setup": setup, "tol": tol}
    if cfg in ("c2", "c3"):
        p = workloads.c2() if cfg == "c2" else workloads.c3()
        return P.Solver(p.xb, p.zb, p.n - 1, **kw)
    if cfg == "c4":
        p = workloads.c4()
        return P.Solver(p.xb, p.zb, p.n - 1, kwaves=p.kwaves, nrhs=2, **kw)
    grids = [(p.xb, p.zb, p.n - 1, float(p.kwaves[0])) for p in workloads.c5()]
    return P.Solver(grids=grids, **kw)


# ---------------------------------------------------------------------------
# Timing

def time_solves(s, fs, u, steps, warmup, stream):
    """Solve fs[i mod len(fs)] for i < steps after `warmup` untimed solves;
    HIP events on `stream` around each solve.  Returns per-solve ms, the
    total ms from the first start to the last end, the stats and statuses."""
    import torch
    for i in range(warmup):
        s.solve(fs[(steps + i) % len(fs)], None, u, check=False)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    stats, statuses = [], []
    for i in range(steps):
        ev[i][0].record(stream)
        _, st, status = s.solve(fs[i % len(fs)], None, u, check=False)
        ev[i][1].record(stream)
        stats.append(st)
        statuses.append(status)
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in ev]
    return per, ev[0][0].elapsed_time(ev[-1][1]), stats, statuses


def kernel_ms(fn, reps, stream):
    """Average ms per call of fn (one kernel launch, or a fixed sequence)
    over `reps` back-to-back calls, HIP events on `stream`."""
    import torch
    for _ in range(5):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / reps


def form_summary(per, total, stats, statuses):
    ok = all(st == 0 for st in statuses)
    mv = sum(st["schur_matvecs"] for st in stats)
    return {"time_to_1e-10_ms": float(np.median(per)) if ok else None,
            "mean_ms": total / len(per), "status": "ok" if ok else f"status {sorted(set(statuses))}",
            "matvecs_per_s": mv / (total * 1e-3) if ok else None,
            "iters_max": max(st["iters_max"] for st in stats),
            "iters_total": stats[0]["iters_total"], "sweeps": max(st["sweeps_max"] for st in stats),
            "rel_residual_max": max(st["rel_residual_max"] for st in stats)}


# ---------------------------------------------------------------------------
# Algorithmic work per launch (nonzero operator entries, distinct blocks once,
# vectors in and out), summed over the systems of a handle

def alg_schur(s, sv):
    fl = sum((2 * i["nnz_W_total"] + i["kS"]) * i["nrhs"] for i in s.info)
    by = sum(sv[0] * i["nnz_W_unique"] + 2 * sv[1] * i["kS"] * i["nrhs"] for i in s.info)
    return fl, by


def alg_bjinv(s, sv):
    fl = sum(2 * i["nnz_M_total"] * i["nrhs"] for i in s.info)
    by = sum(sv[0] * i["nnz_M_unique"] + 2 * sv[1] * i["kS"] * i["nrhs"] for i in s.info)
    return fl, by


def alg_schur_bjinv(s, sv):
    """S M^-1 as the method needs it: both operators once, the vector in and
    out (the fused GEMM reads the stored product blocks instead)."""
    fl = sum((2 * (i["nnz_W_total"] + i["nnz_M_total"]) + i["kS"]) * i["nrhs"] for i in s.info)
    by = sum(sv[0] * (i["nnz_W_unique"] + i["nnz_M_unique"]) + 2 * sv[1] * i["kS"] * i["nrhs"] for i in s.info)
    return fl, by


def alg_ainv(s):
    """A(k)^-1 in the element-parallel (Woodbury in z) form: the element
    inverse on every element column, the z-interface functionals, the
    capacitance inverse per strip and the element corrections; FP64."""
    fl = by = 0
    for i in s.info:
        n, mx, mz, r = i["n"], i["mx"], i["mz"], i["r"]
        n2, nq = n * n, 2 * n * (mz - 1)
        per = 2 * r * n2 + mx * (2 * nq * n + 2 * nq * nq) + (2 * mx * (mz - 1) * 2) * n2 * n
        fl += per * i["nrhs"]
        by += 8 * (i["elem_unique"] * n2 * n2 + i["strip_classes"] * nq * nq) + 2 * 8 * r * i["nrhs"]
    return fl, by


def roofline(name, ms, flops, nbytes, dtype):
    """Rate of one kernel launch against the roof that binds it (the longer
    of the ideal MFMA and HBM times)."""
    t_mfma = flops / (PEAK_MFMA_TFLOPS[dtype] * 1e12)
    t_hbm = nbytes / (PEAK_HBM_GBPS * 1e9)
    tfl = flops / (ms * 1e-3) / 1e12
    gbs = nbytes / (ms * 1e-3) / 1e9
    if t_mfma >= t_hbm:
        out = {"bound": "mfma", "achieved": tfl, "peak": PEAK_MFMA_TFLOPS[dtype], "unit": "TFLOP/s",
               "frac": tfl / PEAK_MFMA_TFLOPS[dtype]}
    else:
        out = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBPS}
    out.update({"traffic": None, "kernel": name, "launch_us": ms * 1e3, "algorithmic_flops_per_launch": flops,
                "algorithmic_bytes_per_launch": nbytes, "achieved_TFLOPs": tfl, "achieved_GBps": gbs})
    return out


def gemm_kernel_name(s, op, dtype):
    """The kernel a shared-block list runs under the schedule picked at setup
    (op 0 S, 1 M^-1, 2 the stored S M^-1 blocks), or the streaming GEMV where
    every half has its own block."""
    names = {0: "k_half_gemm<{t}, 16> (split-K, 16 waves)", 1: "k_half_gemm<{t}, 8> (split-K, 8 waves)",
             2: "k_half_gemm_t<{t}> (LDS-staged, XCD-ordered)", 3: "k_half_gemm_t<{t}> (LDS-staged)",
             4: "k_half_gemm_t<{t}> (LDS-staged, XCD-ordered, 64-value chunks)",
             5: "k_half_gemm_t<{t}> (LDS-staged, 64-value chunks)",
             6: "k_half_gemm<{t}, 8, 24> (split-K, 8 waves, 24 K-steps in flight)",
             7: "k_half_gemm<{t}, 16, 18> (split-K, 16 waves, 18 K-steps in flight)",
             8: "k_half_gemm_t<{t}> (LDS-staged, 128-row tile)",
             9: "k_half_gemm_t<{t}> (LDS-staged, 64-row tile, K split 4 ways)",
             10: "k_half_gemm_t<{t}> (LDS-staged, 128-row tile, K split 2 ways)",
             11: "k_half_gemm_t<{t}> (LDS-staged, 128-row tile, cost-ordered XCD-aware)",
             12: "k_half_gemm_t<{t}> (LDS-staged, 128-row tile, cost-ordered XCD-aware, 64-value chunks)"}
    t = "double" if dtype == "fp64" else "float"
    out = set()
    for i in s.info:
        narrow = False
        if op == 2:
            sched = i["fused_sched"][0 if dtype == "fp64" else 1]
        else:
            sched = i["gemm_sched"][2 * op + (0 if dtype == "fp64" else 1)]
            narrow = i.get("gemm_list", [32] * 4)[2 * op + (0 if dtype == "fp64" else 1)] == 16
        name = names.get(sched, "k_half_gemv_stream<{t}> (distinct blocks)").format(t=t)
        out.add(name + (" on 16-window items" if narrow and sched >= 0 else ""))
    return " + ".join(sorted(out))


# HBM-side bytes per launch of a kernel from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE) over `bench.py --kernel-only ...`, each scaled
# by what the counter reads for a 256 MiB device copy in the same run
# (fetch x2.000, write x1.000 on gfx950); the summaries are in profiles/.
# Keyed by (workload, operation, kernel): a run whose setup picked another
# kernel reports no traffic, and an entry is dropped when its kernel changes.
KERNEL_TRAFFIC = {
    ("c2", "schur", "k_half_gemm<double, 8> (split-K, 8 waves)"): 6.500e6,
    ("c2", "schur", "k_half_gemm<double, 16> (split-K, 16 waves)"): 6.460e6,
    ("c2", "schur", "k_half_gemm<double, 16> (split-K, 16 waves) on 16-window items"): 8.277e6,
    ("c2", "schur_bjinv", "k_half_gemm<double, 8> (split-K, 8 waves) over the stored S M^-1 blocks"): 2.173e7,
    ("c2", "schur_bjinv", "k_half_gemm<double, 16> (split-K, 16 waves) over the stored S M^-1 blocks"): 2.170e7,
    ("c3", "schur", "k_half_gemv_stream<double> (distinct blocks)"): 3.568e8,
    ("c4", "schur", "k_half_gemm_t<double> (LDS-staged, XCD-ordered)"): 9.906e7,
    ("c4", "schur", "k_half_gemm_t<double> (LDS-staged, 128-row tile, cost-ordered XCD-aware)"): 9.800e7,
}


def rooflines(cfg, s64, stream, reps):
    """Standalone launches of the kernels of the FP64 (and FP32) solve."""
    import torch
    import paper_1512_01756_amd as P
    dev = torch.device("cuda:0")
    x = torch.randn(s64.total_kS, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    x32, y32 = x.float(), y.float()
    fused = all(i["fused_op"][0] for i in s64.info)
    out = {}
    ms = kernel_ms(lambda: s64.apply_all(P.OP_SCHUR, x, y, P.FP64), reps, stream)
    fl, by = alg_schur(s64, (8, 8))
    out["schur_matvec_fp64"] = roofline(gemm_kernel_name(s64, 0, "fp64"), ms, fl, by, "fp64")
    ms = kernel_ms(lambda: s64.apply_all(P.OP_SCHUR, x32, y32, P.FP32_IR), reps, stream)
    fl, by = alg_schur(s64, (4, 4))
    out["schur_matvec_fp32"] = roofline(gemm_kernel_name(s64, 0, "fp32"), ms, fl, by, "fp32")
    ms = kernel_ms(lambda: s64.apply_all(P.OP_SCHUR_BJINV, x, y, P.FP64), reps, stream)
    fl, by = alg_schur_bjinv(s64, (8, 8))
    name = (gemm_kernel_name(s64, 2, "fp64") + " over the stored S M^-1 blocks" if fused
            else gemm_kernel_name(s64, 1, "fp64") + " then " + gemm_kernel_name(s64, 0, "fp64"))
    out["schur_bjinv_fp64"] = roofline(name, ms, fl, by, "fp64")
    out["schur_bjinv_fp64"]["fused"] = fused
    r = torch.randn(s64.total_r, dtype=torch.float64, device=dev)
    ro = torch.empty_like(r)
    ms = kernel_ms(lambda: s64.apply_all(P.OP_AINV, r, ro, P.FP64), max(reps // 4, 20), stream)
    fl, by = alg_ainv(s64)
    out["element_interior_fp64"] = roofline("k_colgemm(_t) D^-1, k_lambda, K^-1, correction", ms, fl, by, "fp64")
    for key, op in (("schur_matvec_fp64", "schur"), ("schur_bjinv_fp64", "schur_bjinv")):
        t = KERNEL_TRAFFIC.get((cfg, op, out[key]["kernel"]))
        out[key]["traffic"] = t
    return out


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, on the host cores

def host_cpu():
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except Exception:
        return {}
    keep = ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket", "Socket(s)", "CPU max MHz")
    out = {}
    for line in txt.splitlines():
        k, _, v = line.partition(":")
        if k.strip() in keep:
            out[k.strip()] = v.strip()
    return out


def cpu_baseline(seeds):
    """The oracle (FP64 NumPy/SciPy) on c2: setup once (reported, not in the
    sample), then one DBJ solve per right-hand-side seed with every BLAS
    thread, and three with one thread; plus the oracle's solution of seed 0
    at a 1e-12 residual for the parity figures."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import schur, smpm, solve
    from paper_1512_01756_amd import workloads
    prob = workloads.c2()
    grid = smpm.Grid(prob.xb, prob.zb, prob.n)
    t0 = time.perf_counter()
    o = schur.build(grid)
    setup_s = time.perf_counter() - t0
    Fs = [smpm.rhs(grid, o.tau, workloads.c2(seed=sd).f[0, 0]) for sd in seeds]
    times, mv, its = [], [], []
    for F in Fs:
        t0 = time.perf_counter()
        r = solve.dbj_solve(o, F)
        times.append(time.perf_counter() - t0)
        mv.append(r.iters + 2)     # one S per iteration, one in Q, one residual check
        its.append(r.iters)
    with threadpool_limits(limits=1):
        t1 = []
        for F in Fs[:3]:
            t0 = time.perf_counter()
            solve.dbj_solve(o, F)
            t1.append(time.perf_counter() - t0)
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    solve_s = float(np.median(times))
    ref12 = solve.dbj_solve(o, Fs[0], tol=1e-12)
    # the spread of k = 0 solutions that the null vectors' rounding allows
    floor = solve.null_vector_floor(o, Fs[0], samples=3, tol=1e-12)
    base = {"value": float(np.mean(mv) / solve_s), "unit": "matvecs/s", "cores": threads, "kind": "oracle",
            "sample": f"one full DBJ solve of each of the {len(Fs)} c2 right-hand sides (seeds "
                      f"{seeds[0]}-{seeds[-1]}) after a {setup_s:.1f} s oracle setup (setup not in the sample); "
                      f"median solve {solve_s * 1e3:.1f} ms, {int(np.median(its))} GMRES iterations",
            "time_to_1e-10_ms": solve_s * 1e3, "setup_s": setup_s,
            "one_thread": {"time_to_1e-10_ms": float(np.median(t1)) * 1e3,
                           "value": float(np.mean(mv) / np.median(t1)), "sample": "3 solves (seeds 0-2)"},
            "iterations": its, "host": host_cpu()}
    return base, ref12.u, its, floor


# ---------------------------------------------------------------------------

def bench_forms(cfg, forms, seeds, steps, warmup, stream, inner_tol=0.0, zlabel=0, setup="auto"):
    """Setup and timed solves of one workload in each precision."""
    import torch
    fs_np = [workload_rhs(cfg, sd) for sd in seeds]
    fs = [torch.as_tensor(f).cuda() for f in fs_np]
    u = torch.empty_like(fs[0])
    out = {}
    for name, prec in forms:
        t0 = time.perf_counter()
        s = make_solver(cfg, prec, inner_tol, zlabel, setup)
        setup_s = time.perf_counter() - t0
        per, total, stats, statuses = time_solves(s, fs, u, steps, warmup, stream)
        d = form_summary(per, total, stats, statuses)
        d["setup_s"] = setup_s
        # the solution of seed 0 (for the comparisons against the oracle)
        s.solve(fs[0], None, u, check=False)
        d["u0"] = u.cpu().numpy().copy()
        out[name] = (s, d, stats)
    return out, fs_np


def secondary(cfg, steps, warmup, stream, reps, inner_tol):
    """FP64 against FP32-refined time to 1e-10 on c3, c4 or c5 (3 seeds), and
    the kernels' rooflines there."""
    import torch
    import paper_1512_01756_amd as P
    forms, _ = bench_forms(cfg, (("fp64", P.FP64), ("fp32_ir", P.FP32_IR)), [0, 1, 2], steps, warmup, stream,
                           inner_tol)
    s64, d64, _ = forms["fp64"]
    _, d32, _ = forms["fp32_ir"]
    res = {"workload": WORKLOADS[cfg], "rhs_seeds": [0, 1, 2], "solves_timed": steps}
    for name, d in (("fp64", d64), ("fp32_ir", d32)):
        res[name] = {k: v for k, v in d.items() if k != "u0"}
    if d64["time_to_1e-10_ms"] and d32["time_to_1e-10_ms"]:
        res["fp32_ir_over_fp64"] = d32["time_to_1e-10_ms"] / d64["time_to_1e-10_ms"]
    res["rooflines"] = rooflines(cfg, s64, stream, reps)
    if cfg == "c3":
        # Distinct strips: the matvec streams its operator.  The FP64 blocks
        # (355 MB) exceed the 256 MB last-level cache; the FP32 ones (177 MB)
        # do not, so the FP32 rate is taken alternating two grids (two
        # operators, 354 MB).
        from paper_1512_01756_amd import workloads
        p1 = workloads.c3(seed=1)
        s1 = P.Solver(p1.xb, p1.zb, p1.n - 1)
        x = torch.randn(s64.total_kS, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        both = [s64, s1]
        k = [0]

        def alt():
            both[k[0] & 1].apply_all(P.OP_SCHUR, x, y, P.FP32_IR)
            k[0] += 1

        ms = kernel_ms(alt, 2 * reps, stream)
        fl, by = alg_schur(s64, (4, 4))
        res["rooflines"]["schur_matvec_fp32_two_operators"] = roofline(
            gemm_kernel_name(s64, 0, "fp32") + ", alternating two distinct grids", ms, fl, by, "fp32")
        res["operator_bytes"] = {"fp64": 8 * s64.info[0]["nnz_W_unique"], "fp32": 4 * s64.info[0]["nnz_W_unique"],
                                 "mall": MALL_BYTES}
        s1.close()
    if cfg == "c4":
        # The y transform of the 3-D problem alone (Sec. 5, Alg. 3): 128
        # planes of r nodes to 65 modes (Re, Im) and back; algorithmic bytes
        # are the planes read and the coefficients written (or back).
        from paper_1512_01756_amd import workloads
        p4 = workloads.c4()
        my, ly = 128, 8.0
        sf = P.Solver(p4.xb, p4.zb, p4.n - 1, fourier=(my, ly), tune=False)
        r = sf.info[0]["r"]
        fphys = torch.as_tensor(workloads.fourier_field(0, r, my)).cuda()
        fhat = torch.empty((my // 2 + 1, 2, r), dtype=torch.float64, device="cuda")
        back = torch.empty_like(fphys)
        nb = 8 * r * (my + 2 * (my // 2 + 1))
        ms_f = kernel_ms(lambda: sf.transform_y(fphys, fhat), reps, stream)
        ms_i = kernel_ms(lambda: sf.transform_y(fhat, back, inverse=True), reps, stream)
        res["transform_y"] = {"forward_us": ms_f * 1e3, "inverse_us": ms_i * 1e3, "bytes": nb,
                              "forward_GBps": nb / (ms_f * 1e-3) / 1e9, "inverse_GBps": nb / (ms_i * 1e-3) / 1e9,
                              "kernel": "k_fft_y_4s (length-8 then length-16 register DFTs, one LDS pass between, two real columns per complex FFT, m_y = 128)"}
        # from the physical field: transform, the batched mode solves, inverse
        for name, prec in (("fp64", P.FP64), ("fp32_ir", P.FP32_IR)):
            sp = P.Solver(p4.xb, p4.zb, p4.n - 1, fourier=(my, ly), precision=prec)
            uphys = torch.empty_like(fphys)
            for _ in range(warmup):
                sp.solve_fourier(fphys, None, uphys, check=False)
            res.setdefault("time_from_physical_field_ms", {})[name] = kernel_ms(
                lambda: sp.solve_fourier(fphys, None, uphys, check=False), steps, stream)
            sp.close()
        sf.close()
    for s, _, _ in forms.values():
        s.close()
    return res


def table2(stream, mxs, max_iter):
    """The comparison of Table 2 (Sec. 4) on the GPU: Schur, BJ, DBJ and 2LAS
    iterations and solve times on [0, m_x] x [0, 1] grids of m_x x 10
    elements, n = 10, f ~ U[0, 1] (seed 0), FP64, tol 1e-10.  One setup per
    grid; the other methods load its saved tables."""
    import tempfile
    import torch
    import paper_1512_01756_amd as P
    out = {}
    methods = (("schur", P.METHOD_SCHUR), ("bj", P.METHOD_BJ), ("dbj", P.METHOD_DBJ), ("2las", P.METHOD_2LAS))
    for mx in mxs:
        xb = np.linspace(0.0, float(mx), mx + 1)
        zb = np.linspace(0.0, 1.0, 11)
        n = 10
        f = torch.as_tensor(np.random.default_rng(0).uniform(0.0, 1.0, n * n * mx * 10)).cuda()
        u = torch.empty_like(f)
        t0 = time.perf_counter()
        s = P.Solver(xb, zb, n - 1, max_iter=max_iter)
        setup_s = time.perf_counter() - t0
        row = {"setup_s": setup_s, "k_S": s.total_kS}
        with tempfile.TemporaryDirectory() as td:
            path = os.path.join(td, "t.bin")
            s.save(path)
            for name, m in methods:
                sm = s if m == P.METHOD_DBJ else P.Solver(load_path=path, method=m, max_iter=max_iter)
                per, total, stats, statuses = time_solves(sm, [f], u, 3, 1, stream)
                d = form_summary(per, total, stats, statuses)
                row[name] = {"iterations": d["iters_max"], "solve_ms": d["time_to_1e-10_ms"], "status": d["status"]}
                if sm is not s:
                    sm.close()
        s.close()
        out[str(mx)] = row
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the c3 / c4 / c5 keys")
    ap.add_argument("--no-table2", action="store_true", help="skip the Table 2 method comparison")
    ap.add_argument("--table2-mx", default="64,128,256,512,1024")
    ap.add_argument("--matvec-reps", type=int, default=200)
    ap.add_argument("--kernel-only", choices=("schur", "schur_bjinv", "ainv"),
                    help="run one FP64 kernel alone (plus a 256 MiB copy that calibrates the byte counters)")
    ap.add_argument("--solve-only", action="store_true", help="one precision's setup and timed solves only")
    ap.add_argument("--solve-precision", default="fp64", choices=("fp64", "fp32_ir", "fp16s_ir"),
                    help="the precision --solve-only times")
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

    if args.kernel_only:
        s = make_solver(args.config, P.FP64, setup=args.setup)
        op = {"schur": P.OP_SCHUR, "schur_bjinv": P.OP_SCHUR_BJINV, "ainv": P.OP_AINV}[args.kernel_only]
        n = s.total_r if op == P.OP_AINV else s.total_kS
        x = torch.randn(n, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        ms = kernel_ms(lambda: s.apply_all(op, x, y, P.FP64), args.matvec_reps, stream)
        cbytes = 256 << 20
        a = torch.ones(cbytes // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        cms = kernel_ms(lambda: b.copy_(a), 5, stream)
        alg = {"schur": alg_schur(s, (8, 8)), "schur_bjinv": alg_schur_bjinv(s, (8, 8)), "ainv": alg_ainv(s)}
        print(json.dumps({"config": args.config, "kernel": args.kernel_only, "launch_us": ms * 1e3,
                          "algorithmic_flops": alg[args.kernel_only][0], "algorithmic_bytes": alg[args.kernel_only][1],
                          "copy_bytes_each_way": cbytes, "copy_us": cms * 1e3}), flush=True)
        s.close()
        return

    seeds = list(range(10)) if args.config == "c2" else [0, 1, 2]
    if args.solve_only:
        name = args.solve_precision
        prec = {"fp64": P.FP64, "fp32_ir": P.FP32_IR, "fp16s_ir": P.FP16S_IR}[name]
        forms, _ = bench_forms(args.config, ((name, prec),), seeds, args.steps, args.warmup, stream,
                               args.inner_tol, args.zlabel, args.setup)
        d = forms[name][1]
        print(json.dumps({"config": args.config, name: {k: v for k, v in d.items() if k != "u0"}}), flush=True)
        return

    forms, fs_np = bench_forms(args.config, (("fp64", P.FP64), ("fp32_ir", P.FP32_IR), ("fp16s_ir", P.FP16S_IR)),
                               seeds, args.steps, args.warmup, stream, args.inner_tol, args.zlabel, args.setup)
    s64, fp64, stats64 = forms["fp64"]
    _, ir, _ = forms["fp32_ir"]
    _, ir16, _ = forms["fp16s_ir"]

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
            physical[name] = kernel_ms(lambda: sf.solve_fourier(fphys, None, uphys), args.steps, stream)
            if one:
                _, st1, _ = sf.solve_fourier(fphys, None, uphys)
                physical["one_krylov_iterations"] = st1["iters_max"]
                physical["one_krylov_rel_residual_max"] = st1["rel_residual_max"]
            sf.close()

    rl = rooflines(args.config, s64, stream, args.matvec_reps)
    # The dominant kernel of the timed FP64 solve: the operator it applies in
    # every GMRES iteration (S M^-1, one GEMM where the setup chose the
    # stored product blocks).
    main_rl = dict(rl["schur_bjinv_fp64"])

    value = fp64["matvecs_per_s"]
    i0 = s64.info[0]
    line = {
        "metric": "Schur matvecs/s + time-to-1e-10 residual, FP64 vs FP32-refined, 1 GPU",
        "value": value,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp64["mean_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "systems": s64.nsys,
                   "deflation": "per element segment" if args.zlabel else "per interface",
                   "instances": stats64[0]["instances"], "k_S_total": s64.total_kS, "r_total": s64.total_r,
                   "rhs_seeds": seeds,
                   "first_system": {"mx": i0["mx"], "mz": i0["mz"], "n": i0["n"], "d": i0["d"]}},
        "value_definition": "Schur matvecs of the timed FP64 DBJ solves (step i: right-hand side of seed i mod "
                            f"{len(seeds)}) over their total time",
        "time_to_1e-10_ms": {"fp64": fp64["time_to_1e-10_ms"], "fp32_ir": ir["time_to_1e-10_ms"],
                             "fp16s_ir": ir16["time_to_1e-10_ms"], "statistic": "median over the timed solves"},
        "time_to_1e-10_ms_from_physical_field": physical,
        "iterations": {"fp64_max": fp64["iters_max"], "fp64_total": fp64["iters_total"],
                       "fp32_ir_inner_max": ir["iters_max"], "fp32_ir_inner_total": ir["iters_total"],
                       "fp32_ir_sweeps": ir["sweeps"],
                       "fp16s_ir_inner_max": ir16["iters_max"], "fp16s_ir_inner_total": ir16["iters_total"],
                       "fp16s_ir_sweeps": ir16["sweeps"], "fp16s_ir_status": ir16["status"],
                       "fp32_ir_status": ir["status"], "fp64_status": fp64["status"]},
        "rel_residual_max": {"fp64": fp64["rel_residual_max"], "fp32_ir": ir["rel_residual_max"],
                             "fp16s_ir": ir16["rel_residual_max"]},
        "setup_s": {"fp64": fp64["setup_s"], "fp32_ir": ir["setup_s"], "fp16s_ir": ir16["setup_s"]},
        "gemm_schedules": {"matvec_S64_S32_M64_M32": i0["gemm_sched"],
                           "matvec_windows_per_item": i0["gemm_list"], "element": i0["elem_sched"],
                           "element_16_column_list": i0["elem_alt"], "rhs_gemm_sched_windows": i0["rhs_gemm"],
                           "fused_S_Minv_used_fp64_fp32": [i0["fused_op"][0],
                                                           forms["fp32_ir"][0].info[0]["fused_op"][1]],
                           "fused_S_Minv_sched_fp64_fp32": [i0["fused_sched"][0],
                                                            forms["fp32_ir"][0].info[0]["fused_sched"][1]],
                           "legend": "0 split-K 16 waves, 1 split-K 8 waves, 2 LDS-staged XCD-ordered, 3 LDS-staged plain; matvec lists: "
                                     "4 / 5 = 2 / 3 with 64-value chunks, 6 / 7 split-K 8 / 16 waves with a wave's K range in "
                                     "flight, 8 LDS-staged 128-row tiles, 9 / 10 64- / 128-row tiles whose waves also split K, "
                                     "11 / 12 128-row tiles in a cost-ordered XCD-aware order with 32- / 64-value chunks; "
                                     "element lists: 4 / 5 LDS-staged 32- / 16-row tiles with K split over the waves; -1 unused; "
                                     "element_16_column_list: the schedule of a product run as one launch over items of at "
                                     "most 16 columns, -1 where its two width lists run; picked by timing at setup"},
        "roofline": main_rl,
        "rooflines": rl,
    }
    if not args.no_cpu_baseline and args.config == "c2":
        line["cpu_baseline"], u_oracle, its, floor = cpu_baseline(seeds)
        line["iterations"]["oracle_fp64"] = its
        # Parity: each form solved to a 1e-12 residual on seed 0 against the
        # oracle's 1e-12 solution of the same right-hand side (max abs
        # difference over max |u|, both zero-mean); and the timed 1e-10
        # solutions against the same oracle solution (their distance from
        # the discrete solution, about the 1e-10 tolerance itself).
        scale = float(np.abs(u_oracle).max())
        f0 = torch.as_tensor(fs_np[0]).cuda()
        u = torch.empty_like(f0)
        par = {}
        for name, prec, tol in (("fp64", P.FP64, 1e-12), ("fp32_ir", P.FP32_IR, 4e-12),
                                ("fp16s_ir", P.FP16S_IR, 1e-11)):
            st_ = make_solver(args.config, prec, args.inner_tol, args.zlabel, args.setup, tol=tol)
            _, stt, status = st_.solve(f0, None, u, check=False)
            par[name] = float(np.abs(u.cpu().numpy() - u_oracle).max() / scale) if status == 0 else None
            par[name + "_residual"] = stt["rel_residual_max"]
            st_.close()
        line["error_vs_oracle"] = par
        line["error_vs_oracle"]["bound"] = max(1e-10, 10 * floor)
        line["error_vs_oracle"]["null_vector_floor"] = floor
        line["error_vs_oracle"]["definition"] = (
            "max |u - u_oracle| / max |u_oracle|, seed 0; the oracle at a 1e-12 Schur residual, the GPU at 1e-12 "
            "(FP64), 4e-12 (FP32-IR), 1e-11 (FP16S-IR); bound: the larger of 1e-10 and ten times the oracle's "
            "null-vector floor for this input")
        line["timed_solution_error_vs_oracle"] = {k: float(np.abs(v[1]["u0"] - u_oracle).max() / scale)
                                                 for k, v in forms.items()}
    for s, _, _ in forms.values():
        s.close()
    if not args.no_secondary and args.config == "c2":
        line["workloads"] = {c: secondary(c, 6, 2, stream, max(args.matvec_reps // 4, 20), args.inner_tol)
                             for c in ("c3", "c4", "c5")}
    if not args.no_table2 and not args.no_secondary:
        line["table2"] = table2(stream, [int(v) for v in args.table2_mx.split(",")], 1200)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
