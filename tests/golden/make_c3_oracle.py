"""Write tests/golden/c3_oracle.npz: the oracle's Algorithm 2 solve of the
full-size stretched-grid workload (256 x 16 elements, order 12, seeded strip
widths and f ~ U[0, 1]), for the GPU parity test at that size.

The oracle needs several minutes for this grid (256 dense strip
factorizations and the Schur blocks), too long to repeat inside every GPU
test run, so its results are stored.  For the benchmark's right-hand side:
the FP64 iteration count at the 1e-10 tolerance, the solution at a 1e-12
Schur residual on seeded sample nodes (with max |u| for the relative scale),
and the sweeps and per-sweep inner iterations of the FP32-inner refinement
emulation.  For a compatible right-hand side F = L v on the same grid (v the
seeded smooth field of workloads.smooth_field): the solution samples, the
measured growth of the solution error with the Schur residual, and the
oracle's own distance from v minus its mean (the discrete solution up to
the rounding of F), which is the accuracy FP64 attains on this grid.  Only oracle/
and the seeded input generators are called.

usage: python tests/golden/make_c3_oracle.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np

from oracle import schur, smpm, solve
from paper_1512_01756_amd import workloads

SAMPLES = 40000
SAMPLE_SEED = 12
SMOOTH_SEED = 7


def main():
    p = workloads.c3()
    grid = smpm.Grid(p.xb, p.zb, p.n)
    t0 = time.perf_counter()
    o = schur.build(grid)
    print(f"build {time.perf_counter() - t0:.1f} s", flush=True)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(grid.r, SAMPLES, replace=False))
    out = {"sample_seed": SAMPLE_SEED, "idx": idx.astype(np.int32)}
    # The benchmark's right-hand side, f ~ U[0, 1]: far from compatible.
    F = smpm.rhs(grid, o.tau, p.f[0, 0])
    r10 = solve.dbj_solve(o, F, tol=1e-10)
    print("1e-10:", r10.iters, r10.schur_relres, flush=True)
    r12 = solve.dbj_solve(o, F, tol=1e-12)
    print("1e-12:", r12.iters, r12.schur_relres, "compatibility defect", r12.compat_defect, flush=True)
    ir, sweeps, total = solve.refine_solve(o, F, inner_tol=1e-4, tol=1e-10, floor=0.5)
    print("fp32 refinement:", sweeps, ir.inner, ir.schur_relres, flush=True)
    out.update(u=r12.u[idx], umax=np.abs(r12.u).max(), iters_1e10=r10.iters, iters_1e12=r12.iters,
               relres_1e12=r12.schur_relres, ir_sweeps=sweeps, ir_inner=np.array(ir.inner), ir_total=total,
               compat_defect=r12.compat_defect)
    # A compatible right-hand side on the same grid, F = L v for the seeded
    # smooth field v: its solution does not move with the null vectors.  The
    # solutions at 1e-10 and 1e-12 give the growth of the error with the
    # Schur residual (kappa_u) on this grid.
    v = workloads.smooth_field(p.xb, p.zb, p.n, SMOOTH_SEED)
    Fc = smpm.assemble_L(grid, o.tau) @ v
    c10 = solve.dbj_solve(o, Fc, tol=1e-10)
    c12 = solve.dbj_solve(o, Fc, tol=1e-12)
    scale = np.abs(c12.u).max()
    kappa = float(np.abs(c10.u - c12.u).max() / scale / (c10.schur_relres - c12.schur_relres))
    print("compatible: iterations", c10.iters, c12.iters, "residuals", c10.schur_relres, c12.schur_relres,
          "kappa_u", kappa, "compatibility defect", c12.compat_defect, flush=True)
    exact = v - v.mean()
    c_err = float(np.abs(c12.u - exact).max() / np.abs(exact).max())
    print("compatible: the oracle's 1e-12 solution against v minus its mean", c_err, flush=True)
    out.update(smooth_seed=SMOOTH_SEED, uc=c12.u[idx], ucmax=scale, c_iters_1e10=c10.iters,
               c_relres_1e12=c12.schur_relres, kappa_u=kappa, c_err_exact=c_err)
    np.savez(os.path.join(HERE, "c3_oracle.npz"), **out)


if __name__ == "__main__":
    main()
