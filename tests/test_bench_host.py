"""Host-side pieces of bench.py: the single-GPU rule, the algorithmic work
per launch that the rooflines divide by, and the guard that attaches the
measured HBM traffic only to the kernel the counters were taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import paper_1512_01756_amd as P  # noqa: E402
from paper_1512_01756_amd import workloads  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


class _Info:
    def __init__(self, infos):
        self.info = infos


def test_c2_algorithmic_work_from_the_grid():
    # 128 x 8 elements of order 16: N = 17 * 8 = 136 rows per half, 254 halves,
    # k_S = 254 * 136 = 34544.  Sum_j |W_j| = 126 (2N)^2 + 2 N^2 (the end
    # strips touch one interface); distinct nonzeros: the first and last
    # strips' N x N blocks and the interior strip's two N x 2N row blocks,
    # 6 N^2 = 110976 entries.  Block-Jacobi: 63 blocks of 4N plus one of 2N.
    p = workloads.c2()
    s = P.Solver(p.xb, p.zb, p.n - 1, host_only=True)
    try:
        i = s.info[0]
        N = 136
        assert i["n"] == 17 and i["mz"] == 8 and i["kS"] == 254 * N == 34544
        assert i["nnz_W_total"] == 126 * (2 * N) ** 2 + 2 * N * N == 9358976
        assert i["nnz_W_unique"] == 6 * N * N == 110976
        assert i["nnz_M_total"] == 63 * (4 * N) ** 2 + (2 * N) ** 2 == 18717952
        fl, by = bench.alg_schur(s, (8, 8))
        assert fl == 2 * 9358976 + 34544 and by == 8 * 110976 + 2 * 8 * 34544 == 1440512
        fl2, by2 = bench.alg_schur_bjinv(s, (8, 8))
        assert fl2 == 2 * (9358976 + 18717952) + 34544
        assert by2 == 8 * (110976 + i["nnz_M_unique"]) + 2 * 8 * 34544
        fl3, by3 = bench.alg_ainv(s)
        assert fl3 > 2 * i["r"] * 17 ** 2 and by3 > 2 * 8 * i["r"]
    finally:
        s.close()


def test_roofline_takes_the_binding_roof():
    r = bench.roofline("k", 0.01, 78.6e12 * 1e-6, 1.0, "fp64")     # 1 us of MFMA work in 10 us
    assert r["bound"] == "mfma" and r["frac"] == pytest.approx(0.1)
    r = bench.roofline("k", 0.01, 1.0, 8e12 * 2e-6, "fp64")        # 2 us of HBM traffic in 10 us
    assert r["bound"] == "hbm" and r["frac"] == pytest.approx(0.2)


def test_traffic_only_for_the_measured_kernel():
    shared = {"gemm_sched": [1, 1, 1, 1]}
    name = bench.gemm_kernel_name(_Info([shared]), 0, "fp64")
    assert ("c2", "schur", name) in bench.KERNEL_TRAFFIC
    other = dict(shared, gemm_sched=[3, 3, 3, 3])
    assert ("c2", "schur", bench.gemm_kernel_name(_Info([other]), 0, "fp64")) not in bench.KERNEL_TRAFFIC
    fused = {"fused_sched": [0, 7]}
    name = bench.gemm_kernel_name(_Info([fused]), 2, "fp64") + " over the stored S M^-1 blocks"
    assert ("c2", "schur_bjinv", name) in bench.KERNEL_TRAFFIC
    narrow = dict(shared, gemm_list=[16, 16, 16, 16])   # the same schedule on the 16-window list
    assert ("c2", "schur", bench.gemm_kernel_name(_Info([narrow]), 0, "fp64")) not in bench.KERNEL_TRAFFIC
    distinct = {"gemm_sched": [-1, -1, -1, -1]}
    assert ("c3", "schur", bench.gemm_kernel_name(_Info([distinct]), 0, "fp64")) in bench.KERNEL_TRAFFIC
