"""Host-side pieces of bench.py: the single-GPU rule, the algorithmic work
per Schur matvec that the roofline divides by, and the guard that attaches
the measured HBM traffic only to the kernel the counters were taken on."""
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


def test_c2_matvec_work_from_the_grid():
    # 128 x 8 elements of order 16: N = 17 * 8 = 136 rows per half, 254 halves,
    # k_S = 254 * 136 = 34544.  The uniform x-grid leaves four distinct N x 2N
    # half blocks, one per (strip class, row side) a half can face: the west
    # rows of an interior or the last strip, the east rows of the first or an
    # interior strip.  Bytes 4 * 136 * 272 * 8 plus the input and output
    # vectors; flops 2 * 254 * 136 * 272 + k_S.
    p = workloads.c2()
    s = P.Solver(p.xb, p.zb, p.n - 1, host_only=True)
    try:
        i = s.info[0]
        assert i["n"] == 17 and i["mz"] == 8 and i["kS"] == 34544 and i["unique_W"] == 4
        assert bench.matvec_bytes(s, 8, 8) == 4 * 136 * 272 * 8 + 2 * 34544 * 8 == 1736448
        assert bench.matvec_flops(s) == 2 * 254 * 136 * 272 + 34544 == 18826480
    finally:
        s.close()


def test_traffic_only_for_the_measured_kernel():
    shared = {"unique_W": 4, "mx": 128, "gemm_sched": [0, 0, 0, 0]}
    assert bench.matvec_kernel_name(_Info([shared])) == bench.MATVEC_TRAFFIC["c2"][0]
    other = dict(shared, gemm_sched=[1, 0, 0, 0])
    assert bench.matvec_kernel_name(_Info([other])) != bench.MATVEC_TRAFFIC["c2"][0]
    distinct = {"unique_W": 2 * 255, "mx": 256, "gemm_sched": [-1, -1, -1, -1]}
    assert bench.matvec_kernel_name(_Info([distinct])) == bench.MATVEC_TRAFFIC["c3"][0]
    for sched in range(6):
        assert sched in bench.GEMM_KERNELS
