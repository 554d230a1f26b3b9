"""Device-side setup: the strip solves behind the Schur blocks W, the u_S
block elimination and inverse iteration and the block-Jacobi and coarse
inverses on rocSOLVER / rocBLAS, against the host setup (the same steps on
the host threads, pinned to the oracle by the CPU tests) and against the
oracle's solution."""
import numpy as np
import pytest

import paper_1512_01756_amd as P
from paper_1512_01756_amd import workloads
from oracle import schur, smpm, solve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load()


ACCEPT = 1.001e-10


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("k,zlabel", [(0.0, 0), (0.0, 1), (1.3, 0)])
def test_device_setup_matches_host_setup_and_oracle(k, zlabel):
    p = workloads.random_problem(12, 3, 6, kwaves=(k,), seed=41, stretch=True, with_g=True)
    sh = P.Solver(p.xb, p.zb, p.n - 1, kwaves=p.kwaves, tune=False, zlabel=zlabel, setup="host")
    sd = P.Solver(p.xb, p.zb, p.n - 1, kwaves=p.kwaves, tune=False, zlabel=zlabel, setup="device")
    assert sh.info[0]["setup_device"] == 0
    # every supported step ran on the device: u_S (k = 0 only), M inverses,
    # coarse, W blocks, element and capacitance inverses
    assert sd.info[0]["setup_device"] == (31 if k == 0 else 30)
    assert _rel(sd.export(P.TABLE_SCHUR_DENSE), sh.export(P.TABLE_SCHUR_DENSE)) <= 1e-12
    assert _rel(sd.export(P.TABLE_BJINV_DENSE), sh.export(P.TABLE_BJINV_DENSE)) <= 1e-11
    if k == 0:
        assert _rel(sd.export(P.TABLE_U_S), sh.export(P.TABLE_U_S)) <= 1e-9
        assert _rel(sd.export(P.TABLE_U_C), sh.export(P.TABLE_U_C)) <= 1e-11
    f = _dev(p.f.reshape(-1))
    g = _dev(P.pack_g(p.g, sd.info, 1))
    ud, std_, _ = sd.solve(f, g)
    uh, sth, _ = sh.solve(f, g)
    torch.cuda.synchronize()
    grid = smpm.Grid(p.xb, p.zb, p.n)
    o = schur.build(grid, kwave=k, zlabel=zlabel)
    F = smpm.rhs(grid, o.tau, p.f[0, 0], {side: arr[0, 0] for side, arr in p.g.items()})
    ref = solve.dbj_solve(o, F)
    ud, uh = ud.cpu().numpy(), uh.cpu().numpy()
    print("iters device/host/oracle", std_["iters_max"], sth["iters_max"], ref.iters, "rel", _rel(ud, ref.u))
    assert std_["rel_residual_max"] <= ACCEPT
    assert abs(std_["iters_max"] - ref.iters) <= 1
    assert _rel(ud, ref.u) <= 1e-9
    assert _rel(ud, uh) <= 1e-9


def test_automatic_device_setup_on_a_large_grid():
    # 160 distinct strips of 16 elements, order 12: the u_S elimination (159
    # interfaces of 2N = 416) takes the device path by default; the 80
    # block-Jacobi inverses of 832 x 832 (9.2e10 flops) and the W blocks'
    # strip solves go either way with the host's thread count.
    p = workloads.random_problem(160, 16, 13, seed=7, stretch=True)
    sa = P.Solver(p.xb, p.zb, p.n - 1, tune=False)
    sh = P.Solver(p.xb, p.zb, p.n - 1, tune=False, setup="host")
    print("device steps", sa.info[0]["setup_device"])
    assert sa.info[0]["setup_device"] & 1
    assert sh.info[0]["setup_device"] == 0
    assert _rel(sa.export(P.TABLE_U_S), sh.export(P.TABLE_U_S)) <= 1e-9
    f = _dev(p.f.reshape(-1))
    ua, sta, _ = sa.solve(f)
    uh, sth, _ = sh.solve(f)
    torch.cuda.synchronize()
    print("iters auto/host", sta["iters_max"], sth["iters_max"], "rel", _rel(ua.cpu().numpy(), uh.cpu().numpy()))
    assert sta["rel_residual_max"] <= ACCEPT and sth["rel_residual_max"] <= ACCEPT
    assert abs(sta["iters_max"] - sth["iters_max"]) <= 1
    assert _rel(ua.cpu().numpy(), uh.cpu().numpy()) <= 1e-8
