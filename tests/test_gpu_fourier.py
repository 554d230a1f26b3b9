"""GPU parity of the 3-D path (Sec. 5): physical-space input, the transform in
y, the batched per-mode solves and the inverse transform, against the oracle's
mode-by-mode solve on the same seeded field."""
import numpy as np
import pytest

import paper_1512_01756_amd as P
from oracle import fourier, smpm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("my,with_g,precision", [(8, False, P.FP64), (6, True, P.FP64), (7, False, P.FP64),
                                                 (8, True, P.FP32_IR)])
def test_physical_solve_matches_oracle(my, with_g, precision):
    xb = np.array([0.0, 0.5, 1.1, 1.6, 2.0, 2.7])
    zb = np.array([0.0, 0.4, 1.0])
    n, ly = 6, 2.5
    grid = smpm.Grid(xb, zb, n)
    rng = np.random.default_rng(my + 10 * with_g)
    f = rng.uniform(0.0, 1.0, (my, grid.r))
    g = None
    if with_g:
        mx, mz = len(xb) - 1, len(zb) - 1
        g = {"S": rng.standard_normal((my, mx, n)), "N": rng.standard_normal((my, mx, n)),
             "W": rng.standard_normal((my, mz, n)), "E": rng.standard_normal((my, mz, n))}
    u_ref, res = fourier.solve3d(xb, zb, n, f, ly, g)
    s = P.Solver(xb, zb, n - 1, fourier=(my, ly), precision=precision)
    assert s.nsys == my // 2 + 1
    gd = None
    if g is not None:
        gd = _dev(np.concatenate([g[k].reshape(my, -1) for k in ("S", "N", "W", "E")], axis=1))
    u, st, status = s.solve_fourier(_dev(f), gd)
    torch.cuda.synchronize()
    u = u.cpu().numpy()
    print("fourier", my, with_g, st, _rel(u, u_ref))
    assert st["rel_residual_max"] <= 1.001e-10
    assert _rel(u, u_ref) <= (1e-9 if precision == P.FP64 else 1e-8)


def test_manufactured_3d_solution_on_gpu():
    lx, ly, my = 2.0, 3.0, 6
    xb = np.linspace(0, lx, 5)
    zb = np.linspace(0, 1, 3)
    n = 9
    grid = smpm.Grid(xb, zb, n)
    X, Z = grid.coords()
    ys = np.arange(my) * ly / my
    lap = -(np.pi ** 2 / lx ** 2 + np.pi ** 2 + (2 * np.pi / ly) ** 2)
    ue = np.array([np.cos(np.pi * X / lx) * np.cos(np.pi * Z) * np.cos(2 * np.pi * y / ly) for y in ys])
    s = P.Solver(xb, zb, n - 1, fourier=(my, ly))
    u, st, _ = s.solve_fourier(_dev(lap * ue))
    assert np.abs(u.cpu().numpy() - ue).max() < 1e-6


def test_solve_fourier_rejects_plain_handles():
    s = P.Solver(np.linspace(0, 3, 5), np.linspace(0, 1, 2), 4)
    f = torch.zeros((4, s.info[0]["r"]), dtype=torch.float64, device="cuda")
    with pytest.raises(P.SmpmError):
        s.solve_fourier(f)


@pytest.mark.parametrize("precision", [P.FP64, P.FP32_IR])
def test_one_krylov_over_all_modes_matches_oracle(precision):
    # Sec. 5.2 / Alg. 3: one DBJ-GMRES over the block-diagonal operator of
    # every (mode, Re/Im) instance; same solution, iteration count within one.
    xb = np.array([0.0, 0.6, 1.1, 1.9, 2.4, 3.0])
    zb = np.array([0.0, 0.5, 1.0])
    n, my, ly = 5, 6, 2.0
    grid = smpm.Grid(xb, zb, n)
    f = np.random.default_rng(5).uniform(0, 1, (my, grid.r))
    u_ref, (it_ref, ok) = fourier.solve3d(xb, zb, n, f, ly, one_krylov=True)
    s = P.Solver(xb, zb, n - 1, fourier=(my, ly), one_krylov=True, precision=precision)
    u, st, _ = s.solve_fourier(_dev(f))
    u = u.cpu().numpy()
    print("one krylov", st, "oracle iters", it_ref, _rel(u, u_ref))
    assert ok
    if precision == P.FP64:
        assert abs(st["iters_max"] - it_ref) <= 1
        assert st["iters_total"] == st["iters_max"] * st["instances"]
        assert _rel(u, u_ref) <= 1e-9
    else:
        assert st["rel_residual_max"] <= 1.001e-10 * 10   # the stacked residual is controlled, not each mode's
        assert _rel(u, u_ref) <= 1e-8


def test_one_krylov_needs_dbj():
    with pytest.raises(P.SmpmError):
        P.Solver(np.linspace(0, 3, 5), np.linspace(0, 1, 2), 4, fourier=(4, 1.0), one_krylov=True,
                 method=P.METHOD_BJ)


@pytest.mark.parametrize("my", [2, 4, 8, 16, 32, 64, 128, 256, 2048, 6, 12])
def test_transform_y_matches_numpy_fft(my):
    # The y transform alone (for powers of two an FFT with two real columns
    # per complex FFT: two register steps from m_y = 16 to 128, radix-2
    # stages in LDS for 8 and 256 .. 2048, unpacked below 8; the dense real
    # DFT otherwise) against the oracle's numpy real FFT, both directions, on
    # a seeded field with a ragged last column tile (r = 25 * 2 * 36 = 1800
    # columns is not a multiple of the 4096 / m_y columns a workgroup takes
    # for m_y = 8, 16, 32, 64, 128 and 256).
    xb, zb, n = np.linspace(0.0, 12.5, 26), np.array([0.0, 0.5, 1.0]), 6
    s = P.Solver(xb, zb, n - 1, fourier=(my, 3.0), tune=False)
    r = s.info[0]["r"]
    assert r == 1800
    f = np.random.default_rng(my).uniform(-1.0, 1.0, (my, r))
    fh = torch.empty((my // 2 + 1, 2, r), dtype=torch.float64, device="cuda")
    s.transform_y(_dev(f), fh)
    back = torch.empty((my, r), dtype=torch.float64, device="cuda")
    s.transform_y(fh, back, inverse=True)
    torch.cuda.synchronize()
    ref = fourier.forward(f)
    assert _rel(fh.cpu().numpy(), ref) <= 1e-14
    assert _rel(back.cpu().numpy(), f) <= 1e-14
    # inverse of arbitrary coefficients: Im of modes 0 and m_y/2 are ignored
    c = np.random.default_rng(my + 1).standard_normal((my // 2 + 1, 2, r))
    s.transform_y(_dev(c), back, inverse=True)
    torch.cuda.synchronize()
    assert _rel(back.cpu().numpy(), fourier.inverse(c, my)) <= 1e-13
    s.close()
