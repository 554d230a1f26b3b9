"""Pins of the oracle's 3-D (Fourier in y) path, Sec. 5."""
import numpy as np
import pytest

from oracle import fourier, smpm


def test_forward_of_a_single_cosine_and_sine():
    # closed form: cos(2 pi m0 j / my) has coefficient 1/2 at m0 (Re), sin has -1/2 (Im)
    my, m0 = 8, 3
    j = np.arange(my)
    f = np.stack([np.cos(2 * np.pi * m0 * j / my), np.sin(2 * np.pi * m0 * j / my)], axis=1)
    fh = fourier.forward(f)
    expect = np.zeros_like(fh)
    expect[m0, 0, 0] = 0.5
    expect[m0, 1, 1] = -0.5
    assert np.abs(fh - expect).max() < 1e-15
    # the constant goes to mode 0 with weight 1, the Nyquist mode to m = my/2
    fc = fourier.forward(np.stack([np.ones(my), (-1.0) ** j], axis=1))
    assert abs(fc[0, 0, 0] - 1.0) < 1e-15 and abs(fc[my // 2, 0, 1] - 1.0) < 1e-15


@pytest.mark.parametrize("my", [8, 7])
def test_inverse_undoes_forward(my):
    f = np.random.default_rng(1).standard_normal((my, 5))
    assert np.abs(fourier.inverse(fourier.forward(f), my) - f).max() < 1e-14


def test_manufactured_3d_solution():
    # u = cos(pi x / lx) cos(pi z) cos(2 pi y / ly): Neumann data vanish on the x and z
    # sides; the z-y Laplacian adds -(2 pi / ly)^2, carried by the k_1 mode.
    lx, ly, my = 2.0, 3.0, 6
    xb = np.linspace(0, lx, 5)
    zb = np.linspace(0, 1, 3)
    n = 9
    grid = smpm.Grid(xb, zb, n)
    X, Z = grid.coords()
    ys = np.arange(my) * ly / my
    lap = -(np.pi ** 2 / lx ** 2 + np.pi ** 2 + (2 * np.pi / ly) ** 2)
    ue = np.array([np.cos(np.pi * X / lx) * np.cos(np.pi * Z) * np.cos(2 * np.pi * y / ly) for y in ys])
    u, res = fourier.solve3d(xb, zb, n, lap * ue, ly)
    assert np.abs(u - ue).max() < 1e-6
    # only the k_1 mode was excited
    uh = fourier.forward(u)
    assert np.abs(np.delete(uh, 1, axis=0)).max() < 1e-12


def test_mode_solves_are_independent():
    # a field with one mode gives a solution with that mode only
    xb = np.linspace(0, 3, 4)
    zb = np.linspace(0, 1, 3)
    n, my, ly = 5, 8, 2.0
    grid = smpm.Grid(xb, zb, n)
    rng = np.random.default_rng(3)
    shape = rng.uniform(0, 1, grid.r)
    j = np.arange(my)
    f = np.array([shape * np.sin(2 * np.pi * 2 * jj / my) for jj in j])
    u, _ = fourier.solve3d(xb, zb, n, f, ly)
    uh = fourier.forward(u)
    assert np.abs(np.delete(uh, 2, axis=0)).max() < 1e-12
    assert np.abs(uh[2, 1]).max() > 1e-3


def test_one_krylov_over_all_modes_gives_the_same_solution():
    # Sec. 5.2: one GMRES over the block-diagonal operator of every mode solves
    # the same linear systems; the solution agrees with the per-mode solves.
    xb = np.array([0.0, 0.6, 1.1, 1.9, 2.4, 3.0])
    zb = np.array([0.0, 0.5, 1.0])
    n, my, ly = 5, 6, 2.0
    grid = smpm.Grid(xb, zb, n)
    f = np.random.default_rng(5).uniform(0, 1, (my, grid.r))
    u1, res1 = fourier.solve3d(xb, zb, n, f, ly, tol=1e-12)
    u2, (it, ok) = fourier.solve3d(xb, zb, n, f, ly, tol=1e-12, one_krylov=True)
    assert ok
    assert np.abs(u1 - u2).max() <= 1e-9 * np.abs(u1).max()
