"""Seeded synthetic inputs for the SMPM Schur solver.

This module holds no arithmetic of the method: it draws grids and data only.
It is the one piece shared by the GPU library's tests/benchmark and the CPU
oracle.  Node coordinates are computed here with numpy.polynomial (the
Legendre roots), a third route independent of both solvers.

Layouts (shared by the C ABI and the oracle):
  f, u:  node(j, e, b, a) = ((j * m_z + e) * n + b) * n + a   (a fastest)
  g:     dict of physical sides, 'S'/'N' arrays (m_x, n) [strip, a],
         'W'/'E' arrays (m_z, n) [element, b].

Workloads (the paper's problem class, Sec. 4 and Sec. 5: random right-hand
sides from U[0, 1], zero initial guess, relative tolerance 1e-10):
  c1  [0,8]x[0,1], 8x2 elements, n = 11, u* = cos(pi x/8) cos(pi z)
  c2  [0,64]x[0,1], 128x8 elements, n = 17, u* = cos(pi x/64) cos(pi z)
      plus seeded zero-mean Gaussian forcing
  c3  256x16 elements, n = 13, geometric z stretch (ratio 16^(1/15)), seeded
      strip widths, f ~ U[0,1]
  c4  [0,32]x[0,1], 64x8 elements, n = 13, 128 points in y on [0, 8):
      the rfft in y of a seeded U[0,1] field, modes m = 0..64,
      k_m = 2 pi m / 8; each mode has a real and an imaginary right-hand side
  c5  32 seeded problems of uneven size and order (see `c5`)
"""
from dataclasses import dataclass, field

import numpy as np
from numpy.polynomial import legendre as _leg


@dataclass
class Problem:
    """One grid, its wavenumbers, and right-hand sides [mode][rhs][node]."""
    name: str
    xb: np.ndarray
    zb: np.ndarray
    n: int
    kwaves: np.ndarray                 # (nk,)
    f: np.ndarray                      # (nk, nrhs, r)
    g: dict = field(default_factory=dict)   # side -> (nk, nrhs, m, n); empty = zero
    exact: np.ndarray = None           # (r,) manufactured solution, if any

    @property
    def mx(self):
        return len(self.xb) - 1

    @property
    def mz(self):
        return len(self.zb) - 1

    @property
    def r(self):
        return self.n * self.n * self.mx * self.mz

    @property
    def nk(self):
        return len(self.kwaves)

    @property
    def nrhs(self):
        return self.f.shape[1]


def gll_points(n):
    """GLL points on [-1, 1] from numpy's Legendre-series roots."""
    c = np.zeros(n)
    c[-1] = 1.0
    inner = np.sort(np.real(_leg.legroots(_leg.legder(c))))
    return np.concatenate([[-1.0], inner, [1.0]])


def node_coords(xb, zb, n):
    """(x, z) of every node in node order."""
    xi = gll_points(n)
    xb = np.asarray(xb, float)
    zb = np.asarray(zb, float)
    xs = xb[:-1, None] + (xi[None, :] + 1) * 0.5 * np.diff(xb)[:, None]
    zs = zb[:-1, None] + (xi[None, :] + 1) * 0.5 * np.diff(zb)[:, None]
    shape = (len(xb) - 1, len(zb) - 1, n, n)
    X = np.broadcast_to(xs[:, None, None, :], shape).reshape(-1).copy()
    Z = np.broadcast_to(zs[None, :, :, None], shape).reshape(-1).copy()
    return X, Z


def cosine_problem(name, lx, mx, mz, n, noise=0.0, seed=0):
    """u* = cos(pi x / lx) cos(pi z) on [0, lx] x [0, 1]: f = lap u* (+ seeded
    zero-mean N(0,1) noise of amplitude `noise`), g = n . grad u* = 0."""
    xb = np.linspace(0.0, lx, mx + 1)
    zb = np.linspace(0.0, 1.0, mz + 1)
    X, Z = node_coords(xb, zb, n)
    u = np.cos(np.pi * X / lx) * np.cos(np.pi * Z)
    f = -np.pi ** 2 * (1.0 / lx ** 2 + 1.0) * u
    if noise:
        xi = np.random.default_rng(seed).standard_normal(f.shape)
        f = f + noise * (xi - xi.mean())
    return Problem(name, xb, zb, n, np.zeros(1), f[None, None, :], {}, u)


def c1():
    return cosine_problem("c1", 8.0, 8, 2, 11)


def c2(seed=0, mx=128, mz=8, n=17):
    """Long domain [0, mx/2] x [0, 1] (128 x 8 elements at full size)."""
    return cosine_problem("c2", mx / 2.0, mx, mz, n, noise=1.0, seed=seed)


def stretched_grid(mx, mz, seed=0, ratio_total=16.0):
    """Geometric z breakpoints (largest/smallest = ratio_total) and seeded
    strip widths h_x = h_z,max (1 + 0.25 U), U ~ U[0, 1)."""
    q = ratio_total ** (1.0 / max(mz - 1, 1))
    h = q ** np.arange(mz)
    h = h / h.sum()
    zb = np.concatenate([[0.0], np.cumsum(h)])
    zb[-1] = 1.0
    U = np.random.default_rng(seed).uniform(0.0, 1.0, mx)
    hx = h.max() * (1.0 + 0.25 * U)
    xb = np.concatenate([[0.0], np.cumsum(hx)])
    return xb, zb


def c3(seed=0, mx=256, mz=16, n=13, rhs_seed=None):
    """The stretched grid of `seed`; f ~ U[0, 1] from `rhs_seed` (default: the
    grid's seed), so several right-hand sides can share one grid."""
    xb, zb = stretched_grid(mx, mz, seed)
    r = n * n * mx * mz
    f = np.random.default_rng((seed if rhs_seed is None else rhs_seed) + 1).uniform(0.0, 1.0, r)
    return Problem("c3", xb, zb, n, np.zeros(1), f[None, None, :])


def fourier_field(seed, r, my):
    """The seeded U[0, 1] 3-D forcing: [m_y][r], one 2-D node field per y plane."""
    return np.ascontiguousarray(np.random.default_rng(seed).uniform(0.0, 1.0, (r, my)).T)


def fourier_problem(name, lx, mx, mz, n, my, ly, seed=0):
    """rfft in y (normalized by 1/m_y) of the seeded U[0, 1] field on m_y points:
    modes m = 0 .. m_y/2, k_m = 2 pi m / l_y, RHS [Re, Im] per mode."""
    xb = np.linspace(0.0, lx, mx + 1)
    zb = np.linspace(0.0, 1.0, mz + 1)
    r = n * n * mx * mz
    field3 = fourier_field(seed, r, my).T
    fh = np.fft.rfft(field3, axis=1) / my             # (r, my/2 + 1)
    nk = fh.shape[1]
    f = np.empty((nk, 2, r))
    f[:, 0, :] = fh.real.T
    f[:, 1, :] = fh.imag.T
    k = 2.0 * np.pi * np.arange(nk) / ly
    return Problem(name, xb, zb, n, k, f)


def c4(seed=0, mx=64, mz=8, n=13, my=128):
    return fourier_problem("c4", mx / 2.0, mx, mz, n, my, 8.0, seed)


def c5_specs(seed=0, nprob=32):
    """Sizes of the uneven batch: m_x = round(16 * 2^(4U)) in [16, 256],
    m_z uniform in {2..16}, order uniform in {8..16} (n = order + 1),
    k = 0 with probability 1/4 else U(0, 10]."""
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(nprob):
        mx = int(round(16 * 2 ** (4 * rng.uniform())))
        mz = int(rng.integers(2, 17))
        n = int(rng.integers(8, 17)) + 1
        k = 0.0 if rng.uniform() < 0.25 else float(10.0 * (1.0 - rng.uniform()))
        specs.append((mx, mz, n, k))
    return specs


def c5(seed=0, nprob=32, scale=1.0, rhs_seed=None):
    """The uneven batch; `scale` < 1 shrinks m_x and m_z for tests.  The
    sizes come from `seed`, the forcing from `rhs_seed` (default: `seed`)."""
    probs = []
    rng = np.random.default_rng((seed if rhs_seed is None else rhs_seed) + 1000)
    for i, (mx, mz, n, k) in enumerate(c5_specs(seed, nprob)):
        mx = max(4, int(round(mx * scale)))
        mz = max(1, int(round(mz * scale)))
        xb = np.linspace(0.0, 4.0 * mx / mz, mx + 1)
        zb = np.linspace(0.0, 1.0, mz + 1)
        r = n * n * mx * mz
        f = rng.uniform(0.0, 1.0, r)
        probs.append(Problem(f"c5_{i}", xb, zb, n, np.array([k]), f[None, None, :]))
    return probs


def smooth_field(xb, zb, n, seed):
    """A smooth seeded node field: low Fourier modes in x and z,
    sum_{kx < 4, kz < 3} a_{kx,kz} cos(pi kx x / L_x) cos(pi kz z), a ~ N(0, 1)."""
    X, Z = node_coords(xb, zb, n)
    lx = xb[-1] - xb[0]
    rng = np.random.default_rng(seed)
    v = np.zeros_like(X)
    for kx in range(4):
        for kz in range(3):
            v += rng.standard_normal() * np.cos(np.pi * kx * X / lx) * np.cos(np.pi * kz * Z)
    return v


def random_problem(mx, mz, n, kwaves=(0.0,), nrhs=1, seed=0, lx=None, stretch=False,
                   with_g=False):
    """Small random problems for tests: U[0,1] forcing, optional Neumann data."""
    if stretch:
        xb, zb = stretched_grid(mx, mz, seed, ratio_total=4.0)
    else:
        xb = np.linspace(0.0, lx if lx else mx / 2.0, mx + 1)
        zb = np.linspace(0.0, 1.0, mz + 1)
    rng = np.random.default_rng(seed)
    r = n * n * mx * mz
    kw = np.asarray(kwaves, float)
    f = rng.uniform(0.0, 1.0, (len(kw), nrhs, r))
    g = {}
    if with_g:
        g = {"S": rng.standard_normal((len(kw), nrhs, mx, n)),
             "N": rng.standard_normal((len(kw), nrhs, mx, n)),
             "W": rng.standard_normal((len(kw), nrhs, mz, n)),
             "E": rng.standard_normal((len(kw), nrhs, mz, n))}
    return Problem(f"rand_{mx}x{mz}_n{n}", xb, zb, n, kw, f, g)
