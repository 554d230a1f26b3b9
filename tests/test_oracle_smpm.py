"""Pins of the oracle's SMPM operator and strip split (Sec. 2.2-2.4)."""
import numpy as np
import pytest

from oracle import smpm, solve
from paper_1512_01756_amd import workloads


def _grid(mx=4, mz=2, n=5, lx=None):
    lx = lx if lx else mx / 2.0
    return smpm.Grid(np.linspace(0, lx, mx + 1), np.linspace(0, 1, mz + 1), n)


@pytest.mark.parametrize("tau", [-40.0, -3.0, 7.5])
def test_constant_in_right_null_space_any_tau(tau):
    # Every penalty term annihilates constants and D 1 = 0 (Sec. 2.2).
    grid = _grid(4, 3, 5)
    L = smpm.assemble_L(grid, tau)
    assert np.max(np.abs(L @ np.ones(grid.r))) < 1e-11 * abs(L).max()


def test_split_L_equals_A_plus_EB():
    # Sec. 2.3: L = A + E B, E^T E = I, A block diagonal over strips.
    grid = smpm.Grid([0.0, 0.3, 1.0, 1.2, 2.0], [0.0, 0.4, 1.0], 5)
    tau = smpm.default_tau(grid)
    L = smpm.assemble_L(grid, tau)
    A = smpm.assemble_A(grid, tau)
    B = smpm.assemble_B(grid, tau)
    E = smpm.assemble_E(grid)
    assert abs(L - A - E @ B).max() < 1e-12 * abs(L).max()
    ETE = (E.T @ E).toarray()
    np.testing.assert_array_equal(ETE, np.eye(grid.k))
    m = grid.n ** 2 * grid.mz
    Ad = A.toarray()
    for j in range(grid.mx):
        blk = np.zeros_like(Ad, dtype=bool)
        blk[j * m:(j + 1) * m, j * m:(j + 1) * m] = True
        off = Ad.copy(); off[blk] = 0
        assert np.all(off[j * m:(j + 1) * m, :] == 0)
    # B reads only the strips facing each interface.
    Bd = B.toarray()
    for h in range(2 * (grid.mx - 1)):
        i = h // 2
        facing = i + 1 if h % 2 == 0 else i
        rows = Bd[h * grid.nhalf:(h + 1) * grid.nhalf]
        nz = np.nonzero(np.any(rows != 0, axis=0))[0]
        assert np.all(nz // m == facing)


def test_null_space_is_one_dimensional():
    grid = _grid(4, 2, 5)
    L = smpm.assemble_L(grid, smpm.default_tau(grid)).toarray()
    s = np.linalg.svd(L, compute_uv=False)
    assert s[-1] < 1e-10 * s[0]
    assert s[-2] > 1e-6 * s[0]


def test_helmholtz_shift_is_nonsingular():
    grid = _grid(4, 2, 5)
    tau = smpm.default_tau(grid)
    for k in (0.5, 3.0, 12.0):
        L = smpm.assemble_L(grid, tau, k).toarray()
        s = np.linalg.svd(L, compute_uv=False)
        assert s[-1] > 1e-8 * s[0]
        np.testing.assert_allclose(L, smpm.assemble_L(grid, tau).toarray() - k * k * np.eye(grid.r))


def _manufactured_error(n):
    p = workloads.cosine_problem("m", 8.0, 8, 2, n)
    grid = smpm.Grid(p.xb, p.zb, n)
    tau = smpm.default_tau(grid)
    F = smpm.rhs(grid, tau, p.f[0, 0])
    u = solve.direct_solve(grid, tau, F)
    ue = p.exact - p.exact.mean()
    L = smpm.assemble_L(grid, tau)
    trunc = np.linalg.norm(L @ p.exact - F) / np.linalg.norm(F)
    return np.max(np.abs(u - ue)), trunc


def test_manufactured_solution_spectral_convergence():
    # u* = cos(pi x/8) cos(pi z) with g = 0: error and truncation error decay
    # faster than any power of n (log-error linear in n).
    ns = [3, 5, 7, 9, 11]
    errs, truncs = zip(*[_manufactured_error(n) for n in ns])
    errs = np.array(errs)
    assert np.all(np.diff(np.log(errs)) < -1.5)
    assert errs[-1] < 1e-9
    truncs = np.array(truncs)
    assert truncs[-1] < 1e-8 and truncs[0] > 1e-1
    assert np.all(np.diff(np.log(truncs)) < -2.0)
    slopes = np.diff(np.log(errs)) / np.diff(ns)
    # spectral, not algebraic: the decay rate does not flatten with n
    assert slopes[-1] < -2.0


def test_grid_coordinates_match_generator():
    p = workloads.c1()
    grid = smpm.Grid(p.xb, p.zb, p.n)
    X, Z = grid.coords()
    Xw, Zw = workloads.node_coords(p.xb, p.zb, p.n)
    np.testing.assert_allclose(X, Xw, atol=1e-14)
    np.testing.assert_allclose(Z, Zw, atol=1e-14)


def test_z_constant_fields_see_only_the_x_operator():
    # For a field that is constant in z, the z-Laplacian vanishes (D 1 = 0)
    # and every z-edge penalty term cancels, so L v is z-constant and equals
    # the result of the one-element-high (m_z = 1) operator.
    xb = np.array([0.0, 0.7, 1.5, 2.0, 3.1])
    n = 6
    out = []
    for mz, zb in ((1, [0.0, 1.0]), (3, [0.0, 0.2, 0.65, 1.0])):
        grid = smpm.Grid(xb, zb, n)
        tau = -30.0
        X, Z = grid.coords()
        v = np.cos(np.pi * X / 4) + 0.3 * np.sin(2 * X) + X ** 3 / 10
        Lv = (smpm.assemble_L(grid, tau) @ v).reshape(grid.mx, grid.mz, n, n)
        assert np.max(np.abs(Lv - Lv[:, :1, :1, :])) < 1e-9 * np.abs(Lv).max()
        out.append(Lv[:, 0, 0, :])
    np.testing.assert_allclose(out[0], out[1], atol=1e-9 * np.abs(out[0]).max())


def test_compatibility_defect_separates_compatible_data():
    # Sec. 2.4: the projection removes the component of F along u_L.  For
    # data with int f = oint g that component is at rounding/truncation level;
    # shifting f by a constant (int f != oint g) makes it O(1).
    defects = []
    for n in (4, 6, 8):
        p = workloads.cosine_problem("m", 8.0, 8, 2, n)
        grid = smpm.Grid(p.xb, p.zb, n)
        tau = smpm.default_tau(grid)
        F = smpm.rhs(grid, tau, p.f[0, 0] + 0.25)   # shift: int f != 0 -> incompatible
        L = smpm.assemble_L(grid, tau).toarray()
        uL = np.linalg.svd(L)[0][:, -1]
        defects.append(abs(uL @ F) / np.linalg.norm(F))
        F0 = smpm.rhs(grid, tau, p.f[0, 0])
        assert abs(uL @ F0) / np.linalg.norm(F0) < 1e-3 * defects[-1]
    assert min(defects) > 1e-3


def test_rhs_corner_gets_both_sides():
    grid = _grid(2, 1, 3)
    tau = -2.0
    g = {"S": np.ones((2, 3)), "W": 10 * np.ones((1, 3))}
    F = smpm.rhs(grid, tau, np.zeros(grid.r), g)
    assert F[grid.node(0, 0, 0, 0)] == tau * 11
    assert F[grid.node(0, 0, 0, 1)] == tau * 1
    assert F[grid.node(0, 0, 1, 0)] == tau * 10
    assert F[grid.node(1, 0, 1, 1)] == 0.0


# A manufactured solution with Neumann data on all four sides of a grid
# stretched in x and z (Sec. 2.2, Eq. smpm_poisson): on such a grid the
# physical-boundary term tau n.grad u, the data term tau g (corners take both
# sides) and the neighbour-size factors 2/h of R_ij u_j are all active, and a
# wrong normal, sign or element size leaves an O(1) error.
_XB = np.array([0.0, 0.35, 0.9, 1.2, 1.95, 2.4])
_ZB = np.array([0.0, 0.1, 0.35, 1.0])


def _mms(X, Z):
    """u = sin(0.7x) cosh(0.5z) + 0.3 x^2 z, its Laplacian and gradient."""
    s, c = np.sin(0.7 * X), np.cos(0.7 * X)
    u = s * np.cosh(0.5 * Z) + 0.3 * X ** 2 * Z
    lap = -0.24 * s * np.cosh(0.5 * Z) + 0.6 * Z
    ux = 0.7 * c * np.cosh(0.5 * Z) + 0.6 * X * Z
    uz = 0.5 * s * np.sinh(0.5 * Z) + 0.3 * X ** 2
    return u, lap, ux, uz


def _mms_problem(n, k=0.0):
    """Grid, tau, F = f + tau g with f = (lap - k^2) u and g = n.grad u on
    each physical side, and the exact nodal solution."""
    grid = smpm.Grid(_XB, _ZB, n)
    tau = smpm.default_tau(grid)
    X, Z = grid.coords()
    u, lap, _, _ = _mms(X, Z)
    xi = np.polynomial.legendre.Legendre.basis(n - 1).deriv().roots()
    xi = np.concatenate(([-1.0], xi, [1.0]))
    xs = _XB[:-1, None] + (xi[None, :] + 1) * 0.5 * np.diff(_XB)[:, None]   # (m_x, n)
    zs = _ZB[:-1, None] + (xi[None, :] + 1) * 0.5 * np.diff(_ZB)[:, None]   # (m_z, n)
    g = {"S": -_mms(xs, _ZB[0])[3], "N": _mms(xs, _ZB[-1])[3],
         "W": -_mms(_XB[0], zs)[2], "E": _mms(_XB[-1], zs)[2]}
    F = smpm.rhs(grid, tau, lap - k * k * u, g)
    return grid, tau, F, u


@pytest.mark.parametrize("k", [0.0, 2.5])
def test_manufactured_neumann_data_on_stretched_grid(k):
    # Error relative to max|u|; for k = 0 both sides carry the zero-mean gauge.
    errs = []
    for n in (4, 6, 8, 10):
        grid, tau, F, u = _mms_problem(n, k)
        ue = u - u.mean() if k == 0.0 else u
        uh = solve.direct_solve(grid, tau, F, k)
        errs.append(np.max(np.abs(uh - ue)) / np.max(np.abs(ue)))
    errs = np.array(errs)
    assert errs[0] > 1e-5                       # the coarse grid is visibly off
    assert np.all(np.diff(np.log10(errs)) < -1.3)
    assert errs[-1] < 1e-10


def test_schur_route_on_stretched_grid_with_neumann_data():
    # Algorithm 2 on the same data reaches the manufactured solution too.
    from oracle import schur
    for k in (0.0, 2.5):
        grid, tau, F, u = _mms_problem(10, k)
        ue = u - u.mean() if k == 0.0 else u
        res = solve.dbj_solve(schur.build(grid, tau, k), F)
        assert res.converged
        assert np.max(np.abs(res.u - ue)) / np.max(np.abs(ue)) < 1e-10
