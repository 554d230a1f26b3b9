"""Pins of the oracle's Algorithm 2 solve against the plain definitions."""
import numpy as np
import pytest

from oracle import schur, smpm, solve
from paper_1512_01756_amd import workloads


def _setup(p, k=None):
    grid = smpm.Grid(p.xb, p.zb, p.n)
    kw = p.kwaves[0] if k is None else k
    return grid, schur.build(grid, kwave=kw)


def test_c1_manufactured_matches_direct_and_exact():
    p = workloads.c1()
    grid, s = _setup(p)
    F = smpm.rhs(grid, s.tau, p.f[0, 0])
    r = solve.dbj_solve(s, F)
    ud = solve.direct_solve(grid, s.tau, F)
    assert r.converged and r.schur_relres <= 1e-10
    assert np.max(np.abs(r.u - ud)) < 1e-10 * np.max(np.abs(ud))
    ue = p.exact - p.exact.mean()
    assert np.max(np.abs(r.u - ue)) < 1e-9


@pytest.mark.parametrize("method", ["schur", "bj", "dbj", "2las"])
def test_table1_methods_reach_the_direct_solution(method):
    p = workloads.random_problem(6, 2, 5, seed=4, with_g=True)
    grid, s = _setup(p)
    g = {side: arr[0, 0] for side, arr in p.g.items()}
    F = smpm.rhs(grid, s.tau, p.f[0, 0], g)
    r = solve.dbj_solve(s, F, method=method, tol=1e-12)
    ud = solve.direct_solve(grid, s.tau, F)
    assert r.converged
    # both solve L u = F~ exactly up to rounding amplified by cond(L) ~ 1e5
    assert np.max(np.abs(r.u - ud)) < 1e-8 * np.max(np.abs(ud))


def test_dense_schur_direct_solve_agrees():
    p = workloads.random_problem(4, 2, 4, seed=1)
    grid, s = _setup(p)
    F = smpm.rhs(grid, s.tau, p.f[0, 0])
    u1, xs = solve.dense_schur_solve(grid, s.tau, F)
    u0 = solve.direct_solve(grid, s.tau, F)
    r = solve.dbj_solve(s, F, tol=1e-13)
    np.testing.assert_allclose(u1, u0, atol=1e-9 * np.abs(u0).max())
    np.testing.assert_allclose(r.u, u1, atol=1e-9 * np.abs(u0).max())
    # x_S is unique modulo the interface constant
    d = (r.xS - xs)
    assert np.max(np.abs(d - d.mean())) < 1e-8 * np.abs(xs).max()


@pytest.mark.parametrize("k", [0.7, 4.0])
def test_helmholtz_mode_matches_direct(k):
    p = workloads.random_problem(6, 2, 5, kwaves=(k,), seed=2)
    grid, s = _setup(p)
    F = smpm.rhs(grid, s.tau, p.f[0, 0])
    r = solve.dbj_solve(s, F, tol=1e-12)
    ud = solve.direct_solve(grid, s.tau, F, kwave=k)
    assert r.converged
    np.testing.assert_allclose(r.u, ud, atol=1e-9 * np.abs(ud).max())


def test_iteration_ordering_matches_paper_shape():
    # Table 2 shape: DBJ < BJ < unpreconditioned, and 2LAS needs more than DBJ.
    p = workloads.random_problem(16, 2, 5, seed=0)
    grid, s = _setup(p)
    F = smpm.rhs(grid, s.tau, p.f[0, 0])
    its = {m: solve.dbj_solve(s, F, method=m).iters for m in ("schur", "bj", "dbj", "2las")}
    assert its["dbj"] < its["bj"] < its["schur"]
    assert its["2las"] > its["dbj"]


def test_refinement_emulation_reaches_fp64_solution():
    p = workloads.random_problem(8, 2, 6, seed=3)
    grid, s = _setup(p)
    F = smpm.rhs(grid, s.tau, p.f[0, 0])
    ref = solve.dbj_solve(s, F, tol=1e-13)
    r, sweeps, inner = solve.refine_solve(s, F)
    assert r.converged and sweeps >= 1
    assert np.max(np.abs(r.u - ref.u)) < 1e-8 * np.abs(ref.u).max()
