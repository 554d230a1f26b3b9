"""Pins of the oracle's Schur complement, block-Jacobi, deflation and null
vectors (Sec. 2.3-3.3, Claims 1 and 2)."""
import numpy as np
import pytest

from oracle import schur, smpm, solve


def _sys(mx=5, mz=2, n=5, k=0.0, stretch=False, zlabel=0):
    if stretch:
        xb = np.array([0.0, 0.4, 0.9, 1.2, 1.9, 2.3, 2.8][:mx + 1])
        zb = np.array([0.0, 0.15, 0.45, 1.0][:mz + 1])
        zb[-1] = 1.0
    else:
        xb = np.linspace(0, mx / 2.0, mx + 1)
        zb = np.linspace(0, 1, mz + 1)
    grid = smpm.Grid(xb, zb, n)
    return schur.build(grid, kwave=k, zlabel=zlabel)


@pytest.mark.parametrize("k", [0.0, 2.5])
@pytest.mark.parametrize("stretch", [False, True])
def test_block_schur_equals_dense_definition(k, stretch):
    s = _sys(5, 2, 5, k, stretch)
    Sd = schur.dense_schur(s.grid, s.tau, k)
    assert np.max(np.abs(s.S.toarray() - Sd)) < 1e-12 * np.max(np.abs(Sd))
    # and W_j blocks are exactly the nonzero pattern implied by the strip coupling
    nnz_dense = np.count_nonzero(np.abs(Sd - np.eye(s.grid.k)) > 1e-14 * np.abs(Sd).max())
    assert nnz_dense <= s.S.nnz


def test_schur_annihilates_interface_constant():
    for stretch in (False, True):
        s = _sys(6, 3, 6, 0.0, stretch)
        S = s.S
        assert np.max(np.abs(S @ np.ones(s.grid.k))) < 1e-11 * abs(S).max()


def test_schur_rank_and_left_null_vector():
    s = _sys(5, 2, 5)
    Sd = s.S.toarray()
    sv = np.linalg.svd(Sd, compute_uv=False)
    assert sv[-1] < 1e-11 * sv[0] and sv[-2] > 1e-7 * sv[0]
    assert np.linalg.norm(s.uS @ Sd) < 1e-11 * np.linalg.norm(Sd)
    L = smpm.assemble_L(s.grid, s.tau)
    assert np.linalg.norm(L.T @ s.uL) < 1e-10 * abs(L).max()
    # u_S^T 1 != 0 (Sec. 3.1: proper principal submatrices of S invertible)
    assert abs(s.uS.sum()) > 0.1


def test_left_null_vector_on_a_long_grid():
    # A 24 x 4 grid of order 6 (12:1), where the slow modes make the null
    # space hard to resolve: u_S must match the left singular vector of the
    # smallest singular value of the dense S (a library route), and leave a
    # residual at the rounding of S itself.  (Pinning one component and
    # dropping one equation instead leaves 5.6e-13 here.)
    s = _sys(24, 4, 7)
    Sd = s.S.toarray()
    U, sv, Vt = np.linalg.svd(Sd)
    u_svd = U[:, -1] * np.sign(U[:, -1].sum())
    assert 1 - abs(u_svd @ s.uS) < 1e-12
    assert np.linalg.norm(s.uS @ Sd) < 1e-13 * np.abs(Sd).sum(axis=0).max()


def test_claim1_relations():
    # Claim 1: u_S = E^T u_L and u_L = A^-T B^T u_S, up to scale.
    s = _sys(5, 3, 5, stretch=True)
    v = s.E.T @ s.uL
    assert 1 - abs(v @ s.uS) / np.linalg.norm(v) < 1e-12
    L = smpm.assemble_L(s.grid, s.tau).toarray()
    U, sv, Vt = np.linalg.svd(L)
    uL_svd = U[:, -1] * np.sign(U[:, -1].sum())
    assert 1 - abs(uL_svd @ s.uL) < 1e-10


def test_claim2_bound_on_perturbed_solutions():
    s = _sys(5, 2, 5)
    rng = np.random.default_rng(3)
    F = smpm.rhs(s.grid, s.tau, rng.uniform(0, 1, s.grid.r))
    Ft, bS, _ = solve.schur_rhs(s, F)
    L = smpm.assemble_L(s.grid, s.tau)
    proj_b = bS - s.uS * (s.uS @ bS)
    for scale in (1e-6, 1e-3, 1.0):
        x = rng.standard_normal(s.grid.k) * scale
        u = s.A_solve(Ft - s.E @ x)
        lhs = np.linalg.norm(L @ u - Ft)
        rhs = np.linalg.norm(s.S @ x - proj_b)
        assert lhs <= rhs * (1 + 1e-9) + 1e-12 * np.linalg.norm(Ft)


@pytest.mark.parametrize("k", [0.0, 1.7])
@pytest.mark.parametrize("zlabel", [0, 1])
def test_deflation_identities(k, zlabel):
    s = _sys(7, 2, 5, k, zlabel=zlabel)
    rng = np.random.default_rng(1)
    Sd = s.S.toarray()
    for _ in range(3):
        y = rng.standard_normal(s.grid.k)
        Py = s.P_apply(y)
        np.testing.assert_allclose(s.P_apply(Py), Py, atol=1e-10 * np.linalg.norm(y))
        Qy = s.Q_apply(y)
        np.testing.assert_allclose(s.Q_apply(Qy), Qy, atol=1e-10 * np.linalg.norm(y))
        np.testing.assert_allclose(Sd @ s.Q_apply(y), s.P_apply(Sd @ y),
                                   atol=1e-10 * np.linalg.norm(Sd @ y))
        ZtP = s.Zt(Py)
        expect = s.uC * (s.uC @ s.Zt(y)) if k == 0.0 else np.zeros_like(ZtP)
        np.testing.assert_allclose(ZtP, expect, atol=1e-10 * np.linalg.norm(y))
    d = s.C.shape[0]
    for c in range(d):
        e = np.zeros(d); e[c] = 1
        np.testing.assert_allclose(s.P_apply(s.SZ @ e), 0, atol=1e-10 * np.linalg.norm(s.SZ @ e))


@pytest.mark.parametrize("k", [0.0, 1.3])
def test_per_element_deflation_space(k):
    # Z with one column per element segment of an interface: d = (m_x - 1) m_z
    # columns of 2n ones each; C couples only neighbouring interfaces (block
    # tridiagonal with m_z x m_z blocks); the per-interface space is the sum of
    # the segment columns, so it is deflated too: P_el S Z_if = 0.
    mx, mz, n = 6, 3, 4
    s1 = _sys(mx, mz, n, k, stretch=True, zlabel=1)
    s0 = _sys(mx, mz, n, k, stretch=True, zlabel=0)
    d = (mx - 1) * mz
    assert s1.C.shape == (d, d)
    assert np.all(np.bincount(s1.labels, minlength=d) == 2 * n)
    C = s1.C
    for a in range(mx - 1):
        for b in range(mx - 1):
            if abs(a - b) > 1:
                assert np.abs(C[a * mz:(a + 1) * mz, b * mz:(b + 1) * mz]).max() < 1e-12 * np.abs(C).max()
    if k == 0.0:
        assert np.abs(C @ np.ones(d)).max() < 1e-10 * np.abs(C).max()
        assert np.sum(np.linalg.svd(C, compute_uv=False) < 1e-10 * np.abs(C).max()) == 1
    for c in range(mx - 1):
        e = np.zeros(mx - 1); e[c] = 1
        v = s0.SZ @ e
        np.testing.assert_allclose(s1.P_apply(v), 0, atol=1e-10 * np.linalg.norm(v))


def test_per_element_deflation_solves_the_same_problem():
    xb = np.array([0.0, 0.4, 0.9, 1.2, 1.9, 2.3, 2.8])
    zb = np.array([0.0, 0.3, 1.0])
    grid = smpm.Grid(xb, zb, 5)
    F = np.random.default_rng(2).uniform(0, 1, grid.r)
    s1 = schur.build(grid, zlabel=1)
    r1 = solve.dbj_solve(s1, smpm.rhs(grid, s1.tau, F))
    ud = solve.direct_solve(grid, s1.tau, smpm.rhs(grid, s1.tau, F))
    assert r1.converged
    assert np.abs(r1.u - ud).max() <= 1e-9 * np.abs(ud).max()


def test_coarse_matrix_structure():
    s = _sys(7, 2, 5)
    C = s.C
    d = s.grid.mx - 1
    assert C.shape == (d, d)
    assert np.all(np.abs(np.triu(C, 2)) < 1e-12 * np.abs(C).max())     # tridiagonal (Sec. 3.3)
    assert np.all(np.abs(np.tril(C, -2)) < 1e-12 * np.abs(C).max())
    assert np.max(np.abs(C @ np.ones(d))) < 1e-10 * np.abs(C).max()     # singular, C 1 = 0
    assert np.linalg.norm(s.uC @ C) < 1e-10 * np.linalg.norm(C)
    # Gauge invariance: P does not change when the coarse solution moves along 1_d.
    y = np.random.default_rng(0).standard_normal(s.grid.k)
    t = s.coarse(s.Zt(y))
    np.testing.assert_allclose(y - s.SZ @ (t + 3.0), s.P_apply(y), atol=1e-9 * np.linalg.norm(y))


def test_block_jacobi_blocks():
    # Sec. 3.2: blocks over two interfaces (4 n m_z); the last one is a single
    # interface when m_x - 1 is odd (m_x even).
    s = _sys(6, 2, 5)
    N = s.grid.nhalf
    sizes = [len(i) for i in s.bj_index]
    assert sizes == [4 * N, 4 * N, 2 * N]
    Sd = s.S.toarray()
    rng = np.random.default_rng(0)
    for idx, Mi in zip(s.bj_index, s.bj_inv):
        Mb = Sd[np.ix_(idx, idx)]
        v = rng.standard_normal(len(idx))
        np.testing.assert_allclose(Mi @ (Mb @ v), v, atol=1e-9)
    assert [len(i) for i in _sys(5, 2, 5).bj_index] == [4 * N, 4 * N]


def test_paper_coarse_null_vector_gap_is_reported():
    # Sec. 3.3 takes u_C = Z^T u_S; the oracle uses the computed left null
    # vector of C.  Both annihilate C here to rounding level.
    s = _sys(7, 3, 5, stretch=True)
    v = s.Zt(s.uS); v /= np.linalg.norm(v)
    gap = np.linalg.norm(v @ s.C) / np.linalg.norm(s.C)
    assert np.linalg.norm(s.uC @ s.C) / np.linalg.norm(s.C) < 1e-12
    assert gap < 1e-6


def test_banded_left_null_route_on_a_long_grid(monkeypatch):
    # The route taken above BORDERED_MAX_K unknowns (a banded LU of S^T with
    # one diagonal entry raised), forced on the same 12:1 grid: the same
    # left singular vector of the dense S, and a residual at the rounding of
    # S.  Also with the first pivot entry placed where u_S is smallest.
    from oracle import schur as sch
    s = _sys(24, 4, 7)
    Sd = s.S.toarray()
    U, sv, Vt = np.linalg.svd(Sd)
    u_svd = U[:, -1] * np.sign(U[:, -1].sum())
    v = sch._left_null_banded(s.S, s.grid.nhalf)
    v = v / np.linalg.norm(v) * np.sign(v.sum())
    assert 1 - abs(u_svd @ v) < 1e-12
    assert np.linalg.norm(v @ Sd) < 1e-13 * np.abs(Sd).sum(axis=0).max()
    monkeypatch.setattr(sch, "BORDERED_MAX_K", 0)
    uS, _, _ = sch.null_vectors(s)
    assert np.abs(uS - s.uS).max() < 1e-12
