"""Pins of the oracle's Householder GMRES (Sec. 3.1)."""
import numpy as np

from oracle import gmres


def test_full_krylov_space_solves_exactly():
    rng = np.random.default_rng(0)
    n = 30
    A = rng.standard_normal((n, n)) + 5 * np.eye(n)
    b = rng.standard_normal(n)
    x, it, ok, hist = gmres.gmres(lambda v: A @ v, b, tol=1e-14, maxit=n)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    assert ok and it <= n


def test_identity_converges_in_one_step():
    b = np.arange(1.0, 6.0)
    x, it, ok, _ = gmres.gmres(lambda v: v, b, tol=1e-12)
    assert it == 1 and ok
    np.testing.assert_allclose(x, b)


def test_zero_rhs():
    x, it, ok, _ = gmres.gmres(lambda v: 2 * v, np.zeros(4))
    assert it == 0 and ok and np.all(x == 0)


def test_recursive_residual_equals_true_residual_and_minimality():
    rng = np.random.default_rng(1)
    n = 60
    A = np.diag(np.linspace(1, 3, n)) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    for m in (3, 8, 15):
        x, it, ok, hist = gmres.gmres(lambda v: A @ v, b, tol=0.0, maxit=m)
        true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        assert abs(true - hist[-1]) < 1e-12
        # GMRES minimizes the residual over the Krylov space: compare with a
        # least-squares solve on an explicit (QR-orthonormalized) basis.
        K = np.empty((n, m)); v = b.copy()
        for i in range(m):
            K[:, i] = v; v = A @ v
        Qk, _ = np.linalg.qr(K)
        y = np.linalg.lstsq(A @ Qk, b, rcond=None)[0]
        best = np.linalg.norm(b - A @ Qk @ y) / np.linalg.norm(b)
        assert abs(true - best) < 1e-9


def test_singular_consistent_system():
    # Sec. 3.1: GMRES converges on singular systems with N(S) and R(S)
    # complementary when the right-hand side is consistent.
    rng = np.random.default_rng(2)
    n = 20
    M = rng.standard_normal((n, n)) + 4 * np.eye(n)
    u = np.ones(n) / np.sqrt(n)
    S = M - np.outer(M @ u, u)           # S u = 0
    b = S @ rng.standard_normal(n)       # consistent
    x, it, ok, _ = gmres.gmres(lambda v: S @ v, b, tol=1e-12)
    assert ok
    assert np.linalg.norm(S @ x - b) < 1e-10 * np.linalg.norm(b)
