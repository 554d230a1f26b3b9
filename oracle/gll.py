"""Gauss-Lobatto-Legendre (GLL) grid and spectral differentiation (oracle).

Test infrastructure: see the package docstring.

Paper Sec. 2.2: each element carries an n x n GLL grid, functions are held as
nodal values of the Lagrange interpolant and derivatives are taken with the
spectral differentiation matrix built from that basis (Costa & Don).  Here n
is the number of GLL points per direction; the polynomial degree is n - 1.
"""
import numpy as np


def legendre(N, x):
    """Legendre polynomial P_N and P_{N-1} at x by the three-term recurrence
    (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if N == 0:
        return p_prev, np.zeros_like(x)
    p = x.copy()
    for k in range(1, N):
        p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
    return p, p_prev


def gll_nodes(n):
    """The n GLL nodes on [-1, 1]: the end points and the roots of P'_{n-1}.

    The interior nodes are the roots of q = P_{N+1} - P_{N-1} (N = n - 1),
    which is proportional to (1 - x^2) P'_N; q' = (2N + 1) P_N.  Newton's
    method from the Chebyshev-Lobatto points converges to each root.
    """
    if n < 2:
        raise ValueError("need at least two GLL points")
    N = n - 1
    x = -np.cos(np.pi * np.arange(n) / N)
    for _ in range(100):
        pN1, pN = legendre(N + 1, x)          # P_{N+1}, P_N
        _, pNm1 = legendre(N, x)               # P_{N-1}
        q = pN1 - pNm1
        dq = (2 * N + 1) * pN
        step = np.zeros_like(x)
        step[1:-1] = q[1:-1] / dq[1:-1]
        x = x - step
        if np.max(np.abs(step)) < 1e-16:
            break
    x[0], x[-1] = -1.0, 1.0
    return x


def gll_weights(x):
    """GLL quadrature weights w_i = 2 / (N (N+1) P_N(x_i)^2)."""
    N = len(x) - 1
    pN, _ = legendre(N, x)
    return 2.0 / (N * (N + 1) * pN ** 2)


def diff_matrix(x):
    """Spectral differentiation matrix of the Lagrange basis on GLL nodes.

    Off-diagonal: D_ij = P_N(x_i) / (P_N(x_j) (x_i - x_j)).  Diagonal: the
    negative row sum, so that D annihilates constants to rounding (the
    accuracy fix of Costa & Don cited in Sec. 2.2).
    """
    n = len(x)
    N = n - 1
    pN, _ = legendre(N, x)
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = pN[i] / (pN[j] * (x[i] - x[j]))
    for i in range(n):
        D[i, i] = -np.sum(D[i, :])
    return D
