"""GMRES with Householder Arnoldi (oracle).

Test infrastructure: see the package docstring.

Sec. 3.1: the Krylov solver is GMRES, and its Arnoldi process orthogonalizes
with Householder reflections (Walker 1988), whose loss of orthogonality is
O(eps) instead of O(eps kappa) for modified Gram-Schmidt.  Zero initial guess
and a relative tolerance on the residual (Sec. 4).  No restart.

Steps (Householder Arnoldi as in Saad, Iterative Methods, Alg. 6.10, then the
usual Givens QR of the Hessenberg matrix):
  z_0 = b.  For j = 0, 1, ...:
    choose the reflector P_j = I - 2 w_j w_j^T (w_j zero above index j) that
    zeroes entries j+1.. of z_j; column j-1 of H is the head of P_j z_j;
    v_j = P_0 P_1 ... P_j e_j;  z_{j+1} = P_j ... P_0 (Op v_j).
  Residual norm |g_{j+1}| after the Givens rotations; stop when it is below
  tol times a reference norm (|b| unless the caller passes one).  x = P_0 ... P_{m-1} [y; 0] with R y = g.
"""
import numpy as np


def _house(z, p):
    """Reflector zeroing z[p+1:]; returns (w, alpha) with (I - 2 w w^T) z
    having alpha at p.  w is None when z[p:] is already zero."""
    tail = z[p:]
    sigma = np.linalg.norm(tail)
    if sigma == 0.0:
        return None, 0.0
    alpha = -sigma if tail[0] >= 0 else sigma
    u = tail.copy()
    u[0] -= alpha
    un = np.linalg.norm(u)
    if un == 0.0:
        return None, tail[0]
    w = np.zeros_like(z)
    w[p:] = u / un
    return w, alpha


def _reflect(w, x):
    if w is None:
        return x
    return x - 2.0 * w * (w @ x)


def gmres(op, b, tol=1e-10, maxit=300, ref_norm=None):
    """Solve op(x) = b from x0 = 0; stop when the residual estimate |g_{j+1}|
    is at most tol * ref_norm (default |b|).  Returns (x, iterations,
    converged, residual history |g_j| / |b|)."""
    k = b.shape[0]
    maxit = min(maxit, k)
    Ws = []
    w, beta = _house(b.astype(np.float64), 0)
    Ws.append(w)
    r0 = abs(beta)
    target = tol * (r0 if ref_norm is None else ref_norm)
    hist = [1.0]
    if r0 == 0.0:
        return np.zeros_like(b), 0, True, hist
    H = np.zeros((maxit + 1, maxit))
    g = np.zeros(maxit + 1)
    g[0] = beta
    cs = np.zeros(maxit)
    sn = np.zeros(maxit)
    m = 0
    converged = False
    for j in range(maxit):
        v = np.zeros(k); v[j] = 1.0
        for i in range(j, -1, -1):
            v = _reflect(Ws[i], v)
        z = op(v)
        for i in range(j + 1):
            z = _reflect(Ws[i], z)
        if j + 1 < k:
            w, alpha = _house(z, j + 1)
            Ws.append(w)
            z[j + 1] = alpha
            z[j + 2:] = 0.0
        h = np.zeros(j + 2)
        h[:min(j + 2, k)] = z[:j + 2]
        for i in range(j):
            t = cs[i] * h[i] + sn[i] * h[i + 1]
            h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1]
            h[i] = t
        den = np.hypot(h[j], h[j + 1])
        cs[j] = h[j] / den if den != 0.0 else 1.0
        sn[j] = h[j + 1] / den if den != 0.0 else 0.0
        h[j] = den
        h[j + 1] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        H[:j + 2, j] = h
        m = j + 1
        hist.append(abs(g[j + 1]) / r0)
        if abs(g[j + 1]) <= target:
            converged = True
            break
    R = H[:m, :m]
    y = np.linalg.solve(np.triu(R), g[:m]) if m > 0 else np.zeros(0)
    x = np.zeros(k)
    x[:m] = y
    for i in range(m - 1, -1, -1):
        x = _reflect(Ws[i], x)
    return x, m, converged, hist
