"""Schur-method solves (oracle).

Test infrastructure: see the package docstring.

dbj_solve is the paper's block-Jacobi preconditioned and deflated Schur
method (Alg. 2, Sec. 3.3).  schur_rhs removes the component of the right-hand
side along the left null vector of L (Sec. 2.4, Eq. regularize_poisson), maps
it to the interface through A^-1 and B, and removes the component along the
left null vector of S (Eq. regularize_schur).  schur_solve runs GMRES from a
zero guess on the deflated, right-preconditioned operator P S M^-1
(Eq. deflated_schur), maps the Krylov solution back through M^-1 and Q, and
adds the coarse part Z C^+ (I - u_C u_C^T) Z^T b_S.  recover eliminates the
interior, u = A^-1 (F - E x_S).

The Poisson (k = 0) solution is defined up to a constant (Sec. 2.4); it is
returned with zero nodal mean.  For a Helmholtz mode k > 0 (Sec. 5) the two
null-space projections and the coarse projection I - u_C u_C^T are skipped:
L - k^2 I and C(k) are nonsingular.

The comparison methods of Table 1 (Sec. 4) are selectable with `method`:
'schur' GMRES(S, b_S); 'bj' GMRES(S M^-1, b_S) then M^-1; 'dbj' (above);
'2las' GMRES(S (M^-1 + Z C\\(I - u_C u_C^T) Z^T), b_S).

direct_solve is the plain definition the method must reproduce: the
projected system L(k) u = f - u_L u_L^T f solved by least squares on a dense
L, gauge-fixed.  Tiny grids only.
"""
from dataclasses import dataclass

import numpy as np

from . import gmres as _gmres
from . import schur as _schur
from . import smpm


@dataclass
class Result:
    u: np.ndarray
    xS: np.ndarray
    bS: np.ndarray
    iters: int
    converged: bool
    schur_relres: float
    history: list
    compat_defect: float


def schur_rhs(sysm, F):
    """Steps 1-3: the projected right-hand side and the Schur right-hand side."""
    Ft = F.copy()
    compat = 0.0
    if sysm.singular:
        compat = abs(sysm.uL @ F) / max(np.linalg.norm(F), 1e-300)
        Ft = F - sysm.uL * (sysm.uL @ F)
    bS = sysm.B @ sysm.A_solve(Ft)
    if sysm.singular:
        bS = bS - sysm.uS * (sysm.uS @ bS)
    return Ft, bS, compat


def schur_solve(sysm, bS, method="dbj", tol=1e-10, maxit=300):
    """Solve S x = b_S with one of the Table 1 methods; returns
    (x_S, iterations, converged, history).

    Every method stops when its GMRES residual estimate is below
    tol * |b_S|: Sec. 4 accepts a solution when |S x_S - b_S| / |b_S| < tol,
    and for DBJ the deflated residual equals the true Schur residual while
    its starting vector P b_S can be longer than b_S (P is oblique)."""
    ref = float(np.linalg.norm(bS))
    if method == "schur":
        x, it, ok, hist = _gmres.gmres(sysm.S_apply, bS, tol, maxit, ref)
        return x, it, ok, hist
    if method == "bj":
        op = lambda v: sysm.S_apply(sysm.Minv_apply(v))
        xp, it, ok, hist = _gmres.gmres(op, bS, tol, maxit, ref)
        return sysm.Minv_apply(xp), it, ok, hist
    if method == "dbj":
        op = lambda v: sysm.P_apply(sysm.S_apply(sysm.Minv_apply(v)))
        xp, it, ok, hist = _gmres.gmres(op, sysm.P_apply(bS), tol, maxit, ref)
        x1 = sysm.Q_apply(sysm.Minv_apply(xp))
        x2 = sysm.Z(sysm.coarse(sysm.Zt(bS)))
        return x1 + x2, it, ok, hist
    if method == "2las":
        def prec(v):
            return sysm.Minv_apply(v) + sysm.Z(sysm.coarse(sysm.Zt(v)))
        xp, it, ok, hist = _gmres.gmres(lambda v: sysm.S_apply(prec(v)), bS, tol, maxit, ref)
        return prec(xp), it, ok, hist
    raise ValueError(method)


def recover(sysm, Ft, xS):
    """Step 9: u = A^-1 (b - E x_S), gauge-fixed to zero mean for k = 0."""
    u = sysm.A_solve(Ft - sysm.E @ xS)
    if sysm.singular:
        u = u - u.mean()
    return u


def dbj_solve(sysm, F, method="dbj", tol=1e-10, maxit=300):
    """Algorithm 2 for one right-hand side F = f + tau g (node layout)."""
    Ft, bS, compat = schur_rhs(sysm, F)
    xS, it, ok, hist = schur_solve(sysm, bS, method, tol, maxit)
    res = np.linalg.norm(sysm.S_apply(xS) - bS) / max(np.linalg.norm(bS), 1e-300)
    u = recover(sysm, Ft, xS)
    return Result(u, xS, bS, it, ok, res, hist, compat)


def null_vector_floor(sysm, F, rho=2e-13, samples=2, seed=0, tol=1e-12):
    """How far the k = 0 solution moves when its left null vectors come from
    S perturbed at the rounding level: the largest relative change of u (max
    norm) over `samples` seeded perturbations S -> S (1 + rho xi) entrywise,
    xi ~ N(0, 1), with u_S recomputed from the perturbed S and u_L from
    Claim 1, every other operator unchanged, both solves to `tol`.

    For incompatible data (u_L^T F != 0) the projected right-hand side
    F - u_L u_L^T F moves with u_L, and u_L is determined only to about
    rho |S| / sigma_{k-1}(S), the rounding residual of a null vector route
    over the gap to the next singular value (Sec. 2.4 defines the solution
    through these projections).  Two correct routes to the null vectors,
    each leaving a residual of order rho |S|, can therefore give solutions
    this far apart; rho = 2e-13 matches the residual either side's route
    leaves relative to |S|_1.  The result is a floor for comparisons of
    k = 0 solutions, not a property of either implementation."""
    from . import schur as _sch
    base = dbj_solve(sysm, F, tol=tol).u
    scale = np.abs(base).max()
    uS0, uL0 = sysm.uS, sysm.uL
    rng = np.random.default_rng(seed)
    worst = 0.0
    try:
        for _ in range(samples):
            Sp = sysm.S.copy()
            Sp.data = Sp.data * (1.0 + rho * rng.standard_normal(Sp.data.size))
            sysm.uS = _sch.left_null_S(Sp, sysm.grid.nhalf)
            sysm.uL = _sch.left_null_L(sysm, sysm.uS)
            u = dbj_solve(sysm, F, tol=tol).u
            worst = max(worst, float(np.abs(u - base).max() / scale))
    finally:
        sysm.uS, sysm.uL = uS0, uL0
    return worst


def direct_solve(grid, tau, F, kwave=0.0):
    """Dense least-squares solve of L(k) u = F - u_L u_L^T F (tiny grids)."""
    L = smpm.assemble_L(grid, tau, kwave).toarray()
    if kwave == 0.0:
        U, s, Vt = np.linalg.svd(L)
        uL = U[:, -1]
        F = F - uL * (uL @ F)
        u = np.linalg.lstsq(L, F, rcond=None)[0]
        return u - u.mean()
    return np.linalg.solve(L, F)


def dense_schur_solve(grid, tau, F, kwave=0.0):
    """The explicitly assembled dense Schur matrix solved directly (with the
    null-space projections of Sec. 2.4), then recovery.  Tiny grids only."""
    A = smpm.assemble_A(grid, tau, kwave).toarray()
    B = smpm.assemble_B(grid, tau).toarray()
    E = smpm.assemble_E(grid).toarray()
    Ainv = np.linalg.inv(A)
    S = np.eye(grid.k) + B @ Ainv @ E
    Ft = F.copy()
    if kwave == 0.0:
        L = A + E @ B
        U, s, Vt = np.linalg.svd(L)
        uL = U[:, -1]
        Ft = F - uL * (uL @ F)
    bS = B @ Ainv @ Ft
    if kwave == 0.0:
        Us, ss, Vts = np.linalg.svd(S)
        uS = Us[:, -1]
        bS = bS - uS * (uS @ bS)
        xS = np.linalg.lstsq(S, bS, rcond=None)[0]
    else:
        xS = np.linalg.solve(S, bS)
    u = Ainv @ (Ft - E @ xS)
    if kwave == 0.0:
        u = u - u.mean()
    return u, xS


def refine_solve(sysm, F, inner_tol=1e-6, tol=1e-10, maxit=300, max_sweeps=20,
                 dtype=np.float32, floor=0.0):
    """FP64 iterative refinement around a reduced-precision DBJ inner solve
    (the mixed-precision form; not in the paper).  The inner solve rounds the
    Schur blocks, the block-Jacobi inverses and every inner vector to `dtype`;
    the outer residual b_S - S x, the projections and the coarse solve stay
    FP64.  Each sweep starts from a zero correction and its inner GMRES stops
    once the residual estimate is at most max(inner_tol |r|, floor tol |b_S|),
    r the sweep's FP64 residual (floor = 0: inner_tol |r| alone).  Returns
    (Result, sweeps, total inner iterations); Result.history holds the
    relative FP64 residual before each sweep and extra "inner" the inner
    iteration count of each sweep."""
    Ft, bS, compat = schur_rhs(sysm, F)
    S_lo = sysm.S.astype(dtype)
    Mi_lo = [m.astype(dtype) for m in sysm.bj_inv]
    SZ = sysm.SZ

    def rnd(v):
        return v.astype(dtype).astype(np.float64)

    def Minv_lo(v):
        y = np.empty_like(v)
        vl = v.astype(dtype)
        for idx, Mi in zip(sysm.bj_index, Mi_lo):
            y[idx] = (Mi @ vl[idx]).astype(np.float64)
        return y

    def S_lo_apply(v):
        return (S_lo @ v.astype(dtype)).astype(np.float64)

    def P_lo(y):
        return rnd(y - SZ @ sysm.coarse(sysm.Zt(y)))

    x = np.zeros_like(bS)
    nb = np.linalg.norm(bS)
    total = 0
    sweeps = 0
    hist = []
    inner = []
    for sweeps in range(1, max_sweeps + 1):
        r = bS - sysm.S_apply(x)
        if sysm.singular:
            r = r - sysm.uS * (sysm.uS @ r)
        rel = np.linalg.norm(r) / nb
        hist.append(rel)
        if rel <= tol:
            sweeps -= 1
            break
        op = lambda v: P_lo(S_lo_apply(Minv_lo(v)))
        ref = max(np.linalg.norm(r), floor * tol * nb / inner_tol)
        xp, it, ok, _ = _gmres.gmres(op, P_lo(r), inner_tol, maxit, ref)
        total += it
        inner.append(it)
        d1 = sysm.Q_apply(Minv_lo(xp))
        d2 = sysm.Z(sysm.coarse(sysm.Zt(r)))
        x = x + d1 + d2
    res = np.linalg.norm(sysm.S_apply(x) - bS) / nb
    u = recover(sysm, Ft, x)
    out = Result(u, x, bS, total, res <= tol, res, hist, compat)
    out.inner = inner
    return out, sweeps, total
