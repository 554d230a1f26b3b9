"""Schur complement, block-Jacobi blocks, deflation and null vectors (oracle).

Test infrastructure: see the package docstring.

Sec. 2.3, Eq. (operator_decomp): S = I + B A^-1 E over the inter-strip flux
unknowns x_S = B u, b_S = B A^-1 f, u = A^-1 (f - E x_S).
Sec. 3.1: S is assembled from per-strip blocks and applied as a sum of
block products.  Strip j feeds the rows Gamma_{j-1}^L and Gamma_j^R from its
own edge values Gamma_{j-1}^R, Gamma_j^L, so S = I + sum_j (rows_j) W_j
(cols_j) with W_j = B[rows_j, strip j] A_j^-1 E[strip j, cols_j].  The oracle
computes every W_j with a sparse LU of that strip's block of A.
Sec. 3.2: block-Jacobi blocks are the principal submatrices of S on two
consecutive interfaces (Gamma_{2b}, Gamma_{2b+1}); the last block holds a
single interface when the interface count is odd.
Sec. 3.3, Eqs. (projection1), (projection2): Z holds one indicator column
per interface (or, as a richer space, per element segment of an interface),
C = Z^T S Z, P = I - S Z C^-1 Z^T, Q = I - Z C^-1 Z^T S; for
the singular Poisson case the coarse division is C \\ (I - u_C u_C^T) with u_C
the unit left null vector of C.
Sec. 2.4, Claim 1: u_S = E^T u_L and u_L = A^-T B^T u_S (up to scale).
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import smpm


def strip_range(grid, j):
    m = grid.n * grid.n * grid.mz
    return np.arange(j * m, (j + 1) * m)


def half_range(grid, h):
    N = grid.nhalf
    return np.arange(h * N, (h + 1) * N)


def strip_rows_cols(grid, j):
    """Half-interfaces written (rows) and read (cols) by strip j."""
    nh = 2 * (grid.mx - 1)
    rows = [h for h in (2 * j - 2, 2 * j + 1) if 0 <= h < nh]
    cols = [h for h in (2 * j - 1, 2 * j) if 0 <= h < nh]
    return rows, cols


@dataclass
class SchurSystem:
    grid: smpm.Grid
    tau: float
    kwave: float
    A: sp.csr_matrix
    B: sp.csr_matrix
    E: sp.csr_matrix
    lus: list                 # per-strip sparse LU of A_j(k)
    W: list                   # per-strip dense W_j
    S: sp.csr_matrix          # assembled Schur matrix
    bj_index: list            # per block, Gamma indices
    bj_inv: list              # per block, dense M_b^-1
    labels: np.ndarray        # Z label map: Gamma index -> interface
    C: np.ndarray             # Z^T S Z
    SZ: np.ndarray            # S Z (k x d)
    uS: np.ndarray = None     # left null vectors (k = 0 only)
    uL: np.ndarray = None
    uC: np.ndarray = None
    extra: dict = field(default_factory=dict)

    @property
    def singular(self):
        return self.kwave == 0.0

    # ---- operators -------------------------------------------------------
    def A_solve(self, v, trans=False):
        """A(k)^-1 v (or A(k)^-T v), strip by strip."""
        out = np.empty_like(v)
        for j, lu in enumerate(self.lus):
            idx = strip_range(self.grid, j)
            out[idx] = lu.solve(v[idx], trans="T" if trans else "N")
        return out

    def S_apply(self, x):
        return self.S @ x

    def Minv_apply(self, x):
        y = np.empty_like(x)
        for idx, Mi in zip(self.bj_index, self.bj_inv):
            y[idx] = Mi @ x[idx]
        return y

    def Zt(self, x):
        return np.bincount(self.labels, weights=x, minlength=self.C.shape[0])

    def Z(self, c):
        return c[self.labels]

    def coarse(self, t):
        """C^dagger (I - u_C u_C^T) t: the regularized coarse division of
        Sec. 3.3 (plain C^-1 t when C is nonsingular).  C has rank d - 1 for
        k = 0; C^dagger is the Moore-Penrose inverse of that rank-(d-1)
        matrix, V_{d-1} Sigma_{d-1}^-1 U_{d-1}^T from the SVD of C, whose
        range is orthogonal to 1_d.  P does not depend on which solution is
        taken (a shift along 1_d is annihilated by S Z)."""
        if self.singular:
            U, s, Vt = self.extra["C_svd"]
            return Vt[:-1].T @ ((U[:, :-1].T @ (t - self.uC * (self.uC @ t))) / s[:-1])
        return np.linalg.solve(self.C, t)

    def P_apply(self, y):
        return y - self.SZ @ self.coarse(self.Zt(y))

    def Q_apply(self, x):
        return x - self.Z(self.coarse(self.Zt(self.S_apply(x))))


def _strip(grid, A, B, E, j):
    """Sparse LU of A_j(k) (kept for A^-1 v) and the strip block
    W_j = B[rows_j] A_j^-1 E[cols_j], computed with a dense LU of A_j(k)."""
    sidx = strip_range(grid, j)
    Aj = A[sidx][:, sidx]
    lu = spla.splu(Aj.tocsc())
    rows, cols = strip_rows_cols(grid, j)
    ridx = np.concatenate([half_range(grid, h) for h in rows])
    cidx = np.concatenate([half_range(grid, h) for h in cols])
    X = sla.lu_solve(sla.lu_factor(Aj.toarray()), E[sidx][:, cidx].toarray())
    return lu, B[ridx][:, sidx] @ X, ridx, cidx


def z_labels(grid, zlabel=0):
    """Label map of the deflation space Z (Sec. 3.3): Gamma index -> coarse
    unknown.  zlabel 0: one indicator per interface Gamma_i (the paper's Z,
    d = m_x - 1); zlabel 1: one per element segment of an interface, the n
    nodes of element e on both sides of Gamma_i (d = (m_x - 1) m_z)."""
    nif = grid.mx - 1
    if zlabel == 0:
        return np.repeat(np.arange(nif), 2 * grid.nhalf)
    h = np.repeat(np.arange(2 * nif), grid.nhalf)                    # half of each Gamma index
    e = np.tile(np.repeat(np.arange(grid.mz), grid.n), 2 * nif)      # element of each Gamma index
    return (h // 2) * grid.mz + e


def build(grid, tau=None, kwave=0.0, zlabel=0):
    """Assemble every operator of the Schur method for one 2-D problem.
    zlabel selects the deflation space (see z_labels)."""
    if tau is None:
        tau = smpm.default_tau(grid)
    A = smpm.assemble_A(grid, tau, kwave)
    B = smpm.assemble_B(grid, tau)
    E = smpm.assemble_E(grid)
    k = grid.k
    parts = [_strip(grid, A, B, E, j) for j in range(grid.mx)]
    lus = [p[0] for p in parts]
    W = [p[1] for p in parts]
    Srows, Scols, Svals = [np.arange(k)], [np.arange(k)], [np.ones(k)]
    for (_, Wj, ridx, cidx) in parts:
        rr, cc = np.meshgrid(ridx, cidx, indexing="ij")
        Srows.append(rr.ravel()); Scols.append(cc.ravel()); Svals.append(Wj.ravel())
    S = sp.coo_matrix((np.concatenate(Svals), (np.concatenate(Srows), np.concatenate(Scols))),
                      shape=(k, k)).tocsr()
    # Block-Jacobi: pairs of interfaces (Sec. 3.2).
    nif = grid.mx - 1
    bj_index = []
    for b0 in range(0, nif, 2):
        ifs = [i for i in (b0, b0 + 1) if i < nif]
        bj_index.append(np.concatenate([np.concatenate([half_range(grid, 2 * i),
                                                        half_range(grid, 2 * i + 1)]) for i in ifs]))
    bj_inv = [np.linalg.inv(S[idx][:, idx].toarray()) for idx in bj_index]
    labels = z_labels(grid, zlabel)
    d = int(labels.max()) + 1
    Zs = sp.coo_matrix((np.ones(k), (np.arange(k), labels)), shape=(k, d)).tocsr()
    SZ = (S @ Zs).toarray()
    C = (Zs.T @ SZ)
    sysm = SchurSystem(grid, tau, float(kwave), A, B, E, lus, W, S, bj_index, bj_inv,
                       labels, np.asarray(C), SZ)
    if kwave == 0.0:
        null_vectors(sysm)
    return sysm


# Above this Schur dimension the sparse LU of the bordered system runs out of
# room (SuperLU's fill on the 256 x 16 grid), and the banded route is taken.
BORDERED_MAX_K = 60000


def _left_null_banded(S, N):
    """u with S^T u = 0 and 1^T u = 1 (the bordered system below), through a
    banded LU of M = S^T + e_p e_p^T.

    S couples each half-interface only to the halves of its window, at most
    two halves away, so S^T is banded with 3N - 1 sub- and super-diagonals
    (N nodes per half).  Adding 1 to one diagonal entry p keeps every
    equation of S^T and makes M nonsingular whenever u_S[p] != 0: if
    M v = 0 then S^T v = -v_p e_p, whose left side is orthogonal to 1
    (S 1 = 0) while e_p is not, so v_p = 0, and v is a null vector with a
    zero entry at p, hence v = 0.  c = M^-1 e_p is u_S / u_S[p].

    The bordered equations S^T u + lam 1 = 0, 1^T u = 1 are then solved by
    iterative refinement with M standing in for S^T: a correction (du, dl)
    for the residuals (r1, r2) solves S^T du + dl 1 = r1, 1^T du = r2;
    writing S^T du = M du - e_p du_p gives du = a - dl b + du_p c with
    a = M^-1 r1 and b = M^-1 1, where row p (c_p = 1) fixes dl = a_p / b_p
    and 1^T du = r2 fixes du_p.  The residuals are formed with S itself, so
    the refined u keeps every equation to the rounding of S, like the
    bordered LU (the first solve alone leaves row p satisfied only to the
    rounding of S 1 = 0).  p starts mid-vector and moves to the largest
    entry of c if c_p came out small against c."""
    k = S.shape[0]
    bw = 3 * N - 1
    St = S.T.tocsr()
    coo = St.tocoo()
    assert np.all(np.abs(coo.row - coo.col) <= bw)
    ones = np.ones(k)
    p = k // 2
    for _ in range(2):
        ab = np.zeros((3 * bw + 1, k))     # LAPACK band storage with room for the fill
        ab[2 * bw + coo.row - coo.col, coo.col] = coo.data
        ab[2 * bw, p] += 1.0
        lu, piv, info = sla.lapack.dgbtrf(ab, bw, bw)
        assert info == 0

        def msolve(rhs):
            x, inf = sla.lapack.dgbtrs(lu, bw, bw, rhs, piv)
            assert inf == 0
            return x

        ep = np.zeros(k)
        ep[p] = 1.0
        c = msolve(ep)
        if abs(c[p]) >= 1e-2 * np.abs(c).max():
            break
        p = int(np.argmax(np.abs(c)))
    b = msolve(ones)
    u = c / c.sum()
    lam = 0.0
    for _ in range(3):
        r1 = -(St @ u + lam * ones)
        r2 = 1.0 - u.sum()
        a = msolve(r1)
        dl = a[p] / b[p]
        dup = (r2 - a.sum() + dl * b.sum()) / c.sum()
        u = u + a - dl * b + dup * c
        lam += dl
    return u


def left_null_S(S, N):
    """Unit left null vector of S with a positive sum (see null_vectors);
    N nodes per half-interface."""
    k = S.shape[0]
    if k > BORDERED_MAX_K:
        u = _left_null_banded(S, N)
    else:
        one = sp.csc_matrix(np.ones((k, 1)))
        border = sp.bmat([[S.T.tocsc(), one], [one.T, None]], format="csc")
        rhs = np.zeros(k + 1)
        rhs[k] = 1.0
        u = spla.splu(border).solve(rhs)[:k]
    uS = u / np.linalg.norm(u)
    return uS * np.sign(uS.sum())


def left_null_L(sysm, uS):
    """u_L = A^-T B^T u_S (Claim 1, part 2), unit, positive sum."""
    uL = sysm.A_solve(sysm.B.T @ uS, trans=True)
    uL /= np.linalg.norm(uL)
    return uL * np.sign(uL.sum())


def null_vectors(sysm):
    """Left null vectors for the Poisson (k = 0) case.

    u_S: the bordered system [[S^T, 1], [1^T, 0]] [u; lam] = [0; 1], solved
    by a sparse LU.  It is nonsingular because 1^T u_S != 0 (Sec. 3.1), and
    lam = 0 in exact arithmetic (S 1 = 0); every equation of S^T u = 0 is
    kept, so u is as accurate as S itself (dropping one equation and pinning
    one component instead leaves that equation satisfied only to the rounding
    of S 1 = 0, amplified by the conditioning of the pinned system).  Above
    BORDERED_MAX_K unknowns a banded LU of S^T with one diagonal entry
    raised by 1, which also keeps every equation (_left_null_banded).
    u_L = A^-T B^T u_S (Claim 1, part 2), normalized.
    u_C: the unit left singular vector of the smallest singular value of C.
    Signs: each vector is scaled to have a positive sum.
    """
    uS = left_null_S(sysm.S, sysm.grid.nhalf)
    uL = left_null_L(sysm, uS)
    U, s, Vt = np.linalg.svd(sysm.C)
    sysm.extra["C_svd"] = (U, s, Vt)
    uC = U[:, -1] * np.sign(U[:, -1].sum())
    sysm.uS, sysm.uL, sysm.uC = uS, uL, uC
    return uS, uL, uC


def dense_schur(grid, tau, kwave=0.0):
    """S = I + B A^-1 E formed with a dense inverse of A (tiny grids only)."""
    A = smpm.assemble_A(grid, tau, kwave).toarray()
    B = smpm.assemble_B(grid, tau).toarray()
    E = smpm.assemble_E(grid).toarray()
    return np.eye(grid.k) + B @ np.linalg.inv(A) @ E
