"""SMPM discretization of the 2-D Poisson/Helmholtz-Neumann problem (oracle).

Test infrastructure: see the package docstring.

Paper Sec. 2.2, Eq. (smpm_poisson): on element V_i the residual is the
Laplacian plus tau_i times the Robin-type inter-element mismatch
R_ii u_i - sum_j R_ij u_j (R_ij = I + n_i . grad, n_i the outward normal of
V_i) plus tau_i times the physical Neumann term n_i . grad u_i; the right-hand
side is f_i + tau_i g_i.  The penalty terms sit on the element's edge nodes; a
corner node carries the terms of both of its edges.

Paper Sec. 2.3: the domain is cut into m_x vertical strips of m_z elements.
E (r x k) injects interface values, B (k x r) holds every flux between
elements of different strips, A = L - E B is block diagonal over strips.
The shifted operator of Sec. 5 is L(k) = L - k^2 I, A(k) = A - k^2 I with B
and E unchanged.

Node layout (also the layout of f and u everywhere in this project):
    node(j, e, b, a) = ((j * m_z + e) * n + b) * n + a
j = strip (x index), e = element in the strip (z index, bottom first),
b = GLL index in z, a = GLL index in x (fastest).

Interface (Schur) layout: half-interface h = 2 i is Gamma_i^L (the east-edge
nodes of strip i), h = 2 i + 1 is Gamma_i^R (the west-edge nodes of strip
i + 1), i = 0 .. m_x - 2; inside a half the order is (e, b).  Index
h * n * m_z + e * n + b.

Neumann data g is given per physical side: south/north arrays of shape
(m_x, n) indexed (strip, a); west/east arrays of shape (m_z, n) indexed
(element, b).
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import gll


@dataclass
class Grid:
    """Axis-aligned rectangular elements from breakpoints (Sec. 2.2 maps each
    element affinely from [-1, 1]^2)."""
    xb: np.ndarray   # m_x + 1 increasing x breakpoints
    zb: np.ndarray   # m_z + 1 increasing z breakpoints
    n: int           # GLL points per direction

    def __post_init__(self):
        self.xb = np.asarray(self.xb, dtype=np.float64)
        self.zb = np.asarray(self.zb, dtype=np.float64)
        if len(self.xb) < 3 or len(self.zb) < 2 or self.n < 2:
            raise ValueError("need m_x >= 2, m_z >= 1, n >= 2")
        if np.any(np.diff(self.xb) <= 0) or np.any(np.diff(self.zb) <= 0):
            raise ValueError("breakpoints must increase")

    @property
    def mx(self):
        return len(self.xb) - 1

    @property
    def mz(self):
        return len(self.zb) - 1

    @property
    def r(self):
        """Number of grid nodes, r = n^2 m_x m_z (Sec. 2.2)."""
        return self.n * self.n * self.mx * self.mz

    @property
    def nhalf(self):
        """Nodes on one side of an interface, n m_z (Sec. 2.3)."""
        return self.n * self.mz

    @property
    def k(self):
        """Schur dimension k = 2 n m_z (m_x - 1) (Sec. 2.3)."""
        return 2 * self.nhalf * (self.mx - 1)

    def node(self, j, e, b, a):
        n = self.n
        return ((j * self.mz + e) * n + b) * n + a

    def gamma(self, h, e, b):
        return h * self.nhalf + e * self.n + b

    def coords(self):
        """Physical coordinates (x, z) of every node, in node order."""
        xi = gll.gll_nodes(self.n)
        hx = np.diff(self.xb)
        hz = np.diff(self.zb)
        xs = self.xb[:-1, None] + (xi[None, :] + 1) * 0.5 * hx[:, None]     # (m_x, n): [j, a]
        zs = self.zb[:-1, None] + (xi[None, :] + 1) * 0.5 * hz[:, None]     # (m_z, n): [e, b]
        shape = (self.mx, self.mz, self.n, self.n)
        X = np.broadcast_to(xs[:, None, None, :], shape).reshape(-1).copy()
        Z = np.broadcast_to(zs[None, :, :, None], shape).reshape(-1).copy()
        return X, Z


def default_tau(grid):
    """One global penalty value, a reading of Sec. 2.2: tau = -n(n-1)/h_min,
    h_min the smallest element width or height."""
    n = grid.n
    hmin = min(np.min(np.diff(grid.xb)), np.min(np.diff(grid.zb)))
    return -n * (n - 1) / hmin


_SIDES = ("W", "E", "S", "N")
_OPPOSITE = {"W": "E", "E": "W", "S": "N", "N": "S"}


def _side_nodes(n, side):
    """Local indices (b * n + a) of the n nodes along an element side."""
    t = np.arange(n)
    return {"W": t * n, "E": t * n + n - 1, "S": t, "N": (n - 1) * n + t}[side]


def _outward_dn(n, D, hx, hz, side):
    """Outward normal derivative at the nodes of a side: an n x n^2 matrix,
    row t acting on the element's local nodes."""
    M = np.zeros((n, n * n))
    t = np.arange(n)
    for c in range(n):
        if side == "W":
            M[t, t * n + c] = -(2.0 / hx) * D[0, c]
        elif side == "E":
            M[t, t * n + c] = (2.0 / hx) * D[n - 1, c]
        elif side == "S":
            M[t, c * n + t] = -(2.0 / hz) * D[0, c]
        else:
            M[t, c * n + t] = (2.0 / hz) * D[n - 1, c]
    return M


def _neighbour(grid, j, e, side):
    """Adjacent element across a side, or None on the physical boundary."""
    jj, ee = {"W": (j - 1, e), "E": (j + 1, e), "S": (j, e - 1), "N": (j, e + 1)}[side]
    if 0 <= jj < grid.mx and 0 <= ee < grid.mz:
        return jj, ee
    return None


def _sizes(grid, j, e):
    return grid.xb[j + 1] - grid.xb[j], grid.zb[e + 1] - grid.zb[e]


def _terms(grid, tau, which):
    """COO triplets of the SMPM operator, element by element.

    which: set of parts to include:
      'lap'   the Laplacian at every node
      'self'  tau (R_ii u_i) on interior edges and tau n.grad u_i on physical
              edges
      'intra' -tau R_ij u_j for neighbours in the same strip
      'inter' -tau R_ij u_j for neighbours in another strip
    R_ij u_j = u_j + n_i . grad u_j with n_i = -(outward normal of j), so the
    neighbour block is -tau (facing-node value) + tau (j's outward derivative).
    """
    n = grid.n
    m2 = n * n
    D = gll.diff_matrix(gll.gll_nodes(n))
    D2 = D @ D
    I = np.eye(n)
    KX = np.kron(I, D2)      # d^2/dxi^2 on local index b * n + a
    KZ = np.kron(D2, I)      # d^2/dzeta^2
    rows, cols, vals = [], [], []

    def emit(block, row0, col0):
        rr, cc = np.nonzero(block)
        rows.append(row0 + rr); cols.append(col0 + cc); vals.append(block[rr, cc])

    for j in range(grid.mx):
        for e in range(grid.mz):
            hx, hz = _sizes(grid, j, e)
            base = grid.node(j, e, 0, 0)
            own = np.zeros((m2, m2))
            if "lap" in which:
                own += (2.0 / hx) ** 2 * KX + (2.0 / hz) ** 2 * KZ
            for side in _SIDES:
                nb = _neighbour(grid, j, e, side)
                sn = _side_nodes(n, side)
                if "self" in which:
                    own[sn, :] += tau * _outward_dn(n, D, hx, hz, side)
                    if nb is not None:
                        own[sn, sn] += tau
                if nb is None:
                    continue
                other_strip = nb[0] != j
                if (other_strip and "inter" in which) or (not other_strip and "intra" in which):
                    fside = _OPPOSITE[side]
                    hxn, hzn = _sizes(grid, *nb)
                    blk = np.zeros((m2, m2))
                    blk[sn, :] = tau * _outward_dn(n, D, hxn, hzn, fside)
                    blk[sn, _side_nodes(n, fside)] += -tau
                    emit(blk, base, grid.node(nb[0], nb[1], 0, 0))
            emit(own, base, base)
    if not rows:
        return np.zeros(0, int), np.zeros(0, int), np.zeros(0)
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def assemble_L(grid, tau, k=0.0):
    """The full SMPM operator L(k) = L - k^2 I (Eq. smpm_poisson; Sec. 5)."""
    r, c, v = _terms(grid, tau, {"lap", "self", "intra", "inter"})
    L = sp.coo_matrix((v, (r, c)), shape=(grid.r, grid.r)).tocsr()
    if k != 0.0:
        L = L - (k * k) * sp.identity(grid.r, format="csr")
    return L


def assemble_A(grid, tau, k=0.0):
    """The strip-local part A(k) (Sec. 2.3): Laplacian, boundary terms, R_ii
    terms and fluxes between elements of the same strip, minus k^2 I."""
    r, c, v = _terms(grid, tau, {"lap", "self", "intra"})
    A = sp.coo_matrix((v, (r, c)), shape=(grid.r, grid.r)).tocsr()
    if k != 0.0:
        A = A - (k * k) * sp.identity(grid.r, format="csr")
    return A


def assemble_E(grid):
    """Inclusion Gamma -> Omega (Sec. 2.3): 0/1 entries, E^T E = I."""
    n = grid.n
    rows, cols = [], []
    for i in range(grid.mx - 1):
        for e in range(grid.mz):
            for b in range(n):
                rows.append(grid.node(i, e, b, n - 1)); cols.append(grid.gamma(2 * i, e, b))
                rows.append(grid.node(i + 1, e, b, 0)); cols.append(grid.gamma(2 * i + 1, e, b))
    return sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(grid.r, grid.k)).tocsr()


def assemble_B(grid, tau):
    """Inter-strip fluxes (Sec. 2.3): the row of a Gamma node holds
    -tau (u_j + n_i . grad u_j) read from the facing strip's edge element."""
    n = grid.n
    xi = gll.gll_nodes(n)
    D = gll.diff_matrix(xi)
    rows, cols, vals = [], [], []
    for i in range(grid.mx - 1):
        hxr = grid.xb[i + 2] - grid.xb[i + 1]   # strip i + 1
        hxl = grid.xb[i + 1] - grid.xb[i]       # strip i
        for e in range(grid.mz):
            for b in range(n):
                # Gamma_i^L: node of strip i (normal +x) reads strip i + 1's west node row.
                row = grid.gamma(2 * i, e, b)
                rows.append(row); cols.append(grid.node(i + 1, e, b, 0)); vals.append(-tau)
                for c in range(n):
                    rows.append(row); cols.append(grid.node(i + 1, e, b, c))
                    vals.append(-tau * (2.0 / hxr) * D[0, c])
                # Gamma_i^R: node of strip i + 1 (normal -x) reads strip i's east node row.
                row = grid.gamma(2 * i + 1, e, b)
                rows.append(row); cols.append(grid.node(i, e, b, n - 1)); vals.append(-tau)
                for c in range(n):
                    rows.append(row); cols.append(grid.node(i, e, b, c))
                    vals.append(-tau * (-(2.0 / hxl)) * D[n - 1, c])
    return sp.coo_matrix((vals, (rows, cols)), shape=(grid.k, grid.r)).tocsr()


def rhs(grid, tau, f, g=None):
    """Right-hand side f + tau g of Eq. (smpm_poisson).  g is a dict with keys
    'S', 'N' (shape (m_x, n)) and 'W', 'E' (shape (m_z, n)); missing sides
    are zero.  A corner node receives the data of both of its sides."""
    F = np.array(f, dtype=np.float64).reshape(grid.r).copy()
    if g is None:
        return F
    n = grid.n
    for side, arr in g.items():
        arr = np.asarray(arr, dtype=np.float64)
        if side in ("S", "N"):
            e = 0 if side == "S" else grid.mz - 1
            b = 0 if side == "S" else n - 1
            for j in range(grid.mx):
                for a in range(n):
                    F[grid.node(j, e, b, a)] += tau * arr[j, a]
        else:
            j = 0 if side == "W" else grid.mx - 1
            a = 0 if side == "W" else n - 1
            for e in range(grid.mz):
                for b in range(n):
                    F[grid.node(j, e, b, a)] += tau * arr[e, b]
    return F
