"""The 3-D problem through a Fourier series in the periodic y direction
(Sec. 5) (oracle).

Test infrastructure: see the package docstring.

With u(x, y, z) = sum_m u_m(x, z) exp(i k_m y), k_m = 2 pi m / L_y, on m_y
equispaced points y_j = j L_y / m_y, every mode solves the 2-D Helmholtz
problem (L - k_m^2 I) u_m = f_m (Sec. 5).  The field is real, so only
m = 0 .. m_y/2 are solved and Re, Im of each mode are two real right-hand
sides of the same real operator.  Coefficients are normalized by 1/m_y:

  f_m = (1/m_y) sum_j f(y_j) exp(-2 pi i m j / m_y)      (forward)
  u(y_j) = sum over m of u_m exp(2 pi i m j / m_y)       (inverse, with
           u_{-m} = conj(u_m))

Both directions use numpy's real FFT.
"""
import numpy as np

from . import schur, smpm, solve


def wavenumbers(my, ly):
    """k_m = 2 pi m / L_y for m = 0 .. m_y // 2."""
    return 2.0 * np.pi * np.arange(my // 2 + 1) / ly


def forward(fphys):
    """(m_y, ...) physical samples -> (m_y//2 + 1, 2, ...) [Re, Im] coefficients."""
    my = fphys.shape[0]
    fh = np.fft.rfft(fphys, axis=0) / my
    return np.stack([fh.real, fh.imag], axis=1)


def inverse(uhat, my):
    """(m_y//2 + 1, 2, ...) [Re, Im] coefficients -> (m_y, ...) physical samples."""
    c = (uhat[:, 0] + 1j * uhat[:, 1]) * my
    return np.fft.irfft(c, n=my, axis=0)


def solve3d(xb, zb, n, fphys, ly, gphys=None, method="dbj", tol=1e-10, one_krylov=False):
    """Solve the 3-D Poisson-Neumann problem mode by mode (Alg. 2 per mode).

    fphys: (m_y, r) node values per y-plane; gphys: None or a dict of side
    arrays (m_y, m_x or m_z, n) for S, N, W, E.  Returns (u, results) with u of
    shape (m_y, r); the k = 0 mode carries the zero-mean gauge.

    one_krylov: the paper's form of Alg. 3, one DBJ-GMRES on the
    block-diagonal operator diag_i(P_i S_i M_i^-1) over every (mode, Re/Im)
    instance i (Sec. 5.2), stopping when its residual is below tol times the
    norm of the stacked right-hand sides; results is then (iterations,
    converged)."""
    my = fphys.shape[0]
    grid = smpm.Grid(np.asarray(xb, float), np.asarray(zb, float), n)
    fh = forward(fphys)
    gh = {side: forward(arr) for side, arr in gphys.items()} if gphys else None
    uh = np.zeros_like(fh)
    results = []
    insts = []
    for m, k in enumerate(wavenumbers(my, ly)):
        o = schur.build(grid, kwave=float(k))
        for q in range(2):
            g = {side: arr[m, q] for side, arr in gh.items()} if gh else None
            F = smpm.rhs(grid, o.tau, fh[m, q], g)
            if one_krylov:
                insts.append((m, q, o, F))
                continue
            if not np.any(F):
                results.append(None)
                continue
            res = solve.dbj_solve(o, F, method=method, tol=tol)
            uh[m, q] = res.u
            results.append(res)
    if one_krylov:
        if method != "dbj":
            raise ValueError("one_krylov is defined for the DBJ method")
        rhs = [solve.schur_rhs(o, F) for (_, _, o, F) in insts]
        sizes = [len(b) for (_, b, _) in rhs]
        cuts = np.cumsum([0] + sizes)

        def op(v):
            return np.concatenate([o.P_apply(o.S_apply(o.Minv_apply(v[cuts[i]:cuts[i + 1]])))
                                   for i, (_, _, o, _) in enumerate(insts)])

        b = np.concatenate([o.P_apply(bS) for (_, _, o, _), (_, bS, _) in zip(insts, rhs)])
        ref = float(np.linalg.norm(np.concatenate([bS for (_, bS, _) in rhs])))
        xp, it, ok, _ = solve._gmres.gmres(op, b, tol, 300, ref)
        for i, ((m, q, o, F), (Ft, bS, _)) in enumerate(zip(insts, rhs)):
            x1 = o.Q_apply(o.Minv_apply(xp[cuts[i]:cuts[i + 1]]))
            x2 = o.Z(o.coarse(o.Zt(bS)))
            uh[m, q] = solve.recover(o, Ft, x1 + x2)
        results = (it, ok)
    return inverse(uh, my), results
