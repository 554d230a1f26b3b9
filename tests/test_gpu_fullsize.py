"""GPU checks at the full benchmark sizes.

Two kinds of check.  Against the oracle's Algorithm 2 solve of the
benchmark's own inputs, element by element (c2, four modes of c4, six
problems of c5 computed here; c3 from values the oracle stored, since it
takes minutes at that size), both sides at a tight Schur residual and held
to 1e-10 relative.  And a property that holds at any size: with v a seeded
smooth node field and F = L(k) v formed by the oracle's own sparse operator,
the discrete solution is v (k > 0) or v minus its mean (k = 0, where F is
compatible by construction); the solve stops at a 1e-10 Schur residual, and
the solution error is that residual times the conditioning of the strip
problems, below 1e-7 (1e-6 on the stretched grids) for such v.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import paper_1512_01756_amd as P
from paper_1512_01756_amd import workloads
from oracle import schur, smpm, solve

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ACCEPT = 1.001e-10


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load()


def _smooth_field(xb, zb, n, seed):
    return workloads.smooth_field(xb, zb, n, seed)


def _check(xb, zb, n, kwaves, nrhs=1, precision=P.FP64, seed=0, tol_u=1e-7):
    s = P.Solver(xb, zb, n - 1, kwaves=kwaves, nrhs=nrhs, precision=precision)
    grid = smpm.Grid(xb, zb, n)
    tau = smpm.default_tau(grid)
    assert s.info[0]["tau"] == pytest.approx(tau, rel=1e-15)
    fs, vs = [], []
    for m, k in enumerate(kwaves):
        L = smpm.assemble_L(grid, tau, k)
        for q in range(nrhs):
            v = _smooth_field(xb, zb, n, seed + 97 * m + q)
            fs.append(L @ v)
            vs.append(v - v.mean() if k == 0.0 else v)
    f = torch.as_tensor(np.concatenate(fs)).cuda()
    u, st, status = s.solve(f)
    torch.cuda.synchronize()
    u = u.cpu().numpy().reshape(len(fs), -1)
    errs = [np.abs(u[i] - vs[i]).max() / np.abs(vs[i]).max() for i in range(len(fs))]
    print("stats", st, "max rel err", max(errs))
    assert st["rel_residual_max"] <= ACCEPT
    assert max(errs) <= tol_u
    s.close()
    return st


def test_c2_full_size_fp64_and_refined():
    p = workloads.c2()
    st64 = _check(p.xb, p.zb, p.n, [0.0])
    st32 = _check(p.xb, p.zb, p.n, [0.0], precision=P.FP32_IR)
    assert st32["sweeps_max"] >= 2


@pytest.mark.parametrize("precision", [P.FP64, P.FP32_IR])
def test_c3_full_size_distinct_strips(precision):
    p = workloads.c3()
    _check(p.xb, p.zb, p.n, [0.0], precision=precision, tol_u=1e-6)


def test_c4_full_size_all_modes():
    xb = np.linspace(0, 32, 65)
    zb = np.linspace(0, 1, 9)
    k = 2 * np.pi * np.arange(65) / 8.0
    _check(xb, zb, 13, k, nrhs=2, precision=P.FP32_IR)


def test_c5_full_size_uneven_batch():
    probs = workloads.c5()
    grids = [(p.xb, p.zb, p.n - 1, float(p.kwaves[0])) for p in probs]
    s = P.Solver(grids=grids, precision=P.FP32_IR)
    fs, vs = [], []
    for i, p in enumerate(probs):
        grid = smpm.Grid(p.xb, p.zb, p.n)
        L = smpm.assemble_L(grid, smpm.default_tau(grid), float(p.kwaves[0]))
        v = _smooth_field(p.xb, p.zb, p.n, i)
        fs.append(L @ v)
        vs.append(v - v.mean() if p.kwaves[0] == 0.0 else v)
    f = torch.as_tensor(np.concatenate(fs)).cuda()
    u, st, status = s.solve(f)
    u = u.cpu().numpy()
    off = 0
    worst = 0.0
    for i, p in enumerate(probs):
        ui = u[off:off + p.r]
        off += p.r
        worst = max(worst, np.abs(ui - vs[i]).max() / np.abs(vs[i]).max())
    print("c5 stats", st, "worst rel err", worst)
    assert st["rel_residual_max"] <= ACCEPT
    assert worst <= 1e-6


TIGHT = 1e-12
PARITY = 1e-10
FLOOR_FACTOR = 10
# Tight solves run to 1e-12 where each side's FP64 Schur residual gets
# there.  On the 64:1 c2 grid the GPU's FP64 residual bottoms out near 2e-12
# (CGS2 with the stored S M^-1 blocks; the oracle's Householder GMRES near
# 7e-13), so the check accepts up to 5e-12 there; the FP32-inner refinement
# stops with ENOTCONV below its FP64 floor, so it runs to 4e-12 (c2) or
# 1e-11 (the 130 modes, whose worst floor is near 9e-12).  The uneven batch
# runs in FP64 to 2e-11: several of its stiff problems bottom out near that.
FP64_FLOOR = 5e-12
IR_TOL = {"c2": 4e-12, "c4": 1e-11}


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _bound(o, F):
    """PARITY, or at k = 0 the larger of PARITY and FLOOR_FACTOR times the
    oracle's null-vector floor for this input (see test_gpu_parity)."""
    if not o.singular:
        return PARITY
    return max(PARITY, FLOOR_FACTOR * solve.null_vector_floor(o, F, samples=3, tol=TIGHT))


@pytest.fixture(scope="module")
def c2_oracle():
    p = workloads.c2()
    grid = smpm.Grid(p.xb, p.zb, p.n)
    o = schur.build(grid)
    F = smpm.rhs(grid, o.tau, p.f[0, 0])
    return p, solve.dbj_solve(o, F, tol=TIGHT), solve.dbj_solve(o, F).iters, _bound(o, F)


@pytest.mark.parametrize("precision", [P.FP64, P.FP32_IR])
def test_c2_full_size_matches_oracle_solve(precision, c2_oracle):
    # The benchmark's own input (128 x 8 elements, order 16, manufactured
    # solution plus seeded forcing) against the oracle's Algorithm 2 solve of
    # the same right-hand side, element by element, both at a tight Schur
    # residual; the FP64 iteration count at the paper's 1e-10 within one.
    p, ref, iters10, bound = c2_oracle
    f = torch.as_tensor(p.f.reshape(-1)).cuda()
    if precision == P.FP64:
        s = P.Solver(p.xb, p.zb, p.n - 1, precision=precision)
        _, st, status = s.solve(f)
        assert status == P.OK and st["rel_residual_max"] <= ACCEPT
        print("c2 full size at 1e-10", st, "oracle iters", iters10)
        assert abs(st["iters_max"] - iters10) <= 1
        s.close()
    tol = TIGHT if precision == P.FP64 else IR_TOL["c2"]
    s = P.Solver(p.xb, p.zb, p.n - 1, precision=precision, tol=tol)
    u, st, status = s.solve(f, check=False)
    u = u.cpu().numpy()
    err = _rel(u, ref.u)
    print("c2 full size", st, "status", status, "oracle iters", ref.iters, "err", err, "bound", bound)
    assert status == P.OK and st["rel_residual_max"] <= max(1.001 * tol, FP64_FLOOR)
    assert err <= bound
    s.close()


def test_c4_full_size_modes_match_oracle():
    # All 65 modes x (Re, Im) of the 64 x 8, order-12 grid solved as one
    # batch (FP32 inner, FP64 refinement); modes 0, 1, 32 and 64, both
    # parts, against the oracle's solve of the same Fourier coefficients.
    p = workloads.c4()
    tol = IR_TOL["c4"]
    s = P.Solver(p.xb, p.zb, p.n - 1, kwaves=p.kwaves, nrhs=2, precision=P.FP32_IR, tol=tol)
    u, st, status = s.solve(torch.as_tensor(p.f.reshape(-1)).cuda(), check=False)
    print("c4 full size", st, "status", status)
    assert status == P.OK and st["rel_residual_max"] <= 1.001 * tol
    u = u.cpu().numpy().reshape(p.nk, 2, p.r)
    grid = smpm.Grid(p.xb, p.zb, p.n)
    for m in (0, 1, 32, 64):
        o = schur.build(grid, kwave=float(p.kwaves[m]))
        for q in range(2):
            if np.abs(p.f[m, q]).max() == 0.0:     # Im of the real modes 0 and 64
                assert np.abs(u[m, q]).max() == 0.0
                continue
            F = smpm.rhs(grid, o.tau, p.f[m, q])
            ref = solve.dbj_solve(o, F, tol=TIGHT)
            err, bound = _rel(u[m, q], ref.u), _bound(o, F)
            print("c4 mode", m, q, "oracle iters", ref.iters, "err", err, "bound", bound)
            assert err <= bound, (m, q)


def _c3_golden():
    import os
    return np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_oracle.npz"))


def _k0_determined(grid, tau, L, u, uL, f, st, label):
    """What an incompatible k = 0 right-hand side determines, checked on the
    GPU's solution u and left null vector u_L: u_L is a left null vector of
    the oracle's L at the rounding level, u has zero nodal mean, and u solves
    L u = F - u_L u_L^T F to the Schur residual the solve reports (the
    interior rows of L u - F~ vanish up to the recovery's rounding and the
    interface rows are E (b_S - S x_S), |E|_2 = 1) plus the componentwise
    rounding of L u, 64 eps |L||u| (the entries of L reach tau and the
    derivative scales of the smallest elements)."""
    assert np.abs(L.T @ uL).max() <= 1e-12 * abs(L).max(), label
    assert abs(u.mean()) <= 1e-12 * np.abs(u).max(), label
    F = smpm.rhs(grid, tau, f)
    Ft = F - uL * (uL @ F)
    res = np.linalg.norm(L @ u - Ft)
    bnorm = _schur_rhs_norm(grid, tau, Ft)
    rounding = 64 * np.finfo(float).eps * np.linalg.norm(abs(L) @ np.abs(u))
    print(label, "|L u - F~|", res, "Schur residual x |b_S|", st["rel_residual_max"] * bnorm, "rounding", rounding)
    assert res <= 2.0 * st["rel_residual_max"] * bnorm + rounding, label


def _schur_rhs_norm(grid, tau, Ft):
    """|B A^-1 F~| with the oracle's strip operators (per-strip sparse LU)."""
    A = smpm.assemble_A(grid, tau)
    v = np.empty_like(Ft)
    for j in range(grid.mx):
        idx = schur.strip_range(grid, j)
        v[idx] = spla.splu(A[idx][:, idx].tocsc()).solve(Ft[idx])
    return np.linalg.norm(smpm.assemble_B(grid, tau) @ v)


@pytest.mark.parametrize("precision", [P.FP64, P.FP32_IR])
def test_c3_full_size_matches_oracle_solve(precision):
    # The stretched 256 x 16, order-12 grid with distinct strips against the
    # oracle's Algorithm 2 solves stored by tests/golden/make_c3_oracle.py
    # (the oracle takes minutes here).  On this grid (|tau| = 1.4e4, element
    # aspect ratios up to 20) FP64 itself attains only about 2e-9 in u: the
    # oracle's solution of a compatible F = L v at its residual floor (6e-12)
    # is that far from v minus its mean.
    #
    # The benchmark's f ~ U[0, 1] (u_L^T F / |F| = 0.49): FP64 iterations at
    # 1e-10 within one, FP32-refinement sweeps within one and inner
    # iterations within one per sweep.  Its solution is defined through the
    # projection with the left null vector u_L, which on this grid is known
    # only to about 2e-9 (both sides' u_S leave residuals near 1e-13 |S|_1
    # and differ by that angle); the solution moves about 700 times the
    # angle.  So the element-wise difference is held to 1e-5 only, and what
    # is checked is what the input determines: the GPU's u_L is a left null
    # vector of the oracle's L, and the GPU's u solves L u = F - u_L u_L^T F
    # with it to the Schur residual (|L u - F~| = |S x_S - b_S|, Claim 2).
    #
    # The compatible F = L v (v the seeded smooth field) does not depend on
    # the null vectors: the GPU at 1e-11 must be as close to v minus its mean
    # as twice the oracle's own distance, and within three times that
    # distance of the oracle's solution.
    ref = _c3_golden()
    p = workloads.c3()
    grid = smpm.Grid(p.xb, p.zb, p.n)
    tau = smpm.default_tau(grid)
    L = smpm.assemble_L(grid, tau)
    f = torch.as_tensor(p.f.reshape(-1)).cuda()
    s = P.Solver(p.xb, p.zb, p.n - 1, precision=precision)
    u, st, status = s.solve(f)
    print("c3 at 1e-10", st)
    assert status == P.OK and st["rel_residual_max"] <= ACCEPT
    if precision == P.FP64:
        assert abs(st["iters_max"] - int(ref["iters_1e10"])) <= 1
        uh = u.cpu().numpy()
        _k0_determined(grid, tau, L, uh, s.export(P.TABLE_U_L), p.f[0, 0], st, "c3 U[0,1]")
        err = np.abs(uh[ref["idx"]] - ref["u"]).max() / float(ref["umax"])
        print("c3 U[0,1]: element-wise difference from the oracle", err)
        assert err <= 1e-5
    else:
        inner = ref["ir_inner"]
        print("oracle refinement: sweeps", int(ref["ir_sweeps"]), "inner", inner)
        assert abs(st["sweeps_max"] - int(ref["ir_sweeps"])) <= 1
        assert abs(st["iters_total"] - int(ref["ir_total"])) <= len(inner)
    s.close()
    v = workloads.smooth_field(p.xb, p.zb, p.n, int(ref["smooth_seed"]))
    fc = torch.as_tensor(L @ v).cuda()
    tol = 1e-11
    s = P.Solver(p.xb, p.zb, p.n - 1, precision=precision, tol=tol)
    u, st, status = s.solve(fc, check=False)
    assert status == P.OK and st["rel_residual_max"] <= 1.001 * tol
    u = u.cpu().numpy()
    exact = v - v.mean()
    e_exact = np.abs(u - exact).max() / np.abs(exact).max()
    err = np.abs(u[ref["idx"]] - ref["uc"]).max() / float(ref["ucmax"])
    att = float(ref["c_err_exact"])
    print("c3 compatible", st, "err vs exact", e_exact, "oracle's", att, "err vs oracle", err)
    assert e_exact <= max(PARITY, 2.0 * att)
    assert err <= max(PARITY, 3.0 * att)
    s.close()


C5_ORACLE_PROBLEMS = (1, 3, 5, 6, 14, 20)   # k = 0 and k > 0 (one at k = 0.049), orders 8-15
# An incompatible k = 0 solution moves with the left null vector of L, which
# two correct routes determine only to about 1e-11 on these grids (the host
# setup's u_L and the oracle's differ by 1e-11 at residuals of 1e-16 |L| on
# problem 3): such problems are checked through what the input determines,
# with an element-wise guard at the difference that angle makes (8e-10).
K0_GUARD = 1e-8


def _c5_batch(probs, fs, tol):
    grids = [(p.xb, p.zb, p.n - 1, float(p.kwaves[0])) for p in probs]
    s = P.Solver(grids=grids, tol=tol)
    u, st, status = s.solve(torch.as_tensor(np.concatenate(fs)).cuda(), check=False)
    assert status == P.OK and st["rel_residual_max"] <= 1.001 * tol
    return s, u.cpu().numpy(), st


def test_c5_full_size_problems_match_oracle():
    # The whole 32-problem batch solved at once (FP64) against the oracle's
    # solves of six of its problems: first the seeded forcing, then the
    # compatible right-hand sides F = L v of smooth seeded fields v, whose
    # solutions (v, or v minus its mean at k = 0) do not depend on the null
    # vectors and are compared element by element at every k.
    probs = workloads.c5()
    tol = 2e-11
    offs = np.concatenate([[0], np.cumsum([p.r for p in probs])])
    s, u, st = _c5_batch(probs, [p.f.reshape(-1) for p in probs], tol)
    print("c5 full size", st)
    for i in C5_ORACLE_PROBLEMS:
        p = probs[i]
        k = float(p.kwaves[0])
        grid = smpm.Grid(p.xb, p.zb, p.n)
        o = schur.build(grid, kwave=k)
        F = smpm.rhs(grid, o.tau, p.f[0, 0])
        ui = u[offs[i]:offs[i + 1]]
        err = _rel(ui, solve.dbj_solve(o, F, tol=TIGHT).u)
        print("c5 problem", i, p.xb.size - 1, p.zb.size - 1, p.n, k, "err", err)
        if o.singular:
            L = smpm.assemble_L(grid, o.tau)
            _k0_determined(grid, o.tau, L, ui, s.export(P.TABLE_U_L, i), p.f[0, 0], st, "c5 problem %d" % i)
            assert err <= K0_GUARD, i
        else:
            assert err <= PARITY, i
    s.close()
    fs, exact = [], {}
    for i, p in enumerate(probs):
        k = float(p.kwaves[0])
        grid = smpm.Grid(p.xb, p.zb, p.n)
        v = workloads.smooth_field(p.xb, p.zb, p.n, 100 + i).reshape(-1)
        fs.append(smpm.assemble_L(grid, smpm.default_tau(grid), k) @ v)
        exact[i] = v - v.mean() if k == 0.0 else v
    s, u, st = _c5_batch(probs, fs, tol)
    print("c5 compatible", st)
    for i in C5_ORACLE_PROBLEMS:
        p = probs[i]
        grid = smpm.Grid(p.xb, p.zb, p.n)
        o = schur.build(grid, kwave=float(p.kwaves[0]))
        ref = solve.dbj_solve(o, fs[i], tol=TIGHT).u
        ui = u[offs[i]:offs[i + 1]]
        err, att = _rel(ui, ref), _rel(ref, exact[i])
        print("c5 compatible problem", i, "err", err, "oracle vs exact", att, "GPU vs exact", _rel(ui, exact[i]))
        assert err <= PARITY, i
    s.close()


def test_sampled_schur_blocks_full_size_c3():
    # The oracle computes W_j for a few strips of the full 256 x 16 grid and
    # the GPU matvec must reproduce the rows those strips write.
    p = workloads.c3()
    s = P.Solver(p.xb, p.zb, p.n - 1)
    grid = smpm.Grid(p.xb, p.zb, p.n)
    tau = smpm.default_tau(grid)
    A = smpm.assemble_A(grid, tau)
    B = smpm.assemble_B(grid, tau)
    E = smpm.assemble_E(grid)
    x = np.random.default_rng(5).standard_normal(grid.k)
    xd = torch.as_tensor(x).cuda()
    y = torch.empty_like(xd)
    s.apply(P.OP_SCHUR, 0, xd, y)
    y = y.cpu().numpy()
    for j in (0, 1, 117, 254, 255):
        _, Wj, ridx, cidx = schur._strip(grid, A, B, E, j)
        ref = x[ridx] + Wj @ x[cidx]
        assert np.abs(y[ridx] - ref).max() <= 1e-11 * np.abs(ref).max(), j
