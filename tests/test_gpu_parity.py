"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import paper_1512_01756_amd as P
from paper_1512_01756_amd import workloads
from oracle import schur, smpm, solve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load()


# The stopping test is |g| <= tol |b~|; the recursive and the true residual
# agree to rounding, so the true residual is accepted up to 0.1% above tol.
ACCEPT = 1.001e-10
# Solution parity: both sides solve to a 1e-12 relative Schur residual, so the
# comparison sees the arithmetic (GEMM order, CGS2 against Householder, the two
# routes to the null vectors), not where each side happened to stop; a
# 1e-10-residual solution differs from the exact discrete one by about 1e-10
# itself.  Every case, k = 0 included, is then held to 1e-10 relative: at
# k = 0 the two sides' left null vectors (inverse iteration against a bordered
# sparse LU) differ by about 1e-13 on these grids and 6e-11 on the 64:1 c2
# grid, and the solution moves by less than that angle (the oracle's own
# perturbation measurement), so the null vectors leave the bound untouched.
TIGHT = 1e-12
ACCEPT_TIGHT = 1.001e-12
PARITY = 1e-10
# At k = 0 with incompatible data (u_L^T F != 0) the solution of the
# projected system moves with the left null vectors, which both sides
# compute only to the rounding of S over the gap to its next singular value.
# The oracle measures that spread on the same input (null_vector_floor:
# null vectors from S perturbed at 2e-13, three samples); the bound is the
# larger of PARITY and ten times it.
FLOOR_FACTOR = 10


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _bound(o, F):
    """PARITY, or at k = 0 the larger of PARITY and FLOOR_FACTOR times the
    oracle's null-vector floor for this input."""
    if not o.singular:
        return PARITY
    return max(PARITY, FLOOR_FACTOR * solve.null_vector_floor(o, F, samples=3, tol=TIGHT))


def _oracle(prob, s_idx, q, tol=1e-10, method="dbj", zlabel=0):
    """The oracle's solve of one right-hand side; at the tight tolerance the
    result also carries the parity bound for this input (ref.bound)."""
    grid = smpm.Grid(prob.xb, prob.zb, prob.n)
    k = float(prob.kwaves[s_idx])
    o = schur.build(grid, kwave=k, zlabel=zlabel)
    g = {side: arr[s_idx, q] for side, arr in prob.g.items()} if prob.g else None
    F = smpm.rhs(grid, o.tau, prob.f[s_idx, q], g)
    ref = solve.dbj_solve(o, F, method=method, tol=tol)
    ref.bound = _bound(o, F) if tol == TIGHT else None
    return o, ref


def _gpu_solve(prob, precision=P.FP64, method=P.METHOD_DBJ, **kw):
    nrhs = prob.f.shape[1]
    s = P.Solver(prob.xb, prob.zb, prob.n - 1, kwaves=prob.kwaves, nrhs=nrhs, precision=precision,
                 method=method, **kw)
    f = _dev(prob.f.reshape(-1))
    g = _dev(P.pack_g(prob.g, s.info, nrhs)) if prob.g else None
    u, stats, status = s.solve(f, g)
    torch.cuda.synchronize()
    return s, u.cpu().numpy(), stats


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_c1_fp64_matches_oracle():
    p = workloads.c1()
    s, u, st = _gpu_solve(p)
    o, ref = _oracle(p, 0, 0)
    print("c1 stats", st, "oracle iters", ref.iters)
    assert st["rel_residual_max"] <= ACCEPT
    assert abs(st["iters_max"] - ref.iters) <= 1
    ue = p.exact - p.exact.mean()
    assert np.abs(u - ue).max() < 1e-9
    s, u, st = _gpu_solve(p, tol=TIGHT)
    o, ref = _oracle(p, 0, 0, tol=TIGHT)
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    assert abs(st["iters_max"] - ref.iters) <= 1
    assert _rel(u, ref.u) <= ref.bound


@pytest.mark.parametrize("mx,mz,n,stretch,with_g", [(6, 2, 5, False, True), (9, 3, 7, True, False),
                                                    (16, 2, 6, False, False), (5, 4, 4, True, True)])
def test_random_poisson_matches_oracle(mx, mz, n, stretch, with_g):
    p = workloads.random_problem(mx, mz, n, seed=mx + n, stretch=stretch, with_g=with_g)
    s, u, st = _gpu_solve(p)
    o, ref = _oracle(p, 0, 0)
    print("stats", st, "oracle iters", ref.iters)
    assert st["rel_residual_max"] <= ACCEPT
    assert abs(st["iters_max"] - ref.iters) <= 1
    s, u, st = _gpu_solve(p, tol=TIGHT)
    o, ref = _oracle(p, 0, 0, tol=TIGHT)
    print("tight", st, "oracle iters", ref.iters, "rel", _rel(u, ref.u))
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    assert abs(st["iters_max"] - ref.iters) <= 1
    assert _rel(u, ref.u) <= ref.bound


@pytest.mark.parametrize("mx,mz,n,k", [(4, 1, 2, 0.0), (4, 1, 3, 0.0), (5, 1, 4, 2.0), (4, 2, 2, 0.0),
                                        (6, 1, 5, 0.0)])
@pytest.mark.parametrize("precision", [P.FP64, P.FP32_IR])
def test_degenerate_grids_match_oracle(mx, mz, n, k, precision):
    # The smallest cases the method has: m_x = 4 at k = 0 (two block-Jacobi
    # blocks, the second one short), one element per strip (no z-interface:
    # an empty capacitance system), order 1 (n = 2 nodes per direction).
    p = workloads.random_problem(mx, mz, n, kwaves=(k,), seed=3 + mx + n, stretch=True, with_g=True)
    s, u, st = _gpu_solve(p, precision=precision, tol=TIGHT)
    o, ref = _oracle(p, 0, 0, tol=TIGHT)
    print(mx, mz, n, k, "stats", st, "oracle iters", ref.iters, "rel", _rel(u, ref.u))
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    assert _rel(u, ref.u) <= ref.bound


def test_fourier_modes_batched_match_oracle():
    p = workloads.fourier_problem("f", 4.0, 8, 2, 5, my=8, ly=2.0, seed=3)
    s, u, st = _gpu_solve(p, tol=TIGHT)
    u = u.reshape(p.nk, 2, p.r)
    assert st["instances"] == p.nk * 2
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    for m in range(p.nk):
        for q in range(2):
            o, ref = _oracle(p, m, q, tol=TIGHT)
            if np.abs(p.f[m, q]).max() == 0:
                assert np.abs(u[m, q]).max() == 0
                continue
            assert _rel(u[m, q], ref.u) <= ref.bound, (m, q)


@pytest.mark.parametrize("method,name", [(P.METHOD_DBJ, "dbj"), (P.METHOD_BJ, "bj"), (P.METHOD_SCHUR, "schur"),
                                         (P.METHOD_2LAS, "2las")])
@pytest.mark.parametrize("k", [0.0, 1.7])
def test_methods_match_oracle(method, name, k):
    # Table 1's four methods: same solution, iteration counts within one of
    # the oracle's (Householder GMRES on the same operator).
    p = workloads.random_problem(10, 2, 6, kwaves=(k,), seed=21, stretch=True, with_g=True)
    s, u, st = _gpu_solve(p, method=method)
    o, ref = _oracle(p, 0, 0, method=name)
    print(name, k, "stats", st, "oracle iters", ref.iters)
    assert st["rel_residual_max"] <= ACCEPT
    assert abs(st["iters_max"] - ref.iters) <= 1
    s, u, st = _gpu_solve(p, method=method, tol=TIGHT)
    o, ref = _oracle(p, 0, 0, method=name, tol=TIGHT)
    print(name, k, "tight", st, "oracle iters", ref.iters, "rel", _rel(u, ref.u))
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    assert abs(st["iters_max"] - ref.iters) <= 1
    assert _rel(u, ref.u) <= ref.bound


@pytest.mark.parametrize("method,name", [(P.METHOD_DBJ, "dbj"), (P.METHOD_2LAS, "2las")])
@pytest.mark.parametrize("k", [0.0, 1.7])
def test_per_element_deflation_matches_oracle(method, name, k):
    # Z with one column per element segment of an interface (d = (m_x - 1) m_z)
    p = workloads.random_problem(10, 3, 6, kwaves=(k,), seed=23, stretch=True, with_g=True)
    s, u, st = _gpu_solve(p, method=method, zlabel=1)
    assert s.info[0]["d"] == 9 * 3
    o, ref = _oracle(p, 0, 0, method=name, zlabel=1)
    print("zlabel 1", name, k, st, "oracle iters", ref.iters)
    assert st["rel_residual_max"] <= ACCEPT
    assert abs(st["iters_max"] - ref.iters) <= 1
    s, u, st = _gpu_solve(p, method=method, zlabel=1, tol=TIGHT)
    o, ref = _oracle(p, 0, 0, method=name, zlabel=1, tol=TIGHT)
    print("zlabel 1 tight", name, k, st, "oracle iters", ref.iters, "rel", _rel(u, ref.u))
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    assert _rel(u, ref.u) <= ref.bound


def test_per_element_deflation_fp32_refinement_and_operators():
    p = workloads.random_problem(12, 3, 7, seed=5, stretch=True)
    s, u, st = _gpu_solve(p, precision=P.FP32_IR, zlabel=1, tol=TIGHT)
    o, ref = _oracle(p, 0, 0, tol=TIGHT, zlabel=1)
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    assert _rel(u, ref.u) <= ref.bound
    s64 = P.Solver(p.xb, p.zb, p.n - 1, zlabel=1)
    x = np.random.default_rng(8).standard_normal(o.grid.k)
    xd = _dev(x)
    y = torch.empty_like(xd)
    s64.apply(P.OP_DEFLATE_P, 0, xd, y)
    assert _rel(y.cpu().numpy(), o.P_apply(x)) <= 1e-11
    s64.apply(P.OP_DEFLATE_Q, 0, xd, y)
    dq = y.cpu().numpy() - o.Q_apply(x)
    dq = dq - dq.mean()                    # Q x is defined modulo the interface constant (k = 0)
    assert np.abs(dq).max() <= 1e-9 * np.abs(o.Q_apply(x)).max()


def test_2las_fp32_refinement():
    p = workloads.random_problem(12, 3, 7, seed=5, stretch=True)
    s, u, st = _gpu_solve(p, precision=P.FP32_IR, method=P.METHOD_2LAS, tol=TIGHT)
    o, ref = _oracle(p, 0, 0, tol=TIGHT)
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    assert _rel(u, ref.u) <= ref.bound


@pytest.mark.parametrize("stretch", [False, True])
def test_fp16_scaled_refinement_reaches_fp64_solution(stretch):
    # FP16 operator tables with per-element row-segment scales (shared blocks
    # through the MFMA GEMM without stretch, distinct strips through the
    # streaming kernel with it), FP32 inner GMRES, FP64 refinement.
    p = workloads.random_problem(12, 3, 7, seed=6, stretch=stretch)
    s, u, st = _gpu_solve(p, precision=P.FP16S_IR, tol=TIGHT)
    o, ref = _oracle(p, 0, 0, tol=TIGHT)
    print("fp16s stats", st, "rel", _rel(u, ref.u))
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    assert st["sweeps_max"] >= 2
    assert _rel(u, ref.u) <= ref.bound
    # the FP16 matvec itself: within FP16 rounding of the FP64 product
    x = np.random.default_rng(4).standard_normal(o.grid.k)
    x32 = _dev(x).float()
    y32 = torch.empty_like(x32)
    s.schur_apply_all(x32, y32, P.FP16S_IR)
    assert _rel(y32.double().cpu().numpy(), o.S @ x) <= 5e-3


@pytest.mark.parametrize("n,mz,mx,precision", [(17, 32, 6, P.FP64), (17, 32, 6, P.FP32_IR), (22, 24, 5, P.FP64)])
def test_largest_supported_interface_half(n, mz, mx, precision):
    # N = n m_z at the limit (544 = 17 x 32) and the largest order (n = 22):
    # the widest operator blocks, the most row tiles per half, the longest K
    # in every GEMM schedule, the largest element blocks.  Too large for the
    # oracle's dense strip factorization, so the check is the defining
    # property (k > 0): u = A^-1 (F - E x_S) makes L u - F = E (b_S - S x_S),
    # so the residual of the oracle's sparse SMPM system L(k) u = F must be
    # the Schur tolerance times |b_S|, with b_S = B A^-1 F from a sparse
    # factorization of the strip-block-diagonal A(k).
    xb = np.linspace(0.0, 0.6 * mx, mx + 1)
    zb = np.concatenate([[0.0], np.cumsum(1.06 ** np.arange(mz))])
    zb = zb / zb[-1]
    k = 1.3
    rng = np.random.default_rng(n + mz)
    f = rng.uniform(0, 1, n * n * mx * mz)
    p = workloads.Problem("max", xb, zb, n, np.array([k]), f[None, None, :])
    s, u, st = _gpu_solve(p, precision=precision)
    assert s.info[0]["n"] * s.info[0]["mz"] == n * mz
    grid = smpm.Grid(xb, zb, n)
    tau = smpm.default_tau(grid)
    F = smpm.rhs(grid, tau, f)
    L = smpm.assemble_L(grid, tau, k)
    bS = smpm.assemble_B(grid, tau) @ spla.splu(smpm.assemble_A(grid, tau, k).tocsc()).solve(F)
    res = np.linalg.norm(L @ u - F) / np.linalg.norm(bS)
    print("max size", n, mz, st, "full residual / |b_S|", res)
    assert st["rel_residual_max"] <= ACCEPT
    assert res <= 1e-9


def _sched_problem():
    return workloads.random_problem(12, 4, 7, kwaves=(0.0, 1.3), nrhs=2, seed=31)


@pytest.fixture(scope="module")
def sched_refs():
    p = _sched_problem()
    return {(m, q): _oracle(p, m, q, tol=TIGHT)[1] for m in range(2) for q in range(2)}


@pytest.mark.parametrize("sched", [1, 2, 3, 4, 5])
def test_element_gemm_schedules_match_oracle(sched, monkeypatch, sched_refs):
    # Every element-interior GEMM schedule, pinned for all lists: split K, the
    # LDS-staged 64-row tile (XCD-ordered and plain) and the 32- and 16-row
    # tiles whose waves split K.  A uniform grid, so the elements between the
    # physical z-edges share one inverse and one item list; two systems of two
    # right-hand sides give items of 1 to 3 column tiles (the last one partial)
    # and one-column items in the same launch.  Both sides solve to 1e-12, so
    # at k > 0 the comparison sees the GEMMs' rounding, not the stopping
    # test's error.
    monkeypatch.setenv("SMPM_ELEM_SCHED", str(sched))
    p = _sched_problem()
    s, u, st = _gpu_solve(p, tol=TIGHT)
    assert all(v == sched for i in s.info for v in i["elem_sched"] if v >= 0)
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    u = u.reshape(2, 2, p.r)
    for (m, q), ref in sched_refs.items():
        assert _rel(u[m, q], ref.u) <= (ref.bound if m == 0 else 1e-11), (sched, m, q)


@pytest.mark.parametrize("sched,lst", [(1, 0), (2, 0), (0, 1), (6, 1), (7, 1), (8, 1)])
def test_rhs_gemm_item_lists_match_oracle(sched, lst, monkeypatch, sched_refs):
    # The Schur right-hand side b_S = (B A^-1) F~ as one GEMM over the strips,
    # pinned to a schedule on either item list: up to 32 windows per item, or
    # up to 16 (the narrow schedules 6 and 7 need it).  Two right-hand sides of
    # 10 interior strips give 20 windows per block side: one full 16-window
    # item and a partial one on the second list.
    monkeypatch.setenv("SMPM_RHS_GEMM", f"{sched},{lst}")
    p = _sched_problem()
    s, u, st = _gpu_solve(p, tol=TIGHT)
    assert all(i["rhs_gemm"] == [sched, 16 if lst else 32] for i in s.info)
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    u = u.reshape(2, 2, p.r)
    for (m, q), ref in sched_refs.items():
        assert _rel(u[m, q], ref.u) <= (ref.bound if m == 0 else 1e-11), (sched, lst, m, q)


@pytest.mark.parametrize("sched", [1, 2, 3, 4, 5])
def test_element_gemm_16_column_lists_match_oracle(sched, monkeypatch, sched_refs):
    # Each element-interior product as one launch over items of at most 16
    # columns (the products that have wider items), pinned to every schedule.
    monkeypatch.setenv("SMPM_ELEM_SCHED", str(sched))
    monkeypatch.setenv("SMPM_ELEM_ALT", "1")
    p = _sched_problem()
    s, u, st = _gpu_solve(p, tol=TIGHT)
    assert any(v == sched for i in s.info for v in i["elem_alt"])
    assert all(v in (sched, -1) for i in s.info for v in i["elem_alt"])
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    u = u.reshape(2, 2, p.r)
    for (m, q), ref in sched_refs.items():
        assert _rel(u[m, q], ref.u) <= (ref.bound if m == 0 else 1e-11), (sched, m, q)


@pytest.mark.parametrize("sched", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12])
@pytest.mark.parametrize("precision", [P.FP64, P.FP32_IR])
def test_shared_block_gemm_schedules_match_oracle(sched, precision, monkeypatch, sched_refs):
    # Every schedule of the shared-block S and M^-1 GEMMs, pinned for all lists
    # (the fused S M^-1 block included): split K over 16 or 8 waves, the
    # LDS-staged 64-row tile, XCD-ordered or plain, staging 32 or 64 K-values
    # per chunk, split K with a wave's whole K range in flight (lists of at
    # most 16 windows per item; wider lists run split K 8 under that id), and
    # the staged 128-row tile and the 64- / 128-row tiles whose waves split K.
    # FP32 refinement reaches the same FP64 solution.
    monkeypatch.setenv("SMPM_GEMM_SCHED", str(sched))
    p = _sched_problem()
    s, u, st = _gpu_solve(p, precision=precision, tol=TIGHT)
    assert all(v == sched for i in s.info for v in i["gemm_sched"] if v >= 0)
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    u = u.reshape(2, 2, p.r)
    for (m, q), ref in sched_refs.items():
        assert _rel(u[m, q], ref.u) <= (ref.bound if m == 0 else 1e-11), (sched, m, q)


@pytest.mark.parametrize("sched", [0, 1, 2, 6, 7, 8, 11, 12])
@pytest.mark.parametrize("precision", [P.FP64, P.FP32_IR])
def test_shared_block_gemm_16_window_lists_match_oracle(sched, precision, monkeypatch, sched_refs):
    # The S and M^-1 lists built again in items of at most 16 windows (the
    # narrow schedules' lists), pinned: the interior S blocks' 20 windows per
    # system become a full and a partial item.
    monkeypatch.setenv("SMPM_GEMM_SCHED", str(sched))
    monkeypatch.setenv("SMPM_GEMM_LIST", "1")
    p = _sched_problem()
    s, u, st = _gpu_solve(p, precision=precision, tol=TIGHT)
    assert all(v == sched for i in s.info for v in i["gemm_sched"] if v >= 0)
    assert any(v == 16 for i in s.info for v in i["gemm_list"])
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    u = u.reshape(2, 2, p.r)
    for (m, q), ref in sched_refs.items():
        assert _rel(u[m, q], ref.u) <= (ref.bound if m == 0 else 1e-11), (sched, m, q)


def _tall_problem():
    # N = 14 * 10 = 140 rows per half: two 128-row tiles (the second ragged),
    # three 64-row tiles, and K = 2N .. 8N spans several staged chunks and
    # K parts of every schedule.  k > 0: the solution does not move with the
    # null vectors, which at k = 0 on this order-13 grid are determined only
    # to about 4e-10 in u.
    return workloads.random_problem(8, 10, 14, kwaves=(1.3,), seed=41)


@pytest.fixture(scope="module")
def tall_ref():
    return _oracle(_tall_problem(), 0, 0, tol=TIGHT)[1]


@pytest.mark.parametrize("sched", [0, 2, 6, 8, 9, 10, 11, 12])
def test_shared_block_gemm_schedules_on_tall_blocks(sched, monkeypatch, tall_ref):
    monkeypatch.setenv("SMPM_GEMM_SCHED", str(sched))
    p = _tall_problem()
    s, u, st = _gpu_solve(p, tol=TIGHT)
    assert all(v == sched for i in s.info for v in i["gemm_sched"] if v >= 0)
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    assert _rel(u, tall_ref.u) <= tall_ref.bound, sched


@pytest.fixture(scope="module")
def table2_grid():
    # The m_x = 64 grid of the Table 2 comparison: 64 x 10 elements, order 9,
    # U[0, 1] forcing.  Its coarse matrix C is singular only to 1e-9 of |C|
    # (the rounding of S 1_Gamma), which a coarse inverse must not amplify.
    mx, mz, n = 64, 10, 10
    xb, zb = np.linspace(0.0, float(mx), mx + 1), np.linspace(0.0, 1.0, mz + 1)
    grid = smpm.Grid(xb, zb, n)
    o = schur.build(grid)
    f = np.random.default_rng(0).uniform(0.0, 1.0, n * n * mx * mz)
    F = smpm.rhs(grid, o.tau, f)
    its = {m: solve.dbj_solve(o, F, method=m, tol=1e-10, maxit=400).iters for m in ("dbj", "2las")}
    return xb, zb, n, f, o, its


@pytest.mark.parametrize("method", ["dbj", "2las"])
def test_deflation_iterations_on_table2_grid(method, table2_grid):
    xb, zb, n, f, o, its = table2_grid
    m = {"dbj": P.METHOD_DBJ, "2las": P.METHOD_2LAS}[method]
    s = P.Solver(xb, zb, n - 1, method=m, max_iter=400)
    _, st, status = s.solve(_dev(f))
    print(method, "GPU", st["iters_max"], "oracle", its[method])
    assert status == P.OK and abs(st["iters_max"] - its[method]) <= 1
    # P itself: C is singular only to its rounding, so u_C, and with it the
    # coarse projection, is determined to sigma_min(C) / sigma_{d-1}(C)
    # (6e-9 here); the two sides' P agree to that.
    sv = o.extra["C_svd"][1]
    x = np.random.default_rng(3).standard_normal(o.SZ.shape[0])
    y = torch.empty(x.size, dtype=torch.float64, device="cuda")
    s.apply(P.OP_DEFLATE_P, 0, _dev(x), y)
    assert _rel(y.cpu().numpy(), o.P_apply(x)) <= max(1e-11, sv[-1] / sv[-2])
    s.close()


@pytest.mark.parametrize("k", [0.0, 2.1])
def test_fp32_refinement_reaches_fp64_solution(k):
    p = workloads.random_problem(12, 3, 7, kwaves=(k,), seed=5, stretch=True)
    s, u, st = _gpu_solve(p, precision=P.FP32_IR, tol=TIGHT)
    o, ref = _oracle(p, 0, 0, tol=TIGHT)
    print("ir stats", st, "rel", _rel(u, ref.u))
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    assert st["sweeps_max"] >= 2
    assert _rel(u, ref.u) <= ref.bound


@pytest.mark.parametrize("k,inner_tol", [(0.0, 1e-4), (2.1, 1e-4), (0.0, 1e-6)])
def test_fp32_refinement_counts_match_oracle(k, inner_tol):
    # Sweeps and inner GMRES iterations of the refined form against the
    # oracle's emulation (operators and inner vectors rounded to FP32, the
    # same inner stopping rule max(inner_tol |r|, tol |b~| / 2)): sweeps
    # within one, the inner iterations summed over the sweeps within one per
    # sweep (the FP32 rounding of the two Arnoldi processes can move an
    # iteration from one sweep to the next).
    p = workloads.random_problem(12, 3, 7, kwaves=(k,), seed=5, stretch=True)
    s, u, st = _gpu_solve(p, precision=P.FP32_IR, inner_tol=inner_tol)
    grid = smpm.Grid(p.xb, p.zb, p.n)
    o = schur.build(grid, kwave=k)
    ref, sweeps, total = solve.refine_solve(o, smpm.rhs(grid, o.tau, p.f[0, 0]), inner_tol=inner_tol,
                                           floor=0.5)
    print("ir counts", st, "oracle sweeps", sweeps, "inner", ref.inner)
    assert ref.converged and st["rel_residual_max"] <= ACCEPT
    assert abs(st["sweeps_max"] - sweeps) <= 1
    assert abs(st["iters_total"] - total) <= sweeps


@pytest.mark.parametrize("batched", [False, True])
def test_repeated_fp64_solves_resume_after_a_short_prediction(batched):
    # An FP64 solve runs the previous solve's iteration count, then the tail
    # (epilogue, residual, recovery) and one check.  An easy right-hand side
    # first (few iterations predicted), then one that needs more: the loop
    # resumes after the tail and the tail runs again.
    if batched:
        p = workloads.fourier_problem("f", 4.0, 8, 2, 5, my=8, ly=2.0, seed=3)
        s = P.Solver(p.xb, p.zb, p.n - 1, kwaves=p.kwaves, nrhs=2, tune=False)
    else:
        p = workloads.random_problem(10, 3, 6, seed=17, stretch=True)
        s = P.Solver(p.xb, p.zb, p.n - 1, tune=False)
    f_hard = p.f.reshape(-1)
    f_easy = np.zeros_like(f_hard)
    if batched:   # per-mode counts differ from the random forcing's
        f_easy[::7] = 1.0
    # (one system: f = 0 stops at once, so the next solve predicts 0 iterations)
    its = []
    for f in (f_easy, f_hard, f_easy, f_hard):
        u, st, status = s.solve(_dev(f))
        torch.cuda.synchronize()
        assert status == P.OK
        assert st["rel_residual_max"] <= ACCEPT
        its.append(st["iters_max"])
    print("iterations", its)
    # the same right-hand side gives the same counts whatever came before,
    # and the two differ (so one of them resumes after its tail)
    assert its[0] == its[2] and its[1] == its[3] and its[0] != its[1]
    if not batched:   # the last (resumed) solve, at 1e-10 on both sides
        grid = smpm.Grid(p.xb, p.zb, p.n)
        o = schur.build(grid)
        ref = solve.dbj_solve(o, smpm.rhs(grid, o.tau, f_hard)).u
        assert _rel(u.cpu().numpy(), ref) <= 1e-9


@pytest.mark.parametrize("precision", [P.FP32_IR, P.FP16S_IR])
def test_repeated_refinement_solves(precision):
    # The second and later solves of a handle run the previous solve's sweeps
    # (and per-sweep inner iterations) without host checks, then check and go
    # on if needed: same right-hand side (exact prediction), then a harder one
    # (a 40x larger random part, prediction too short), then the first again.
    p = workloads.random_problem(12, 3, 7, seed=5, stretch=True)
    s = P.Solver(p.xb, p.zb, p.n - 1, precision=precision, tune=False, tol=TIGHT)
    f1 = p.f.reshape(-1)
    f2 = f1 + 40.0 * np.random.default_rng(9).standard_normal(f1.size)
    grid = smpm.Grid(p.xb, p.zb, p.n)
    o = schur.build(grid)
    refs = {}
    for name, f in (("f1", f1), ("f1", f1), ("f2", f2), ("f1", f1)):
        u, st, status = s.solve(_dev(f))
        torch.cuda.synchronize()
        if name not in refs:
            F = smpm.rhs(grid, o.tau, f)
            refs[name] = (solve.dbj_solve(o, F, tol=TIGHT).u, _bound(o, F))
        print(name, st, "rel", _rel(u.cpu().numpy(), refs[name][0]))
        assert status == P.OK
        assert st["rel_residual_max"] <= ACCEPT_TIGHT
        assert _rel(u.cpu().numpy(), refs[name][0]) <= refs[name][1]


@pytest.mark.parametrize("k", [0.0, 2.3])
def test_operator_applies_match_oracle(k):
    xb = np.array([0, 0.4, 0.9, 1.2, 1.9, 2.3, 2.8, 3.5])
    zb = np.array([0, 0.15, 0.45, 1.0])
    n = 6
    s = P.Solver(xb, zb, n - 1, kwaves=[k])
    grid = smpm.Grid(xb, zb, n)
    o = schur.build(grid, kwave=k)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(grid.k)
    xd = _dev(x)
    y = torch.empty_like(xd)
    for op, ref in ((P.OP_SCHUR, o.S @ x), (P.OP_BJINV, o.Minv_apply(x)), (P.OP_DEFLATE_P, o.P_apply(x))):
        s.apply(op, 0, xd, y)
        assert _rel(y.cpu().numpy(), ref) <= 1e-11, op
    s.apply(P.OP_DEFLATE_Q, 0, xd, y)
    dq = y.cpu().numpy() - o.Q_apply(x)     # Q x is defined modulo the interface constant (coarse gauge)
    if k == 0.0:
        dq = dq - dq.mean()
    assert np.abs(dq).max() <= 1e-9 * np.abs(o.Q_apply(x)).max()
    v = rng.standard_normal(grid.r)
    vd = _dev(v)
    yr = torch.empty_like(vd)
    s.apply(P.OP_AINV, 0, vd, yr)
    assert _rel(yr.cpu().numpy(), o.A_solve(v)) <= 1e-11
    yb = torch.empty_like(xd)
    s.apply(P.OP_B, 0, vd, yb)
    assert _rel(yb.cpu().numpy(), o.B @ v) <= 1e-13
    # FP32 tables: within single-precision rounding of the FP64 product
    x32 = xd.float()
    y32 = torch.empty_like(x32)
    s.apply(P.OP_SCHUR, 0, x32, y32, precision=P.FP32_IR)
    assert _rel(y32.double().cpu().numpy(), o.S @ x) <= 1e-4


def test_solve_is_bitwise_deterministic():
    p = workloads.random_problem(10, 2, 6, seed=11)
    s = P.Solver(p.xb, p.zb, p.n - 1)
    f = _dev(p.f.reshape(-1))
    u1, _, _ = s.solve(f)
    u2, _, _ = s.solve(f)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2)


def test_batch_of_uneven_problems():
    probs = workloads.c5(seed=0, nprob=4, scale=0.1)
    grids = [(p.xb, p.zb, p.n - 1, float(p.kwaves[0])) for p in probs]
    s = P.Solver(grids=grids, tol=TIGHT)
    f = _dev(np.concatenate([p.f.reshape(-1) for p in probs]))
    u, st, status = s.solve(f)
    assert st["rel_residual_max"] <= ACCEPT_TIGHT
    u = u.cpu().numpy()
    off = 0
    for i, p in enumerate(probs):
        o, ref = _oracle(p, 0, 0, tol=TIGHT)
        ui = u[off:off + p.r]
        off += p.r
        assert _rel(ui, ref.u) <= ref.bound, i


def test_notconv_and_nonfinite_statuses():
    p = workloads.random_problem(8, 2, 6, seed=2)
    s = P.Solver(p.xb, p.zb, p.n - 1, max_iter=2)
    f = _dev(p.f.reshape(-1))
    u, st, status = s.solve(f, check=False)
    assert status == P.ENOTCONV
    assert np.all(np.isfinite(u.cpu().numpy()))
    s2 = P.Solver(p.xb, p.zb, p.n - 1)
    fbad = f.clone()
    fbad[3] = float("nan")
    u, st, status = s2.solve(fbad, check=False)
    assert status == P.ENONFINITE


def test_loaded_handle_solves_bitwise_like_the_saved_one(tmp_path):
    p = workloads.random_problem(9, 3, 6, seed=31, stretch=True, with_g=True)
    s = P.Solver(p.xb, p.zb, p.n - 1, tune=False)
    path = str(tmp_path / "tables.bin")
    s.save(path)
    t = P.Solver(load_path=path, tune=False)
    f = _dev(p.f.reshape(-1))
    g = _dev(P.pack_g(p.g, s.info, 1))
    u1, st1, _ = s.solve(f, g)
    u2, st2, _ = t.solve(f, g)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2)
    assert st1["iters_max"] == st2["iters_max"]


def test_loaded_fourier_handle(tmp_path):
    xb, zb, n, my, ly = np.linspace(0, 3, 6), np.array([0.0, 0.4, 1.0]), 5, 6, 2.0
    s = P.Solver(xb, zb, n - 1, fourier=(my, ly), tune=False)
    path = str(tmp_path / "fourier.bin")
    s.save(path)
    t = P.Solver(load_path=path, tune=False)
    assert t.nsys == my // 2 + 1 and t.nrhs == 2
    f = _dev(np.random.default_rng(2).uniform(0, 1, (my, s.info[0]["r"])))
    u1, _, _ = s.solve_fourier(f)
    u2, _, _ = t.solve_fourier(f)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2)
