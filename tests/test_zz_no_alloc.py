"""smpm_apply_noalloc (the operator applies that allocate nothing) against
smpm_apply on the same handle: two calls in a row, the second on a smaller
system, so the fixed device scratch is reused with a different layout."""
import numpy as np
import pytest

import paper_1512_01756_amd as P
from paper_1512_01756_amd import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load()


CASES = [  # (m_x, m_z, n, k, zlabel): a larger system first, then smaller ones
    (12, 3, 7, 0.0, 0),
    (6, 2, 4, 1.7, 0),
    (9, 3, 5, 0.0, 1),
    (5, 1, 3, 2.3, 1),
]

OPS = [(P.OP_SCHUR, P.FP64), (P.OP_SCHUR, P.FP32_IR), (P.OP_BJINV, P.FP64), (P.OP_BJINV, P.FP32_IR),
       (P.OP_DEFLATE_P, P.FP64), (P.OP_DEFLATE_Q, P.FP64)]


def test_noalloc_applies_match_smpm_apply():
    for mx, mz, n, k, zlabel in CASES:
        p = workloads.random_problem(mx, mz, n, kwaves=(k,), seed=mx + n, stretch=True)
        s = P.Solver(p.xb, p.zb, p.n - 1, kwaves=[k], zlabel=zlabel)
        kS = s.info[0]["kS"]
        x = torch.as_tensor(np.random.default_rng(mx * n).standard_normal(kS)).cuda()
        for op, prec in OPS:
            xx = x if prec == P.FP64 else x.float()
            y_ref = torch.empty_like(xx)
            y = torch.full_like(xx, float("nan"))
            s.apply(op, 0, xx, y_ref, precision=prec)
            s.apply_noalloc(op, 0, xx, y, precision=prec)
            torch.cuda.synchronize()
            a, b = y.double().cpu().numpy(), y_ref.double().cpu().numpy()
            print(mx, mz, n, k, zlabel, op, prec, np.abs(a - b).max())
            assert np.all(np.isfinite(a))
            if op == P.OP_DEFLATE_Q and k == 0.0:   # Q x is defined modulo the interface constant
                a, b = a - a.mean(), b - b.mean()
            assert np.abs(a - b).max() <= 1e-13 * max(np.abs(b).max(), 1e-300), (mx, op, prec)
        s.close()


def test_noalloc_rejects_bad_arguments():
    p = workloads.random_problem(6, 2, 4, seed=1)
    s = P.Solver(p.xb, p.zb, p.n - 1)
    x = torch.zeros(s.info[0]["kS"], dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for op, prec, xx, yy in ((P.OP_AINV, P.FP64, x, y), (P.OP_DEFLATE_P, P.FP32_IR, x, y),
                             (P.OP_SCHUR, P.FP64, x, x)):
        with pytest.raises(P.SmpmError) as e:
            s.apply_noalloc(op, 0, xx, yy, precision=prec)
        assert e.value.status == P.EINVAL
    with pytest.raises(P.SmpmError):
        s.apply_noalloc(P.OP_SCHUR, 3, x, y)
    s.close()
