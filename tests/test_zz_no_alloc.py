"""The allocation-free product (static device work space) against
anova_matvec on the same plan and vectors: the same kernels, so the results
must agree bit for bit, and both must meet the float32 gate against the
oracle's direct sum.  Two calls in a row, the second on a smaller problem
(the static array keeps the first call's contents), then a column count
whose work space exceeds the maximum, which must be refused before anything
is launched.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import dev_cols, dev_rows, empty_cols, rel_err, to_np

pytestmark = pytest.mark.gpu

F32, F64 = 1, 0


@pytest.fixture(scope="module")
def A():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2111_10140_amd import _lib
    _lib.load()
    return _lib


def _both(A, plan, alpha, beta):
    import torch
    nrhs = 1 if alpha.ndim == 1 else alpha.shape[1]
    a = dev_cols(alpha)
    ref = empty_cols(alpha.shape[0], nrhs)
    out = empty_cols(alpha.shape[0], nrhs)
    out.fill_(np.nan)
    A.anova_matvec(plan, a, ref, beta)
    A.anova_matvec_noalloc(plan, a, out, beta)
    torch.cuda.synchronize()
    return to_np(out), to_np(ref)


def _cases(precision):
    if precision == F32:  # automatic parameters, three 3-D windows
        return [(workloads.feature_grouped(60_000, seed=31, nrhs=2), {}),
                (workloads.feature_grouped(3_000, seed=32), {})]
    # the plain float64 configuration's parameters (M = 32, m = 4, n = 64, h = 1)
    fixed = dict(M=32, m=4, n=64, h=1.0)
    return [(workloads.plain_fp64(20_000), fixed), (workloads.plain_fp64(2_000), fixed)]


@pytest.mark.parametrize("precision", [F32, F64])
def test_noalloc_equals_matvec_twice(A, precision):
    for p, kw in _cases(precision):  # the second call on a smaller problem
        print(f"noalloc: N={p.N} nrhs={p.alpha.shape[1]} precision={precision}", flush=True)
        plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows,
                                    A.make_params(p.ell, precision, **kw))
        alpha = p.alpha if p.alpha.shape[1] > 1 else p.alpha[:, 0]
        out, ref = _both(A, plan, alpha, p.beta)
        assert np.array_equal(out, ref), float(np.max(np.abs(out - ref)))
        if p.N <= 3_000:
            dref = oracle.direct.anova_matvec(p.X, p.windows, p.ell, p.beta, alpha)
            assert rel_err(out, dref, alpha) <= (1e-4 if precision == F32 else 1e-8)
        plan.destroy()


def test_noalloc_refuses_oversized_work_space(A):
    import torch
    p = workloads.feature_grouped(1_000_000, seed=33)
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows, A.make_params(p.ell, F32))
    # float32 work space: about 4 bytes per point, window and column
    nrhs = A.anova_matvec_noalloc_max_bytes() // (4 * p.N * len(p.windows)) + 1
    a = torch.zeros((nrhs, p.N), dtype=torch.float64, device="cuda").T
    out = torch.zeros_like(a)
    with pytest.raises(A.AnovaError) as ei:
        A.anova_matvec_noalloc(plan, a, out, p.beta)
    assert ei.value.status == A.ANOVA_E_INVALID
    assert "static work space" in str(ei.value)
    # nothing was launched: out keeps its zeros, and a fitting call still works
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0
    o1, r1 = _both(A, plan, p.alpha[:, 0], p.beta)
    assert np.array_equal(o1, r1)
    plan.destroy()


def test_noalloc_matrix_core_kernels(A):
    # 12-point supports (the paper's M = 64, m = 6, n = 128) on clustered
    # points, so that the windows run the matrix-core per-tile kernels, whose
    # regions then live in the static work space; two calls, the second on
    # a smaller problem, each bit for bit equal to the allocating product
    for N, seed in ((40_000, 61), (12_000, 62)):
        rng = np.random.default_rng(seed)
        X = np.ascontiguousarray(rng.uniform(0.0, 0.1, size=(N, 3)))
        a = rng.standard_normal(N)
        print(f"noalloc matrix-core: N={N}", flush=True)
        plan = A.anova_fastsum_plan(dev_rows(X), [workloads.Window((0, 1, 2), 1.0)],
                                    A.make_params(0.2, F32, M=64, m=6, n=128))
        assert plan.info(0).per_cell == 1 and plan.info(0).m == 6
        out, ref = _both(A, plan, a, 1.0)
        assert np.array_equal(out, ref), float(np.max(np.abs(out - ref)))
        plan.destroy()
