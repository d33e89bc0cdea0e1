"""The batched and large configurations at their full sizes.

Batched: 64 independent problems (N log-uniform in [5000, 200000], windows of
3, 2 and 1 features, 4 right-hand sides each, ell in {0.1, 0.2, 0.4}) solved
together, float32 products with float64 CG and residuals; every column
converges on the float64 residual, problems solved alone give the same bits,
and sampled rows of the exact operator confirm the solutions.

Large: N = 2e6 points of a 16-component Gaussian mixture in R^15 in five
windows of three features, at the fixed bandwidth M = 64, m = 6, n = 128;
float32 and float64 products on sampled rows against the direct sum.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import dev_cols, dev_rows, empty_cols, to_np

pytestmark = pytest.mark.gpu

F32, F64 = 1, 0


@pytest.fixture(scope="module")
def A():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2111_10140_amd import _lib
    _lib.load()
    return _lib


def test_batched_configuration_full(A):
    import torch
    probs = workloads.batched()
    assert len(probs) == 64 and all(p.nrhs == 4 for p in probs)
    plans = [A.anova_fastsum_plan_host(p.X, p.windows, A.make_params(p.ell, F32, target_err=1e-4))
             for p in probs]
    ys = [dev_cols(p.y) for p in probs]
    xs = [empty_cols(p.N, p.nrhs) for p in probs]
    infos = A.krr_cg_solve_batched(plans, ys, xs, [p.beta for p in probs], 1e-6, 3000)
    torch.cuda.synchronize()
    for inf in infos:
        assert all(i["converged"] and i["true_relres"] <= 1e-6 for i in inf)
    # problems solved alone give the same bits as in the batch
    for k in (0, 31, 63):
        x1 = empty_cols(probs[k].N, 4)
        A.krr_cg_solve(plans[k], ys[k], x1, probs[k].beta, 1e-6, 3000)
        torch.cuda.synchronize()
        assert np.array_equal(to_np(x1), to_np(xs[k]))
    # the exact operator on sampled rows of a few problems
    for k in (int(np.argmin([p.N for p in probs])), int(np.argmax([p.N for p in probs]))):
        p = probs[k]
        x = to_np(xs[k]).reshape(p.N, 4)
        rows = np.random.default_rng(k).choice(p.N, 64, replace=False)
        Kx = oracle.direct.anova_matvec(p.X, p.windows, p.ell, p.beta, x, rows=rows)
        res = np.max(np.abs(p.y[rows] - Kx), axis=0) / np.abs(x).sum(axis=0)
        print(f"problem {k} N={p.N} ell={p.ell}: sampled exact residual / ||x||_1 {res}")
        assert np.all(res <= 1e-4)
        # and the product itself on those rows
        a = p.alpha
        out = empty_cols(p.N, 4)
        A.anova_matvec(plans[k], dev_cols(a), out, p.beta)
        torch.cuda.synchronize()
        ref = oracle.direct.anova_matvec(p.X, p.windows, p.ell, p.beta, a, rows=rows)
        E = np.max(np.abs(to_np(out).reshape(p.N, 4)[rows] - ref), axis=0) / np.abs(a).sum(axis=0)
        assert np.all(E <= 1e-4) and np.all(E <= plans[k].err_estimate())
    for pl in plans:
        pl.destroy()


def test_large_configuration_sampled_rows(A):
    import torch
    p = workloads.large()
    assert p.N == 2_000_000 and len(p.windows) == 5
    X = dev_rows(p.X)
    a = dev_cols(p.alpha[:, 0])
    rows = np.random.default_rng(44).choice(p.N, 128, replace=False)
    ref = oracle.direct.anova_matvec(p.X, p.windows, p.ell, p.beta, p.alpha[:, 0], rows=rows)
    norm1 = np.abs(p.alpha[:, 0]).sum()
    errs = {}
    for prec in (F32, F64):
        plan = A.anova_fastsum_plan(X, p.windows, A.make_params(p.ell, prec, M=64, m=6, n=128))
        out = torch.empty_like(a)
        A.anova_matvec(plan, a, out, p.beta)
        torch.cuda.synchronize()
        E = float(np.max(np.abs(to_np(out)[rows] - ref)) / norm1)
        errs[prec] = (E, plan.err_estimate())
        plan.destroy()
    print(f"large configuration: E float32 {errs[F32]}, float64 {errs[F64]}")
    assert errs[F32][0] <= 1e-4 and errs[F32][0] <= errs[F32][1]
    assert errs[F64][0] <= 1e-8 and errs[F64][0] <= errs[F64][1]


def test_large_mixture_cg_float32_matches_float64(A):
    # the large configuration's distribution at N = 2e5: float32 products
    # with float64 residuals against the plain float64 path, same parameters
    p = workloads.large(N=200_000)
    X = dev_rows(p.X)
    xs = {}
    for prec in (F32, F64):
        plan = A.anova_fastsum_plan(X, p.windows, A.make_params(p.ell, prec, M=64, m=6, n=128))
        y = dev_cols(p.y[:, 0])
        x = empty_cols(p.N, 1)
        info = A.krr_cg_solve(plan, y, x, p.beta, 1e-6, 3000)
        print(prec, info)
        assert info[0]["converged"] and info[0]["true_relres"] <= 1e-6
        xs[prec] = to_np(x)
        plan.destroy()
    d = np.linalg.norm(xs[F32] - xs[F64]) / np.linalg.norm(xs[F64])
    print(f"relative difference float32 vs float64 solutions {d:.2e}")
    assert d <= 1e-4
