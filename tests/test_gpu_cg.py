"""Parity of the HIP conjugate-gradient solver with the oracle.

The plain float64 case is solved to a relative residual of 1e-6 and checked
by the oracle's own direct product (the true residual of the GPU solution
against the exact K) and against the oracle's CG solution; float32-NFFT
solves report their residuals and are checked on the oracle's matvec within
the matvec tolerance.
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


def solve(A, plan, y, beta, tol, maxit, **kw):
    import torch
    yd = dev_cols(y)
    x = empty_cols(y.shape[0], 1 if y.ndim == 1 else y.shape[1])
    info = A.krr_cg_solve(plan, yd, x, beta, tol, maxit, **kw)
    torch.cuda.synchronize()
    return to_np(x), info


def test_plain_fp64_cg(A):
    p = workloads.plain_fp64()
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows,
                                A.make_params(p.ell, F64, M=32, m=4, n=64, h=1.0))
    y = p.y[:, 0]
    x, info = solve(A, plan, y, p.beta, 1e-6, 2000)
    print(info)
    assert info[0]["converged"] and info[0]["true_relres"] <= 1e-6
    # the oracle's exact operator: residual of the GPU solution
    apply = lambda v: oracle.direct.anova_matvec(p.X, p.windows, p.ell, p.beta, v)
    rr = np.linalg.norm(y - apply(x)) / np.linalg.norm(y)
    print(f"oracle relres of GPU solution {rr:.3e}")
    assert rr <= 1.0e-6 + 1e-7
    ref = oracle.cg.cg_solve(apply, y, 1e-10, 5000)
    dx = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    print(f"||x_gpu - x_oracle|| / ||x_oracle|| = {dx:.3e} (oracle iters {ref.iters}, gpu {info[0]['iters']})")
    assert dx <= 1e-5


def test_fp32_nfft_cg_feature_grouped(A):
    p = workloads.feature_grouped(20000, seed=21)
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows, A.make_params(p.ell, F32))
    y = p.y[:, 0]
    x, info = solve(A, plan, y, p.beta, 1e-6, 3000)
    print(info)
    assert info[0]["converged"]
    # convergence is declared on the float64 residual
    assert info[0]["true_relres"] <= 1e-6
    rows = np.random.default_rng(0).choice(p.N, 200, replace=False)
    Ax = oracle.direct.anova_matvec(p.X, p.windows, p.ell, p.beta, x, rows=rows)
    # sampled rows of the exact residual, relative to the matvec tolerance
    res = np.max(np.abs(y[rows] - Ax)) / np.abs(x).sum()
    print(f"sampled exact residual / ||x||_1 = {res:.3e}")
    assert res <= 1e-4


def test_fp32_products_fp64_residuals_large_kernel(A):
    # a wide kernel at N=60000: ||K|| ~ N * mean kernel value, so the float32
    # product's rounding error is far above tol * beta; the float64 residual
    # recomputation still takes CG to tol on the float64 operator
    p = workloads.random_problem(60000, 6, [(0, 1, 2), (3, 4, 5)], 0.33, nrhs=2, seed=24)
    X = dev_rows(p.X)
    plan = A.anova_fastsum_plan(X, p.windows, A.make_params(p.ell, F32, target_err=1e-4))
    x, info = solve(A, plan, p.y, 1.0, 1e-6, 3000)
    print(info)
    assert all(i["converged"] and i["true_relres"] <= 1e-6 for i in info)
    x = x.reshape(p.N, 2)
    # against the plain float64 fast path with the same parameters
    inf0 = plan.info(0)
    plan64 = A.anova_fastsum_plan(X, p.windows, A.make_params(p.ell, F64, M=inf0.M, m=inf0.m,
                                                              n=inf0.n, h=inf0.h))
    x64, info64 = solve(A, plan64, p.y, 1.0, 1e-6, 3000)
    x64 = x64.reshape(p.N, 2)
    dx = np.linalg.norm(x - x64, axis=0) / np.linalg.norm(x64, axis=0)
    print(f"iterations fp32+fp64 residual {[i['iters'] for i in info]}, fp64 "
          f"{[i['iters'] for i in info64]}; relative difference of solutions {dx}")
    assert np.all(dx <= 1e-4)
    # the exact operator on sampled rows
    rows = np.arange(0, p.N, 600)
    Kx = oracle.direct.anova_matvec(p.X, p.windows, p.ell, 1.0, x, rows=rows)
    res = np.max(np.abs(p.y[rows] - Kx), axis=0) / np.abs(x).sum(axis=0)
    assert np.all(res <= 1e-4)
    # float32 residuals (opt-out) hold no float64 windows: a smaller plan
    plan_s = A.anova_fastsum_plan(X, p.windows, A.make_params(p.ell, F32, target_err=1e-4,
                                                              residual=A.ANOVA_RESIDUAL_SAME))
    assert plan_s.footprint(1)[0] < plan.footprint(1)[0]


def test_multi_rhs_columns_independent(A):
    p = workloads.random_problem(3000, 6, [(0, 1, 2), (3, 4), (5,)], 0.2, nrhs=3, seed=22)
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows, A.make_params(p.ell, F64))
    X3, info3 = solve(A, plan, p.y, 1.0, 1e-8, 2000)
    # products and reductions are deterministic and columns iterate
    # independently, so each column equals its solve alone bitwise
    for c in range(3):
        x1, info1 = solve(A, plan, np.ascontiguousarray(p.y[:, c]), 1.0, 1e-8, 2000)
        assert info1[0]["iters"] == info3[c]["iters"]
        assert info1[0]["converged"] and info3[c]["converged"]
        assert np.array_equal(X3[:, c], x1)


def test_not_converged_and_invalid(A):
    p = workloads.random_problem(500, 3, [(0, 1, 2)], 0.2, seed=23, eta=[1.0])
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows, A.make_params(p.ell, F64))
    y = p.y[:, 0]
    x, info = solve(A, plan, y, 1.0, 1e-12, 1, allow_not_converged=True)
    assert info[0]["status"] == "E_NOT_CONVERGED" and info[0]["iters"] == 1
    assert not info[0]["converged"]
    with pytest.raises(A.AnovaError) as ei:
        solve(A, plan, y, 0.0, 1e-6, 10)
    assert ei.value.status == A.ANOVA_E_INVALID
    # zero right-hand side: converged at once with alpha = 0
    x, info = solve(A, plan, np.zeros(500), 1.0, 1e-6, 10)
    assert info[0]["converged"] and info[0]["iters"] == 0 and not x.any()


def _batched_problems():
    # uneven sizes, windows of 3, 2 and 1 features, 1-3 right-hand sides,
    # different widths (the batched configuration at reduced sizes)
    probs = []
    for i, (N, ell, nrhs) in enumerate([(3000, 0.2, 2), (800, 0.1, 1), (5000, 0.4, 3), (1700, 0.2, 1)]):
        probs.append(workloads.random_problem(N, 6, [(0, 1, 2), (3, 4), (5,)], ell, beta=1.0,
                                              nrhs=nrhs, seed=60 + i))
    return probs


@pytest.mark.parametrize("precision", [F32, F64])
def test_batched_solves_equal_alone_bitwise(A, precision):
    import torch
    probs = _batched_problems()
    plans = [A.anova_fastsum_plan(dev_rows(p.X), p.windows, A.make_params(p.ell, precision))
             for p in probs]
    ys = [dev_cols(p.y) for p in probs]
    xs = [empty_cols(p.N, p.nrhs) for p in probs]
    infos = A.krr_cg_solve_batched(plans, ys, xs, [q.beta for q in probs], 1e-6, 2000)
    torch.cuda.synchronize()
    for p, plan, y, x, inf in zip(probs, plans, ys, xs, infos):
        x1 = empty_cols(p.N, p.nrhs)
        inf1 = A.krr_cg_solve(plan, y, x1, p.beta, 1e-6, 2000)
        torch.cuda.synchronize()
        assert [i["iters"] for i in inf] == [i["iters"] for i in inf1]
        assert all(i["converged"] and i["true_relres"] <= 1e-5 for i in inf)
        assert np.array_equal(to_np(x), to_np(x1)), "a problem solved in the batch differs from alone"
        # the oracle's exact operator on a sample of rows
        rows = np.arange(0, p.N, max(1, p.N // 50))
        xn = to_np(x).reshape(p.N, p.nrhs)
        ref = oracle.direct.anova_matvec(p.X, p.windows, p.ell, p.beta, xn, rows=rows)
        res = np.max(np.abs(p.y[rows] - ref)) / np.abs(xn).sum(axis=0).min()
        assert res <= (1e-4 if precision == F32 else 1e-8)


def test_solves_join_and_leave_the_batch(A):
    # continuous batching: a solve that starts late joins the running list,
    # and the result equals the same solve run alone.  The float32 plans'
    # columns stop only on a recomputed residual (every 50th iteration), so
    # each solve runs at least 50 iterations and, joining 5 and 12
    # iterations apart, the list meets iterations in which only some of its
    # solves recompute their residual
    import torch
    probs = _batched_problems()
    plans = [A.anova_fastsum_plan(dev_rows(p.X), p.windows, A.make_params(p.ell, F32)) for p in probs]
    ys = [dev_cols(p.y) for p in probs]
    xs = [empty_cols(p.N, p.nrhs) for p in probs]
    live = [A.Solve(plans[0], ys[0], xs[0], 1.0, 1e-6, 2000)]
    A.krr_cg_iterate(live, 5)
    live.append(A.Solve(plans[1], ys[1], xs[1], 1.0, 1e-6, 2000))
    A.krr_cg_iterate(live, 7)
    live += [A.Solve(plans[2], ys[2], xs[2], 1.0, 1e-6, 2000),
             A.Solve(plans[3], ys[3], xs[3], 1.0, 1e-6, 2000)]
    done = []
    for _ in range(400):
        A.krr_cg_iterate(live, 3)
        still = []
        for s in live:
            act, _ = s.poll()
            (still if act else done).append(s)
        live = still
        if not live:
            break
    assert not live
    for s in done:
        s.finish()
    torch.cuda.synchronize()
    for k, (p, plan) in enumerate(zip(probs, plans)):
        x1 = empty_cols(p.N, p.nrhs)
        A.krr_cg_solve(plan, ys[k], x1, 1.0, 1e-6, 2000)
        torch.cuda.synchronize()
        assert np.array_equal(to_np(xs[k]), to_np(x1)), "joined late: differs from alone"
    for s in done:
        s.destroy()
