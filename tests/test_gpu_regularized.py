"""Parity of plans with the regularised kernel (Sec. 4.2: the kernel kept on
[-L, L], joined to its periodic continuation by a derivative-matching
polynomial on (L, h - L)) with the oracle's direct Gaussian sum.  The
regularised kernel equals the Gaussian for every pair of points, so the
plain definition is the oracle; the gates are the plan's own per-entry
estimates and the target errors.  The cases include a fixed period too
short for the plain periodisation (a kernel wider than the data), where
only the regularised plan meets the target."""
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


def product(A, plan, a, beta):
    import torch
    out = empty_cols(a.shape[0])
    A.anova_matvec(plan, dev_cols(a), out, beta)
    torch.cuda.synchronize()
    return to_np(out)


def check(A, p, plan, gate):
    a = p.alpha[:, 0]
    out = product(A, plan, a, p.beta)
    ref = oracle.direct.anova_matvec(p.X, p.windows, p.ell, p.beta, a)
    e = rel_err(out, ref, a)
    est = plan.err_estimate()
    print(f"{p.name} ell={p.ell}: E = {e:.3e}, estimate {est:.3e}, params",
          [(i.M, i.n, i.m, round(i.h, 4), round(i.err_images, 3)) for i in
           (plan.info(l) for l in range(plan.P))], flush=True)
    assert e <= gate and e <= est
    return e


def test_fixed_period_wide_kernel_fp64(A):
    # points in [-1/4, 1/4)^3 (extent 0.5), period fixed at 1.2, kernel
    # width 1: the periodised Gaussian's images are far from negligible
    p = workloads.random_problem(3000, 3, [(0, 1, 2)], 1.0, seed=70)
    with pytest.raises(A.AnovaError):
        A.anova_fastsum_plan(dev_rows(p.X), p.windows,
                             A.make_params(p.ell, F64, h=1.2, target_err=1e-6))
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows,
                                A.make_params(p.ell, F64, h=1.2, target_err=1e-6, reg_q=8))
    assert plan.info(0).err_images == 0.0
    check(A, p, plan, 1e-6)


@pytest.mark.parametrize("ell", [0.2, 1.0, 5.0])
def test_auto_period_fp32(A, ell):
    p = workloads.random_problem(20000, 6, [(0, 1, 2), (3, 4), (5,)], ell, seed=71)
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows,
                                A.make_params(p.ell, F32, target_err=1e-4, reg_q=8))
    check(A, p, plan, 1e-4)


@pytest.mark.parametrize("q", [2, 6, 12])
def test_fixed_parameters_fp64_orders(A, q):
    p = workloads.random_problem(2500, 3, [(0, 1), (2,)], 0.6, seed=72)
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows,
                                A.make_params(p.ell, F64, M=48, m=6, n=64, reg_q=q))
    check(A, p, plan, 1e-3)


def test_period_must_exceed_twice_the_extent(A):
    p = workloads.random_problem(500, 3, [(0, 1, 2)], 0.5, seed=73)
    with pytest.raises(A.AnovaError, match="twice the extent"):
        A.anova_fastsum_plan(dev_rows(p.X), p.windows,
                             A.make_params(p.ell, F64, h=0.9, reg_q=8))


def test_prediction_with_regularised_kernel(A):
    import torch
    p, Z = workloads.train_test(6000, 2000, d=6, seed=74, ell=1.5, test_lo=-0.3, test_hi=0.3)
    plan = A.anova_predict_plan(dev_rows(p.X), dev_rows(Z), p.windows,
                                A.make_params(p.ell, F32, target_err=1e-4, reg_q=8))
    out = empty_cols(Z.shape[0])
    A.anova_predict(plan, dev_cols(p.alpha[:, 0]), out)
    torch.cuda.synchronize()
    ref = oracle.direct.anova_predict(Z, p.X, p.windows, p.ell, p.alpha[:, 0])
    e = rel_err(to_np(out), ref, p.alpha[:, 0])
    print(f"prediction E = {e:.3e}, estimate {plan.err_estimate():.3e}", flush=True)
    assert e <= 1e-4 and e <= plan.err_estimate()


def test_headline_size_sampled_rows(A):
    # the benchmark's regularised leg: headline points (N = 1e6), reg_q = 8,
    # float32, per-entry estimate <= 1e-4; 512 sampled rows
    p = workloads.headline()
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows,
                                A.make_params(p.ell, F32, target_err=1e-4, reg_q=8))
    a = np.ascontiguousarray(p.alpha[:, 0])
    out = product(A, plan, a, p.beta)
    rows = np.sort(np.random.default_rng(75).choice(p.N, 512, replace=False))
    ref = oracle.direct.anova_matvec(p.X, p.windows, p.ell, p.beta, a, rows=rows)
    e = float(np.max(np.abs(out[rows] - ref)) / np.abs(a).sum())
    rel = float(np.max(np.abs(out[rows] - ref)) / np.max(np.abs(ref)))
    est = plan.err_estimate()
    assert rel <= 1e-4, rel
    print(f"N=1e6 reg_q=8: E = {e:.3e}, relative {rel:.3e}, estimate {est:.3e}, params",
          [(i.M, i.n, i.m, round(i.h, 4), i.per_cell) for i in
           (plan.info(l) for l in range(plan.P))], flush=True)
    assert e <= 1e-4 and e <= est
