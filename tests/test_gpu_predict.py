"""Parity of the HIP prediction path (the fast sum with separate target and
source node sets, Sec. 4.2; evaluation of the trained model at test data,
Sec. 4.3) with the oracle's direct two-set sum.

Gate per column: E = ||s~ - s||_inf / ||alpha||_1 <= 1e-4 for float32 plans
(and within the plan's own per-entry error estimate, which holds for every
pair inside the box the plan was built for) and <= 1e-8 for the float64
plain-double parameters.  Inputs: seeded training points shaped like the
feature-grouped workload and test points from the same distribution or a
wider box, at sizes the oracle finishes in seconds; the full size is checked
on sampled rows.
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


def predict_plan(A, p, Z, precision, **kw):
    return A.anova_predict_plan(dev_rows(p.X), dev_rows(Z), p.windows,
                                A.make_params(p.ell, precision, **kw))


def gpu_predict(A, plan, alpha):
    import torch
    a = dev_cols(alpha)
    out = empty_cols(plan.Nz, 1 if alpha.ndim == 1 else alpha.shape[1])
    A.anova_predict(plan, a, out)
    torch.cuda.synchronize()
    return to_np(out)


def check(A, p, Z, plan, alpha, gate, rows=None):
    out = gpu_predict(A, plan, alpha)
    if rows is not None:
        out = out[rows]
    ref = oracle.direct.anova_predict(Z, p.X, p.windows, p.ell, alpha, rows=rows)
    e = rel_err(out, ref, alpha)
    est = plan.err_estimate()
    print(f"N={p.N} Nz={Z.shape[0]} E = {e:.3e} (estimate {est:.3e}); params",
          [(i.M, i.n, i.m, round(i.h, 3), i.per_cell) for i in
           (plan.info(l) for l in range(plan.P))], flush=True)
    assert e <= gate
    return e, est


def test_plain_fp64_parameters(A):
    # the plain-double case's parameters (M = 32, m = 4, n = 64, h = 1) on
    # 2000 training and 777 test points of one three-feature window
    p, Z = workloads.train_test(2000, 777, d=3, seed=21, ell=0.1)
    plan = predict_plan(A, p, Z, F64, M=32, m=4, n=64, h=1.0)
    check(A, p, Z, plan, p.alpha[:, 0], 1e-8)


def test_fp32_auto_feature_grouped(A):
    p, Z = workloads.train_test(20000, 7001, seed=22)
    plan = predict_plan(A, p, Z, F32, target_err=1e-4)
    e, est = check(A, p, Z, plan, p.alpha[:, 0], 1e-4)
    assert e <= est


@pytest.mark.parametrize("N,Nz", [(30000, 900), (900, 30000), (5000, 5000)])
@pytest.mark.parametrize("precision,gate", [(F32, 1e-4), (F64, 1e-9)])
def test_windows_of_one_two_three_features(A, N, Nz, precision, gate):
    # d_A = 3, 2, 1 windows; dense training points with sparse targets, the
    # reverse, and equal sizes (each side picks its own per-cell or per-point
    # kernels)
    rng = np.random.default_rng(23)
    X = rng.uniform(-0.25, 0.25, (N, 6))
    Z = rng.uniform(-0.25, 0.25, (Nz, 6))
    p = workloads.Problem("mixed", X, [workloads.Window((0, 1, 2), 0.5),
                                       workloads.Window((3, 4), 0.3),
                                       workloads.Window((5,), 0.2)],
                          0.25, 1.0, np.asfortranarray(rng.standard_normal((N, 1))),
                          np.asfortranarray(np.zeros((N, 1))))
    plan = predict_plan(A, p, Z, precision, target_err=gate)
    e, est = check(A, p, Z, plan, p.alpha[:, 0], gate)
    if precision == F32:
        assert e <= est


def test_targets_outside_the_training_box(A):
    # test points in a wider box than the training points: the plan's period
    # and centre cover both sets
    p, Z = workloads.train_test(8000, 3000, seed=24, test_lo=-0.4, test_hi=0.35)
    plan = predict_plan(A, p, Z, F32, target_err=1e-4)
    for l in range(plan.P):
        inf = plan.info(l)
        assert inf.extent >= 0.74
    e, est = check(A, p, Z, plan, p.alpha[:, 0], 1e-4)
    assert e <= est


def test_at_the_training_points_equals_the_product(A):
    # Z = X: the prediction is the unshifted product, computed by the same
    # kernels on identically binned points, hence bit for bit
    import torch
    p, _ = workloads.train_test(12000, 1, seed=25)
    plan = predict_plan(A, p, p.X, F32, target_err=1e-4)
    a = dev_cols(p.alpha[:, 0])
    pred = empty_cols(p.N)
    prod = empty_cols(p.N)
    A.anova_predict(plan, a, pred)
    A.anova_matvec(plan, a, prod, 0.0)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(pred), to_np(prod))


def test_columns_leading_dimensions_and_repeat(A):
    import torch
    p, Z = workloads.train_test(6000, 2500, seed=26)
    rng = np.random.default_rng(27)
    alpha = rng.standard_normal((p.N, 3))
    plan = predict_plan(A, p, Z, F32, target_err=1e-4)
    lda, ldo = p.N + 17, Z.shape[0] + 5
    abuf = torch.zeros((3, lda), dtype=torch.float64, device="cuda")
    abuf[:, :p.N] = torch.from_numpy(alpha.T.copy()).cuda()
    obuf = torch.full((3, ldo), 7.0, dtype=torch.float64, device="cuda")
    a, o = abuf[:, :p.N].T, obuf[:, :Z.shape[0]].T
    A.anova_predict(plan, a, o)
    torch.cuda.synchronize()
    first = to_np(obuf).copy()
    assert np.all(first[:, Z.shape[0]:] == 7.0)  # padding untouched
    ref = oracle.direct.anova_predict(Z, p.X, p.windows, p.ell, alpha)
    assert rel_err(first[:, :Z.shape[0]].T, ref, alpha) <= 1e-4
    # one column at a time gives the same values, and a repeat is identical
    for c in range(3):
        col = gpu_predict(A, plan, np.ascontiguousarray(alpha[:, c]))
        np.testing.assert_array_equal(col, first[c, :Z.shape[0]])
    A.anova_predict(plan, a, o)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(obuf), first)


def test_single_target_and_single_training_point(A):
    p, Z = workloads.train_test(4000, 1, seed=28)
    plan = predict_plan(A, p, Z, F32, target_err=1e-4)
    check(A, p, Z, plan, p.alpha[:, 0], 1e-4)
    q, Zq = workloads.train_test(1, 300, seed=29)
    plan = predict_plan(A, q, Zq, F64, target_err=1e-9)
    check(A, q, Zq, plan, q.alpha[:, 0], 1e-9)


def test_fit_then_predict(A):
    # the plan trains by CG (its points are X) and then predicts at Z: the
    # prediction of the GPU's own coefficients matches the oracle's sum
    import torch
    p, Z = workloads.train_test(10000, 4000, seed=30)
    plan = predict_plan(A, p, Z, F32, target_err=1e-4)
    y = dev_cols(p.y[:, 0])
    x = empty_cols(p.N)
    info = A.krr_cg_solve(plan, y, x, p.beta, 1e-6, 2000)
    assert info[0]["converged"]
    alpha = to_np(x)
    out = empty_cols(Z.shape[0])
    A.anova_predict(plan, x, out)
    torch.cuda.synchronize()
    ref = oracle.direct.anova_predict(Z, p.X, p.windows, p.ell, alpha)
    e = rel_err(to_np(out), ref, alpha)
    print(f"fit {info[0]['iters']} iterations, prediction E = {e:.3e}", flush=True)
    assert e <= 1e-4


def test_full_size_sampled_rows(A):
    # 1e6 training and 1e6 test points (the headline size, split as the
    # paper's experiments split their samples), float32, per-entry estimate
    # <= 1e-4; 512 sampled target rows against the oracle
    p, Z = workloads.train_test(1_000_000, 1_000_000, seed=31)
    plan = predict_plan(A, p, Z, F32, target_err=1e-4)
    rows = np.sort(np.random.default_rng(32).choice(Z.shape[0], 512, replace=False))
    e, est = check(A, p, Z, plan, p.alpha[:, 0], 1e-4, rows=rows)
    assert e <= est
    assert all(plan.info(l).per_cell for l in range(plan.P))


def test_host_plan_equals_device_plan(A):
    # the same plan built from host arrays gives the same predictions, bit for bit
    p, Z = workloads.train_test(9000, 4000, seed=33)
    prm = A.make_params(p.ell, F32, target_err=1e-4)
    dev = A.anova_predict_plan(dev_rows(p.X), dev_rows(Z), p.windows, prm)
    host = A.anova_predict_plan_host(p.X, Z, p.windows, prm)
    assert host.Nz == dev.Nz == Z.shape[0]
    for l in range(dev.P):
        a, b = dev.info(l), host.info(l)
        assert (a.M, a.n, a.m, a.h, a.center) == (b.M, b.n, b.m, b.h, b.center)
    np.testing.assert_array_equal(gpu_predict(A, host, p.alpha[:, 0]),
                                  gpu_predict(A, dev, p.alpha[:, 0]))
