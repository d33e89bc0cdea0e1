"""Parity of the HIP shifted CG (one solve for every lambda of the
regularisation grid, Sec. 6) with the oracle.

Each shift's solution must satisfy what a solve of its own system satisfies:
the plain float64 case is checked on the oracle's exact operator (true
residual) and against numpy's dense solve of (K + lambda I) alpha = y with
the oracle's kernel matrix; float32-NFFT solves converge on the float64
residual, match the GPU's single-shift solves of the same systems, and are
checked on sampled rows of the oracle's product within the product
tolerance.  The paper's grid is lambda in {1, 10, 100, 1000}.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import dev_cols, dev_rows, empty_cols, to_np

pytestmark = pytest.mark.gpu

F32, F64 = 1, 0
GRID = [1.0, 10.0, 100.0, 1000.0]


@pytest.fixture(scope="module")
def A():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2111_10140_amd import _lib
    _lib.load()
    return _lib


def solve_shifts(A, plan, y, shifts, tol, maxit, **kw):
    import torch
    yd = dev_cols(y)
    x = empty_cols(y.shape[0], len(shifts))
    info = A.krr_cg_solve_shifts(plan, yd, x, shifts, tol, maxit, **kw)
    torch.cuda.synchronize()
    return to_np(x).reshape(y.shape[0], len(shifts)), info


def solve_one(A, plan, y, beta, tol, maxit):
    import torch
    x = empty_cols(y.shape[0])
    info = A.krr_cg_solve(plan, dev_cols(y), x, beta, tol, maxit)
    torch.cuda.synchronize()
    return to_np(x), info


def test_plain_fp64_grid_against_dense_solves(A):
    p = workloads.plain_fp64()
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows,
                                A.make_params(p.ell, F64, M=32, m=4, n=64, h=1.0))
    y = p.y[:, 0]
    shifts = GRID
    x, info = solve_shifts(A, plan, y, shifts, 1e-6, 3000)
    print(info, flush=True)
    K = oracle.direct.kernel_matrix(p.X, p.windows, p.ell)
    for s, lam in enumerate(shifts):
        assert info[s]["converged"] and info[s]["true_relres"] <= 1e-6
        apply = lambda v: oracle.direct.anova_matvec(p.X, p.windows, p.ell, lam, v)
        rr = np.linalg.norm(y - apply(x[:, s])) / np.linalg.norm(y)
        ref = np.linalg.solve(K + lam * np.eye(p.N), y)
        dx = np.linalg.norm(x[:, s] - ref) / np.linalg.norm(ref)
        print(f"lambda {lam}: iters {info[s]['iters']}, oracle relres {rr:.3e}, "
              f"||x - x_dense|| / ||x_dense|| = {dx:.3e}", flush=True)
        # the exact operator's residual: tol plus the product's own error
        assert rr <= 1e-6 + 1e-7
        assert dx <= 1e-5
    # larger shifts converge in no more shared iterations than the base
    assert info[-1]["iters"] <= info[0]["iters"]


def test_fp32_grid_matches_single_shift_solves(A):
    p = workloads.feature_grouped(20000, seed=41)
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows, A.make_params(p.ell, F32))
    y = p.y[:, 0]
    x, info = solve_shifts(A, plan, y, GRID, 1e-6, 3000)
    print(info, flush=True)
    rows = np.random.default_rng(42).choice(p.N, 200, replace=False)
    for s, lam in enumerate(GRID):
        assert info[s]["converged"] and info[s]["true_relres"] <= 1e-6
        one, inf1 = solve_one(A, plan, y, lam, 1e-6, 3000)
        d = np.linalg.norm(x[:, s] - one) / np.linalg.norm(one)
        Ax = oracle.direct.anova_matvec(p.X, p.windows, p.ell, lam, x[:, s], rows=rows)
        res = np.max(np.abs(y[rows] - Ax)) / np.abs(x[:, s]).sum()
        print(f"lambda {lam}: shared+refined iters {info[s]['iters']}, alone "
              f"{inf1[0]['iters']}; ||x - x_alone|| / ||x_alone|| = {d:.3e}; sampled exact "
              f"residual / ||x||_1 = {res:.3e}", flush=True)
        assert d <= 2e-3
        assert res <= 1e-4


def test_order_repeats_and_single_shift(A):
    # columns follow the caller's order; a repeated lambda gives identical
    # columns; one shift is plain CG on that system
    p = workloads.feature_grouped(8000, seed=43)
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows, A.make_params(p.ell, F64))
    y = p.y[:, 0]
    shifts = [100.0, 1.0, 10.0, 1.0]
    x, info = solve_shifts(A, plan, y, shifts, 1e-8, 3000)
    np.testing.assert_array_equal(x[:, 1], x[:, 3])
    for s, lam in enumerate(shifts):
        assert info[s]["converged"] and info[s]["true_relres"] <= 1e-8
        one, _ = solve_one(A, plan, y, lam, 1e-10, 5000)
        assert np.linalg.norm(x[:, s] - one) / np.linalg.norm(one) <= 1e-6
    x1, info1 = solve_shifts(A, plan, y, [10.0], 1e-8, 3000)
    assert info1[0]["converged"]
    assert np.linalg.norm(x1[:, 0] - x[:, 2]) / np.linalg.norm(x[:, 2]) <= 1e-6


def test_padded_columns_zero_rhs_and_limits(A):
    import torch
    p = workloads.feature_grouped(3000, seed=44)
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows, A.make_params(p.ell, F64))
    y = dev_cols(p.y[:, 0])
    ld = p.N + 9
    buf = torch.full((3, ld), 5.0, dtype=torch.float64, device="cuda")
    info = A.krr_cg_solve_shifts(plan, y, buf[:, :p.N].T, [1.0, 10.0, 100.0], 1e-8, 3000)
    torch.cuda.synchronize()
    b = to_np(buf)
    assert np.all(b[:, p.N:] == 5.0)  # padding untouched
    assert all(i["converged"] for i in info)
    # y = 0: alpha = 0, converged without iterating
    z = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    out = empty_cols(p.N, 2)
    info = A.krr_cg_solve_shifts(plan, z, out, [1.0, 10.0], 1e-8, 100)
    torch.cuda.synchronize()
    assert np.all(to_np(out) == 0.0) and all(i["converged"] and i["iters"] == 0 for i in info)
    # too few iterations: NOT_CONVERGED with the last iterates
    out = empty_cols(p.N, 2)
    info = A.krr_cg_solve_shifts(plan, y, out, [1.0, 10.0], 1e-12, 3,
                                 allow_not_converged=True)
    assert any(not i["converged"] for i in info)
    assert info[0]["status"] == "E_NOT_CONVERGED"
    with pytest.raises(A.AnovaError):
        A.krr_cg_solve_shifts(plan, y, empty_cols(p.N, 2), [1.0, -1.0], 1e-8, 10)


def test_headline_size_grid(A):
    # the benchmark's grid at N = 1e6 (feature-grouped, float32 plan, tol
    # 1e-6): every shift against its single-shift solve and 128 sampled rows
    # of the oracle's exact product
    p = workloads.feature_grouped(1_000_000, seed=2)
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows, A.make_params(p.ell, F32))
    y = p.y[:, 0]
    x, info = solve_shifts(A, plan, y, GRID, 1e-6, 5000)
    rows = np.sort(np.random.default_rng(45).choice(p.N, 128, replace=False))
    for s, lam in enumerate(GRID):
        assert info[s]["converged"] and info[s]["true_relres"] <= 1e-6
        one, _ = solve_one(A, plan, y, lam, 1e-6, 5000)
        d = np.linalg.norm(x[:, s] - one) / np.linalg.norm(one)
        Ax = oracle.direct.anova_matvec(p.X, p.windows, p.ell, lam, x[:, s], rows=rows)
        res = np.max(np.abs(y[rows] - Ax)) / np.abs(x[:, s]).sum()
        print(f"N=1e6 lambda {lam}: iters {info[s]['iters']}, ||x - x_alone|| / ||x_alone|| "
              f"= {d:.3e}, sampled exact residual / ||x||_1 = {res:.3e}", flush=True)
        assert d <= 2e-3
        assert res <= 1e-4
