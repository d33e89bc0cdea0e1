"""Pins for the oracle's conjugate gradients (CPU only): against
numpy.linalg.solve on the dense (K + beta I), finite termination on a tiny
system, and the monotone decrease of the energy-norm error that CG guarantees.
"""
import numpy as np

import oracle
import workloads


def _dense(p):
    K = oracle.direct.kernel_matrix(p.X, p.windows, p.ell)
    return K + p.beta * np.eye(p.N)


def test_cg_matches_library_solve():
    p = workloads.random_problem(300, 6, [(0, 1, 2), (3, 4, 5)], 0.2, beta=1.0, seed=7)
    A = _dense(p)
    y = p.y[:, 0]
    res = oracle.cg.cg_solve(lambda v: oracle.direct.anova_matvec(p.X, p.windows, p.ell, p.beta, v),
                             y, 1e-10, 1000)
    ref = np.linalg.solve(A, y)
    assert res.converged
    cond = np.linalg.cond(A)
    assert np.linalg.norm(res.x - ref) / np.linalg.norm(ref) <= cond * 1e-10
    assert res.true_relres < 1e-9


def test_cg_finite_termination_and_energy_decrease():
    p = workloads.random_problem(12, 3, [(0, 1, 2)], 0.3, beta=0.5, seed=8, eta=[1.0])
    A = _dense(p)
    y = p.y[:, 0]
    xs = np.linalg.solve(A, y)

    def apply(v):
        return A @ v

    # run CG step by step by re-solving with increasing maxit
    errs = []
    for k in range(1, 13):
        r = oracle.cg.cg_solve(apply, y, 0.0, k)
        e = r.x - xs
        errs.append(float(e @ A @ e))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) + 1e-28 for i in range(len(errs) - 1))
    # in exact arithmetic CG ends in at most N = 12 steps (here: to rounding)
    assert errs[-1] <= 1e-12 * float(xs @ A @ xs)


def test_cg_zero_rhs():
    r = oracle.cg.cg_solve(lambda v: 2 * v, np.zeros(5), 1e-6, 10)
    assert r.converged and r.iters == 0 and not r.x.any()
