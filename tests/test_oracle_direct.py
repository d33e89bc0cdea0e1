"""Pins for the oracle's direct summation (CPU only).

Each test checks the oracle against something other than itself: a library
routine (scikit-learn's RBF kernel under the paper's mapping gamma = 1/sigma^2,
numpy.linalg), brute force on tiny inputs, invariants of a Gaussian kernel
matrix, or closed-form special cases.  A plausible mistake (a dropped
diagonal, a factor 1/2 in the exponent, a wrong feature index, a missing
weight or shift) fails at least one of them.
"""
import math

import numpy as np
import pytest
from sklearn.metrics.pairwise import rbf_kernel

import oracle
import workloads
from workloads import Window

D = oracle.direct


def _prob(N=80, d=6, windows=((0, 1, 2), (3, 4), (5,)), ell=0.2, seed=0, eta=None):
    return workloads.random_problem(N, d, windows, ell, seed=seed, eta=eta)


def test_matches_sklearn_rbf_per_window():
    # Sec. 6 ties the paper's sigma to sklearn's gamma = 1/sigma^2, i.e.
    # exp(-gamma ||r||^2) = exp(-||r||^2/sigma^2).  The combined kernel is
    # sum_l eta_l K_l (Sec. 5).
    p = _prob(eta=[0.5, 0.3, 0.2])
    K = D.kernel_matrix(p.X, p.windows, p.ell)
    ref = sum(w.eta * rbf_kernel(p.X[:, list(w.feat)], gamma=1.0 / p.ell ** 2) for w in p.windows)
    np.testing.assert_allclose(K, ref, rtol=1e-14, atol=1e-15)


def test_matvec_matches_dense_library_product():
    p = _prob(N=150)
    alpha = np.random.default_rng(1).standard_normal((150, 3))
    ref = sum(w.eta * rbf_kernel(p.X[:, list(w.feat)], gamma=1.0 / p.ell ** 2)
              for w in p.windows) @ alpha + 0.7 * alpha
    out = D.anova_matvec(p.X, p.windows, p.ell, 0.7, alpha)
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13)


def test_brute_force_python_loop():
    rng = np.random.default_rng(2)
    N, d = 12, 4
    X = rng.uniform(-1, 1, (N, d))
    wins = [Window((2, 0), 0.25), Window((3,), 0.75)]
    ell, beta = 0.6, 0.3
    a = rng.standard_normal(N)
    ref = np.zeros(N)
    for i in range(N):
        s = beta * a[i]
        for j in range(N):
            k = 0.0
            for w in wins:
                r2 = sum((X[i, f] - X[j, f]) ** 2 for f in w.feat)
                k += w.eta * math.exp(-r2 / ell ** 2)
            s += k * a[j]
        ref[i] = s
    np.testing.assert_allclose(D.anova_matvec(X, wins, ell, beta, a), ref, rtol=1e-14, atol=1e-14)


def test_invariants_symmetry_diagonal_bounds_pd():
    p = _prob(N=120)
    K = D.kernel_matrix(p.X, p.windows, p.ell)
    eta_sum = sum(w.eta for w in p.windows)
    assert np.array_equal(K, K.T)
    np.testing.assert_allclose(np.diag(K), eta_sum, rtol=0, atol=1e-15)
    off = K[~np.eye(K.shape[0], dtype=bool)]
    assert off.min() > 0 and off.max() <= eta_sum
    # Gaussian kernels are positive definite for distinct points (Bochner)
    assert np.linalg.eigvalsh(K).min() > -1e-12
    # symmetry of the operator through the matvec itself: u^T K v = v^T K u
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(120), rng.standard_normal(120)
    Ku = D.anova_matvec(p.X, p.windows, p.ell, 0.0, u)
    Kv = D.anova_matvec(p.X, p.windows, p.ell, 0.0, v)
    assert abs(v @ Ku - u @ Kv) <= 1e-12 * (abs(v @ Ku) + 1)


def test_identical_points_and_limits():
    rng = np.random.default_rng(4)
    a = rng.standard_normal(40)
    wins = [Window((0, 1, 2), 0.4), Window((3,), 0.6)]
    # all points identical: every entry of K is sum(eta) = 1
    X = np.tile(rng.uniform(-1, 1, (1, 4)), (40, 1))
    np.testing.assert_allclose(D.anova_matvec(X, wins, 0.1, 0.0, a), a.sum(), rtol=1e-13)
    # ell -> infinity: K -> (sum eta) 1 1^T
    X = rng.uniform(-0.25, 0.25, (40, 4))
    np.testing.assert_allclose(D.anova_matvec(X, wins, 1e8, 0.0, a), a.sum(), rtol=1e-12)
    # ell -> 0 with distinct points: K -> (sum eta) I, plus the shift beta
    np.testing.assert_allclose(D.anova_matvec(X, wins, 1e-6, 2.5, a), 3.5 * a, rtol=1e-13)


def test_two_points_one_feature():
    # N = 2, d_A = 1: K = [[eta, eta e], [eta e, eta]] with e = exp(-r^2/ell^2)
    X = np.array([[0.0], [0.3]])
    K = D.kernel_matrix(X, [Window((0,), 0.5)], 0.2)
    e = math.exp(-(0.3 / 0.2) ** 2)
    np.testing.assert_allclose(K, [[0.5, 0.5 * e], [0.5 * e, 0.5]], rtol=1e-15)


def test_three_dim_window_is_kronecker_of_one_dim():
    # points on a tensor lattice: the 3-D Gaussian matrix is the Kronecker
    # product of the three 1-D Gaussian matrices (separability of exp).
    ax = [np.linspace(-0.2, 0.2, 4), np.linspace(-0.1, 0.25, 3), np.linspace(-0.25, 0.0, 5)]
    grid = np.stack(np.meshgrid(*ax, indexing="ij"), -1).reshape(-1, 3)
    K3 = D.kernel_matrix(grid, [Window((0, 1, 2), 1.0)], 0.15)
    K1 = [D.kernel_matrix(a[:, None], [Window((0,), 1.0)], 0.15) for a in ax]
    np.testing.assert_allclose(K3, np.kron(np.kron(K1[0], K1[1]), K1[2]), rtol=1e-13)


def test_window_linearity_and_feature_permutation():
    p = _prob(N=90, eta=[0.2, 0.5, 0.3])
    a = p.alpha[:, 0]
    total = D.anova_matvec(p.X, p.windows, p.ell, 0.0, a)
    parts = sum(D.anova_matvec(p.X, [Window(w.feat, 1.0)], p.ell, 0.0, a) * w.eta
                for w in p.windows)
    np.testing.assert_allclose(total, parts, rtol=1e-13, atol=1e-13)
    # relabelling features (permuting the columns of X and the window indices
    # consistently) leaves the kernel unchanged
    perm = np.array([4, 2, 5, 0, 3, 1])
    inv = np.argsort(perm)
    Xp = p.X[:, perm]
    wins_p = [Window(tuple(int(inv[f]) for f in w.feat), w.eta) for w in p.windows]
    np.testing.assert_allclose(D.anova_matvec(Xp, wins_p, p.ell, 0.0, a), total, rtol=1e-13)


def test_row_sampling_and_multi_rhs():
    p = _prob(N=200)
    A = np.random.default_rng(5).standard_normal((200, 3))
    full = D.anova_matvec(p.X, p.windows, p.ell, 1.3, A)
    rows = [0, 17, 199, 3]
    sub = D.anova_matvec(p.X, p.windows, p.ell, 1.3, A, rows=rows)
    np.testing.assert_array_equal(sub, full[rows])
    for c in range(3):
        np.testing.assert_array_equal(D.anova_matvec(p.X, p.windows, p.ell, 1.3, A[:, c]), full[:, c])


def test_shift_is_exact():
    p = _prob(N=60)
    a = p.alpha[:, 0]
    d = D.anova_matvec(p.X, p.windows, p.ell, 2.0, a) - D.anova_matvec(p.X, p.windows, p.ell, 0.0, a)
    np.testing.assert_allclose(d, 2.0 * a, rtol=1e-12, atol=1e-12)


def test_golden_figure_gaussian_value():
    # Consistency of the periodisation figure's printed ticks, not an
    # independent pin of the oracle: the figure marks the Gaussian at r = -L
    # and r = L with value 0.2821 (4 digits) but does not print its width;
    # sigma = 2/3 is the width that gives 0.2821 at L = 0.75, so the value
    # check only confirms the kernel convention exp(-r^2/sigma^2) (no factor
    # 1/2, which would give 0.5311).  The ticks fix the period h = 2 (h/2) =
    # 2.5, and the other marked points are the images -L + h and L + h.
    import json
    import os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fastsum_figure.json")))
    L = fx["ticks"]["L"]
    h = 2 * fx["ticks"]["h/2"]
    assert fx["ticks"]["3h/2"] == pytest.approx(1.5 * h)
    X = np.array([[0.0], [L], [-L]])
    K = D.kernel_matrix(X, [Window((0,), 1.0)], 2.0 / 3.0)
    for r, val in fx["marked_points"]:
        # reduce the marked abscissa to the cell [-h/2, h/2)
        rr = (r + h / 2) % h - h / 2
        assert abs(abs(rr) - L) < 1e-12
        assert round(K[0, 1], 4) == val and round(K[0, 2], 4) == val
    # the convention with a factor 1/2 does not reproduce the printed value
    assert round(float(np.exp(-L ** 2 / (2 * (2.0 / 3.0) ** 2))), 4) != fx["marked_points"][0][1]


# ---------------------------------------------------------------- prediction
# s(z_i) = sum_j alpha_j kappa(z_i, x_j) over two node sets (Sec. 4.2,
# eq. kernelsum; Sec. 4.3 evaluates the trained model at test points so).

def test_predict_matches_library_rectangular_kernel():
    p = _prob(N=120)
    rng = np.random.default_rng(11)
    Z = rng.uniform(-0.3, 0.3, (45, p.X.shape[1]))
    alpha = rng.standard_normal((120, 2))
    ref = sum(w.eta * rbf_kernel(Z[:, list(w.feat)], p.X[:, list(w.feat)], gamma=1.0 / p.ell ** 2)
              for w in p.windows) @ alpha
    out = D.anova_predict(Z, p.X, p.windows, p.ell, alpha)
    assert out.shape == (45, 2)
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13)


def test_predict_at_the_training_points_is_the_unshifted_product():
    # the special case Z = X of the two-set sum is the product K alpha
    p = _prob(N=90)
    alpha = np.random.default_rng(12).standard_normal(90)
    out = D.anova_predict(p.X, p.X, p.windows, p.ell, alpha)
    ref = D.anova_matvec(p.X, p.windows, p.ell, 0.0, alpha)
    np.testing.assert_allclose(out, ref, rtol=1e-15, atol=1e-15)


def test_predict_single_training_point_closed_form():
    # one training point x0 with alpha = 2: s(z) = 2 sum_l eta_l exp(-r_l^2/ell^2)
    ell = 0.3
    x0 = np.array([[0.1, -0.2, 0.05, 0.0, 0.2]])
    wins = [Window((0,), 0.5), Window((1, 2), 0.3), Window((4,), 0.2)]
    Z = np.repeat(x0, 5, axis=0)
    Z[1, 0] += ell                     # r = ell in window 0
    Z[2, 1] += ell / math.sqrt(2.0)    # r = ell in window 1, split over two features
    Z[2, 2] -= ell / math.sqrt(2.0)
    Z[3, 3] += 5.0                     # feature 3 is in no window
    Z[4, :] += 10.0                    # far from x0 in every window
    s = D.anova_predict(Z, x0, wins, ell, np.array([2.0]))
    e1 = math.exp(-1.0)
    expect = [2.0, 2.0 * (0.5 * e1 + 0.5), 2.0 * (0.7 + 0.3 * e1), 2.0, 0.0]
    np.testing.assert_allclose(s, expect, rtol=1e-14, atol=1e-300)


def test_predict_adjoint_identity():
    # gamma^T K(Z, X) alpha = alpha^T K(X, Z) gamma: a transposed operand or an
    # index taken from the wrong set fails this
    rng = np.random.default_rng(13)
    wins = [Window((0, 2), 0.6), Window((1,), 0.4)]
    X = rng.uniform(-0.25, 0.25, (70, 3))
    Z = rng.uniform(-0.25, 0.25, (33, 3))
    a, g = rng.standard_normal(70), rng.standard_normal(33)
    lhs = g @ D.anova_predict(Z, X, wins, 0.15, a)
    rhs = a @ D.anova_predict(X, Z, wins, 0.15, g)
    assert abs(lhs - rhs) <= 1e-13 * (np.abs(g).sum() * np.abs(a).sum())


def test_predict_rows_and_columns():
    p = _prob(N=64)
    rng = np.random.default_rng(14)
    Z = rng.uniform(-0.25, 0.25, (40, p.X.shape[1]))
    alpha = rng.standard_normal((64, 3))
    full = D.anova_predict(Z, p.X, p.windows, p.ell, alpha)
    rows = [39, 0, 17, 17]
    np.testing.assert_array_equal(D.anova_predict(Z, p.X, p.windows, p.ell, alpha, rows=rows),
                                  full[rows])
    for c in range(3):
        np.testing.assert_array_equal(D.anova_predict(Z, p.X, p.windows, p.ell, alpha[:, c]),
                                      full[:, c])
    with pytest.raises(IndexError):
        D.anova_predict(Z, p.X, p.windows, p.ell, alpha, rows=[40])
