"""Pins for the oracle's Fourier-side functions (CPU only).

NDFTs are pinned by numpy.fft on equispaced nodes and by adjointness; the
analytic Gaussian coefficients by scipy quadrature; the sampled coefficients
(FFT of equidistant samples, Sec. 4.2) by the Poisson aliasing identity
b_k = sum_n c_{k+nM}; the Kaiser-Bessel transform by quadrature; the exact
fast-summation formula (Sec. 4.2, eq. fastsum) by the direct sum within the
closed-form truncation and image errors.
"""
import math

import numpy as np
import pytest
import scipy.integrate

import oracle
import workloads
from workloads import Window

F = oracle.fastsum


def test_ndft_on_grid_nodes_is_fft():
    M = 8
    u = np.arange(M) / M - 0.5  # equispaced nodes on the torus [-1/2, 1/2)
    rng = np.random.default_rng(0)
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    # adjoint NDFT at x_j = u_j: g_k = sum_j c_j e^{-2 pi i k x_j}
    g = F.adjoint_ndft(c, u[:, None], M)
    k = F.index_set(M)
    # e^{-2 pi i k (j/M - 1/2)} = e^{i pi k} e^{-2 pi i k j / M}
    ref = np.exp(1j * math.pi * k) * np.fft.fft(c)[k % M]
    np.testing.assert_allclose(g, ref, rtol=1e-12, atol=1e-12)
    # NDFT at the same nodes: f_j = sum_k fhat_k e^{2 pi i k x_j}
    fhat = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    f = F.ndft(fhat, u[:, None], M)
    full = np.zeros(M, complex)
    full[k % M] = fhat * np.exp(-1j * math.pi * k)
    np.testing.assert_allclose(f, M * np.fft.ifft(full), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_ndft_adjointness(d):
    M, N = 6, 13
    rng = np.random.default_rng(d)
    x = rng.uniform(-0.5, 0.5, (N, d))
    c = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    fhat = rng.standard_normal((M,) * d) + 1j * rng.standard_normal((M,) * d)
    lhs = np.vdot(F.ndft(fhat, x, M), c)          # <Phi fhat, c>
    rhs = np.vdot(fhat, F.adjoint_ndft(c, x, M))  # <fhat, Phi^* c>
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_gaussian_coefficients_by_quadrature():
    ell, h = 0.2, 1.3
    for k in [0, 1, 3, 7]:
        re = scipy.integrate.quad(lambda r: math.exp(-r * r / ell ** 2) * math.cos(2 * math.pi * k * r / h),
                                  -np.inf, np.inf, epsabs=1e-15, epsrel=1e-13)[0] / h
        assert F.gaussian_fourier_analytic(k, ell, h) == pytest.approx(re, rel=1e-10, abs=1e-16)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_sampled_coefficients_poisson_aliasing(d):
    ell, h, M = 0.15, 1.0, 16
    b = F.sampled_coefficients(ell, h, M, d, zero_nyquist=False)
    k = F.index_set(M)
    c1 = sum(F.gaussian_fourier_analytic(k + n * M, ell, h) for n in range(-6, 7))
    ref = c1
    for _ in range(d - 1):
        ref = np.multiply.outer(ref, c1)
    np.testing.assert_allclose(b, ref, rtol=1e-12, atol=1e-15)
    # zeroing any k_t = -M/2 leaves the rest unchanged
    bz = F.sampled_coefficients(ell, h, M, d)
    inner = (slice(1, None),) * d
    np.testing.assert_array_equal(bz[inner], b[inner])
    assert np.all(bz[(0,) + (slice(None),) * (d - 1)] == 0)


def test_sampled_trig_polynomial_interpolates_and_is_periodic():
    # the trigonometric polynomial with the FFT coefficients of M equidistant
    # samples reproduces the samples (Sec. 4.2) and has period h.
    ell, h, M = 0.3, 2.5, 32
    b = F.sampled_coefficients(ell, h, M, 1, zero_nyquist=False)
    k = F.index_set(M)
    r = np.array([0.0, 0.75, -0.75, 1.75, 3.25, 0.75 + h]).astype(float)
    T = (np.exp(2j * math.pi * np.outer(r, k) / h) @ b)
    samples = F.periodized_gaussian(np.arange(-M // 2, M // 2) * h / M, ell, h)
    Tj = np.exp(2j * math.pi * np.outer(np.arange(-M // 2, M // 2) * h / M, k) / h) @ b
    np.testing.assert_allclose(Tj.real, samples, rtol=1e-12, atol=1e-14)
    assert abs(T[1] - T[5]) < 1e-12 and abs(T[2] - T[3]) < 1e-12


def test_kaiser_bessel_transform_by_quadrature():
    m, sig = 4, 2.0
    b = F.kb_beta(m, sig)
    for xi in [0.0, 0.1, 0.25, 0.6, 1.3]:
        # substitute t = m sin(theta): the integrand's square-root edge
        # behaviour becomes smooth for the quadrature
        def f(th):
            t = m * math.sin(th)
            return float(F.kb_window(np.array([t]), m, b)[0]) * math.cos(2 * math.pi * xi * t) * m * math.cos(th)
        q = scipy.integrate.quad(f, -math.pi / 2, math.pi / 2, limit=400, epsabs=1e-13, epsrel=1e-13)[0]
        assert float(F.kb_window_hat(np.array([xi]), m, b)[0]) == pytest.approx(q, rel=1e-9, abs=1e-9)
    assert F.kb_window(np.array([m + 1e-9, -m - 0.5]), m, b).tolist() == [0.0, 0.0]


@pytest.mark.parametrize("dA", [1, 2, 3])
def test_fastsum_exact_matches_direct_sum(dA):
    # with h from the image rule and M large, the exact fast summation formula
    # equals the direct sum up to the closed-form truncation/image errors
    N, ell = 60, 0.12
    p = workloads.random_problem(N, dA, [tuple(range(dA))], ell, seed=10 + dA, eta=[1.0])
    D = 0.5
    h = max(2 * D, D + ell * math.sqrt(math.log(2 * dA / 1e-13)))
    M = 2 * int(math.ceil(h / (math.pi * ell) * math.sqrt(math.log(1e13)) + 1))
    b = F.sampled_coefficients(ell, h, M, dA)
    a = p.alpha[:, 0]
    s = F.fastsum_exact(a, p.X, b, h)
    ref = oracle.direct.anova_matvec(p.X, p.windows, ell, 0.0, a)
    assert np.max(np.abs(s - ref)) / np.abs(a).sum() < 1e-11
    # coarse M visibly fails: the test can tell a truncated sum apart
    b8 = F.sampled_coefficients(ell, h, 8, dA)
    s8 = F.fastsum_exact(a, p.X, b8, h)
    assert np.max(np.abs(s8 - ref)) / np.abs(a).sum() > 1e-6
