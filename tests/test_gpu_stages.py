"""Stage parity of one window's fast summation (Sec. 4.1 eqs. nfft and
adjnfft; Sec. 4.2 eq. fastsum), each stage of the HIP path through the C ABI
against a reference written from its definition:

* convolve: grid <- inverse DFT(b~ . DFT(grid)) with the per-axis multiplier
  b~_k = b_k / (phihat(k/n) / I0(b))^2 for |k| < M/2 (0 at k = -M/2 and
  outside), b_k the oracle's sampled coefficients of the periodised
  Gaussian and phihat the oracle's Kaiser-Bessel transform; the reference
  is numpy's FFT (unnormalised inverse: no 1/n, the normalisation lives in
  the multiplier).  Both the small-grid tap path (n <= 32 in 2-D and 3-D)
  and the FFT path (n >= 64, and every 1-D grid) are covered.
* gather: for a trigonometric polynomial f = sum_{k in I_M} fhat_k
  e^{2 pi i k.x}, the grid G_u = sum_k fhat_k / (phihat(k/n)/I0(b))^d
  e^{2 pi i k.(u/n - 1/2)} gathered at x~ reproduces the oracle's NDFT of
  fhat at x~ up to the window error of the NFFT.

Together with the spread stage test (against the adjoint NDFT) this splits
the product's error into its NFFT part and the kernel approximation.
Tolerances: the window error bound of the Kaiser-Bessel window at
oversampling sigma (Potts and Steidl's estimate for this window,
4 pi (sqrt(m) + m) (1 - 1/sigma)^(1/4) exp(-2 pi m sqrt(1 - 1/sigma)), per
unit of ||fhat||_1), plus the rounding of the working precision.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import dev_cols, dev_rows, to_np

pytestmark = pytest.mark.gpu

F32, F64 = 1, 0


@pytest.fixture(scope="module")
def A():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2111_10140_amd import _lib
    _lib.load()
    return _lib


def kb_bound(m: int, sigma: float) -> float:
    s = 1.0 - 1.0 / sigma
    return 4 * math.pi * (math.sqrt(m) + m) * s ** 0.25 * math.exp(-2 * math.pi * m * math.sqrt(s))


def axis_multiplier(ell, h, M, n, m):
    """b~ on the FFT index k = 0..n-1 (k >= n/2 standing for k - n)."""
    b1 = oracle.fastsum.sampled_coefficients(ell, h, M, 1)  # index k + M/2, k = -M/2..M/2-1
    beta = oracle.fastsum.kb_beta(m, n / M)
    i0 = oracle.fastsum.kb_window(np.array([0.0]), m, beta)[0]
    out = np.zeros(n)
    for k in range(n):
        ks = k if k < n // 2 else k - n
        if abs(ks) >= M // 2:
            continue
        ph = oracle.fastsum.kb_window_hat(np.array([ks / n]), m, beta)[0] / i0
        out[k] = b1[ks + M // 2] / (ph * ph)
    return out


@pytest.mark.parametrize("precision,d,M,n,m", [
    (F32, 3, 16, 32, 3),    # taps: x-y planes, then z (the headline's grid)
    (F32, 3, 32, 64, 4),    # FFT per axis
    (F32, 3, 64, 128, 6),   # FFT per axis at the paper's parameters
    (F32, 2, 12, 16, 3),    # taps, one plane
    (F32, 1, 48, 64, 4),    # 1-D: FFT
    (F32, 2, 128, 256, 4),  # 16 x 16 register transforms
    (F32, 1, 96, 128, 5),
    (F64, 3, 32, 64, 4),
    (F64, 2, 64, 128, 4),   # float64, 16 x 8 register transforms
    (F64, 3, 16, 32, 4),    # taps in float64
    (F64, 2, 24, 32, 4),
    (F64, 1, 12, 16, 3),    # 1-D, small n: FFT
])
def test_stage_convolve_matches_fft_times_multiplier(A, precision, d, M, n, m):
    import torch
    windows = [tuple(range(d))]
    p = workloads.random_problem(2000, d, windows, 0.15, seed=50 + d, eta=[1.0])
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows,
                                A.make_params(p.ell, precision, M=M, n=n, m=m))
    info = plan.info(0)
    assert (info.M, info.n, info.m) == (M, n, m)
    rng = np.random.default_rng(60 + n + d)
    g0 = rng.standard_normal((n,) * d)
    g = A.grid_tensor(plan, 0)
    g.copy_(torch.from_numpy(g0).to(g.dtype))
    A.anova_stage_convolve(plan, 0, g)
    torch.cuda.synchronize()
    got = to_np(g).astype(np.float64)
    b = axis_multiplier(p.ell, info.h, M, n, m)
    B = b
    for _ in range(d - 1):
        B = np.multiply.outer(B, b)
    g_in = to_np(torch.from_numpy(g0).to(g.dtype)).astype(np.float64)  # the values the GPU saw
    ref = np.real(np.fft.ifftn(np.fft.fftn(g_in) * B)) * float(n) ** d
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref)) / scale
    # float32: a few ulps of the largest value per pass and tap sum
    tol = 1e-5 if precision == F32 else 1e-12
    print(f"convolve d={d} n={n} prec={precision}: max rel err {err:.3e}")
    assert err <= tol


def hermitian_coefficients(rng, M, d):
    """Random fhat on I_M^d with fhat_{-k} = conj(fhat_k) and 0 where some
    k_t = -M/2, so that sum_k fhat_k e^{2 pi i k.x} is real."""
    f = rng.standard_normal((M,) * d) + 1j * rng.standard_normal((M,) * d)
    # index k + M/2; k -> -k maps index i to M - i (mod M), with i = 0 <-> -M/2
    idx = [(-np.arange(M)) % M for _ in range(d)]
    f = 0.5 * (f + np.conj(f[np.ix_(*idx)]))
    for t in range(d):
        sl = [slice(None)] * d
        sl[t] = 0
        f[tuple(sl)] = 0.0
    return f


@pytest.mark.parametrize("precision,N,d,M,n,m,h,per_cell", [
    (F64, 700, 3, 16, 32, 6, 1.0, 0),        # per-point kernel, float64
    (F32, 20000, 3, 16, 32, 6, 1.0, 1),      # matrix-core per-tile kernel (W = 12)
    (F32, 20000, 3, 16, 32, 3, 1.3334, 1),   # the headline's per-cell kernel (W = 6)
    (F32, 400000, 3, 64, 128, 6, 1.3334, 1),  # the paper's parameters, matrix-core kernel
    (F32, 3000, 2, 16, 32, 4, 1.0, None),    # 2-D
    (F64, 500, 1, 24, 64, 5, 1.0, 0),        # 1-D, float64
])
def test_stage_gather_matches_ndft(A, precision, N, d, M, n, m, h, per_cell):
    import torch
    p = workloads.random_problem(N, d, [tuple(range(d))], 0.1, seed=80 + d, eta=[0.75])
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows,
                                A.make_params(p.ell, precision, M=M, n=n, m=m, h=h, center=1))
    info = plan.info(0)
    if per_cell is not None:
        assert info.per_cell == per_cell
    rng = np.random.default_rng(90 + N)
    fhat = hermitian_coefficients(rng, M, d)
    k = np.arange(-M // 2, M // 2)
    beta = oracle.fastsum.kb_beta(m, n / M)
    i0 = oracle.fastsum.kb_window(np.array([0.0]), m, beta)[0]
    ph = oracle.fastsum.kb_window_hat(k / n, m, beta) / i0
    # grid point u sits at torus position u/n - 1/2: phase (-1)^k per dimension
    w1 = ((-1.0) ** k) / ph
    W = w1
    for _ in range(d - 1):
        W = np.multiply.outer(W, w1)
    spec = np.zeros((n,) * d, dtype=np.complex128)
    spec[np.ix_(*([k % n] * d))] = fhat * W
    G = np.fft.ifftn(spec) * float(n) ** d  # numpy index [u1, u2, u3]
    assert np.max(np.abs(G.imag)) <= 1e-12 * np.max(np.abs(G.real))
    grid_np = np.ascontiguousarray(G.real.transpose(*range(d)[::-1]))  # x fastest: [u3, u2, u1]
    g = A.grid_tensor(plan, 0)
    g.copy_(torch.from_numpy(grid_np).to(g.dtype))
    out = dev_cols(np.zeros(N))
    A.anova_stage_gather(plan, 0, g, out)
    torch.cuda.synchronize()
    got = to_np(out)
    # every row at small N, 400 seeded rows otherwise (the NDFT costs |I_M| per row)
    rows = np.arange(N) if N <= 5000 else np.sort(rng.choice(N, 400, replace=False))
    ref = 0.75 * oracle.fastsum.ndft(fhat, p.X[rows] / h, M).real
    err = np.max(np.abs(got[rows] - ref)) / (0.75 * np.abs(fhat).sum())
    tol = kb_bound(m, n / M) + (3e-6 if precision == F32 else 1e-13)
    print(f"gather d={d} M={M} n={n} m={m} prec={precision}: err {err:.3e} (gate {tol:.2e})")
    assert err <= tol


def direct_window_weights(X, h, n, m):
    """Per point and axis the grid indices u = floor(t) - m + 1 + a (mod n)
    and the window weights phi0(t - u) / phi0(0), a = 0 .. 2m-1, with
    t = n (x / h) + n / 2 (grid point u sits at torus position u/n - 1/2):
    the window sums of the spread and gather steps written out (Sec. 4.1)."""
    b = oracle.fastsum.kb_beta(m, 2.0)
    w0 = oracle.fastsum.kb_window(np.array([0.0]), m, b)[0]
    t = n * (X / h) + n / 2.0
    base = np.floor(t).astype(np.int64) - m + 1
    offs = np.arange(2 * m)
    u = base[:, :, None] + offs[None, None, :]            # (N, d, 2m)
    w = oracle.fastsum.kb_window(t[:, :, None] - u, m, b) / w0
    return u % n, w


@pytest.mark.parametrize("m", [2, 3])
def test_fp64_per_cell_stages_match_direct_window_sums(A, m):
    # float64 per-cell kernels (3-D, W = 2m <= 6, many points per cell):
    # the spread grid and the interpolated values against the window sums
    # evaluated point by point in float64.  The kernels' window polynomials
    # (degree 11) fit the window to about 2e-10 of its maximum, three
    # factors per weight: 1e-9 relative leaves room for that and nothing
    # else (a wrong offset, plane or lane sum is an O(1) error)
    import torch
    N, M, n, h = 20000, 16, 32, 1.0
    p = workloads.random_problem(N, 3, [(0, 1, 2)], 0.2, seed=60 + m, eta=[1.0])
    plan = A.anova_fastsum_plan(dev_rows(p.X), p.windows,
                                A.make_params(p.ell, F64, M=M, n=n, m=m, h=h, center=1))
    assert plan.info(0).per_cell == 1
    u, w = direct_window_weights(p.X, h, n, m)
    a = p.alpha[:, 0]
    # spread: grid[u3, u2, u1] = sum_j a_j w1 w2 w3
    g = A.grid_tensor(plan, 0)
    A.anova_stage_spread(plan, 0, dev_cols(a), g)
    torch.cuda.synchronize()
    got = to_np(g)
    ref = np.zeros((n, n, n))
    for i1 in range(2 * m):
        for i2 in range(2 * m):
            for i3 in range(2 * m):
                np.add.at(ref, (u[:, 2, i3], u[:, 1, i2], u[:, 0, i1]),
                          a * w[:, 0, i1] * w[:, 1, i2] * w[:, 2, i3])
    err_s = np.max(np.abs(got - ref)) / np.abs(ref).max()
    # gather: out_i = sum_u grid[u] w1 w2 w3 on an arbitrary grid
    G = np.random.default_rng(70 + m).standard_normal((n, n, n))
    g.copy_(torch.from_numpy(G))
    out = dev_cols(np.zeros(N))
    A.anova_stage_gather(plan, 0, g, out)
    torch.cuda.synchronize()
    got_g = to_np(out)
    ref_g = np.zeros(N)
    for i1 in range(2 * m):
        for i2 in range(2 * m):
            for i3 in range(2 * m):
                ref_g += G[u[:, 2, i3], u[:, 1, i2], u[:, 0, i1]] * \
                    w[:, 0, i1] * w[:, 1, i2] * w[:, 2, i3]
    err_g = np.max(np.abs(got_g - ref_g)) / np.abs(G).max()
    print(f"float64 per-cell m={m}: spread {err_s:.2e}, gather {err_g:.2e}")
    assert err_s <= 1e-9 and err_g <= 1e-9
