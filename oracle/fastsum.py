"""Oracle pieces for the Fourier side of the method, in numpy float64.

Test infrastructure only.  Each function is a plain definition:

* ``ndft``            f_j = sum_{k in I_M} fhat_k exp(+2 pi i k.x_j)   (Sec. 4.1, eq. nfft)
* ``adjoint_ndft``    g_k = sum_j c_j exp(-2 pi i k.x_j), k in I_M      (Sec. 4.1, eq. adjnfft)
* ``index_set``       I_M = {-M/2, ..., M/2-1}^d                         (Sec. 4.1)
* ``sampled_coefficients``  the Fourier coefficients of the h-periodic
  kernel obtained by the ordinary FFT of M equidistant samples per dimension
  (Sec. 4.2, the sentence after the definition of the smooth periodisation).
  The kernel is periodised by summing its periodic images; with the period
  chosen so that the Gaussian has decayed below the working precision at the
  edge of the cell, this periodisation is already smooth, so the boundary
  polynomial p of Sec. 4.2 is not needed (reading stated in the design notes).
  Coefficients with some k_t = -M/2 are set to zero so that the trigonometric
  approximation is real and even.
* ``gaussian_fourier_analytic``  c_k of the h-periodised Gaussian,
  (sqrt(pi) ell / h)^d exp(-pi^2 ell^2 |k|^2 / h^2), by Poisson summation (not
  printed in the paper; a textbook identity).
* ``fastsum_exact``   s_i = sum_{k in I_M} b_k (sum_j alpha_j e^{-2 pi i k.x~_j}) e^{2 pi i k.x~_i}
  with x~ = x/h, the fast summation formula (Sec. 4.2, eq. fastsum) with both
  inner and outer sums taken exactly (no NFFT approximation).
* ``kb_window`` / ``kb_window_hat``  the Kaiser-Bessel window in grid units,
  phi0(t) = I0(b sqrt(1 - (t/m)^2)) for |t| <= m, and its continuous Fourier
  transform 2m sinh(sqrt(b^2 - (2 pi m xi)^2)) / sqrt(b^2 - (2 pi m xi)^2).
  The paper leaves the NFFT window to its reference on NFFT parameters
  (Sec. 4.1); this is the classical compactly supported Kaiser-Bessel pair.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special


def index_set(M: int) -> np.ndarray:
    """1-D frequencies -M/2, ..., M/2-1 (M even), Sec. 4.1."""
    if M % 2:
        raise ValueError("M must be even")
    return np.arange(-M // 2, M // 2)


def _phase_factors(x: np.ndarray, M: int, sign: float) -> list:
    """Per-dimension exp(sign 2 pi i k x_t) for k in I_M: list of (N, M)."""
    k = index_set(M)
    return [np.exp(sign * 2j * math.pi * np.outer(x[:, t], k)) for t in range(x.shape[1])]


def adjoint_ndft(c: np.ndarray, x: np.ndarray, M: int) -> np.ndarray:
    """g_k = sum_j c_j exp(-2 pi i k.x_j) for k in I_M (eq. adjnfft).
    x: (N, d) torus nodes; returns an array of shape (M,)*d indexed by k+M/2."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    if x.shape[0] != c.shape[0]:
        x = x.T
    E = _phase_factors(x, M, -1.0)
    d = x.shape[1]
    c = c.astype(np.complex128)
    if d == 1:
        return E[0].T @ c
    if d == 2:
        return np.einsum("j,ja,jb->ab", c, E[0], E[1], optimize=True)
    if d == 3:
        return np.einsum("j,ja,jb,jc->abc", c, E[0], E[1], E[2], optimize=True)
    raise ValueError("d <= 3")


def ndft(fhat: np.ndarray, x: np.ndarray, M: int) -> np.ndarray:
    """f_j = sum_{k in I_M} fhat_k exp(+2 pi i k.x_j) (eq. nfft)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    d = fhat.ndim
    if x.shape[1] != d:
        x = x.T
    E = _phase_factors(x, M, +1.0)
    if d == 1:
        return E[0] @ fhat
    if d == 2:
        return np.einsum("ab,ja,jb->j", fhat, E[0], E[1], optimize=True)
    if d == 3:
        return np.einsum("abc,ja,jb,jc->j", fhat, E[0], E[1], E[2], optimize=True)
    raise ValueError("d <= 3")


def gaussian_fourier_analytic(k: np.ndarray, ell: float, h: float) -> np.ndarray:
    """1-D Fourier coefficients of the h-periodised Gaussian exp(-r^2/ell^2):
    c_k = (1/h) int_R exp(-r^2/ell^2) exp(-2 pi i k r/h) dr
        = (sqrt(pi) ell / h) exp(-(pi ell k / h)^2)."""
    k = np.asarray(k, dtype=np.float64)
    return (math.sqrt(math.pi) * ell / h) * np.exp(-(math.pi * ell * k / h) ** 2)


def periodized_gaussian(r: np.ndarray, ell: float, h: float, images: int = 8) -> np.ndarray:
    """sum_{n=-images}^{images} exp(-(r + n h)^2 / ell^2), 1-D."""
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros_like(r)
    for n in range(-images, images + 1):
        out += np.exp(-((r + n * h) ** 2) / ell ** 2)
    return out


def sampled_coefficients(ell: float, h: float, M: int, d: int,
                         zero_nyquist: bool = True) -> np.ndarray:
    """b_k for k in I_M^d from the ordinary FFT of M^d equidistant samples of
    the h-periodised d-dimensional Gaussian on the cell [-h/2, h/2)^d:
        b_k = M^-d sum_{j in I_M^d} kappa~(j h / M) exp(-2 pi i k.j / M).
    Returned real (the samples are even), shape (M,)*d indexed by k+M/2."""
    j = index_set(M)
    s1 = periodized_gaussian(j * h / M, ell, h)
    # the d-dimensional samples of the separable periodised kernel
    samples = s1
    for _ in range(d - 1):
        samples = np.multiply.outer(samples, s1)
    # ordinary FFT over the index set I_M (shift so index 0 <-> j = 0)
    b = np.fft.fftn(np.fft.ifftshift(samples)) / float(M) ** d
    b = np.fft.fftshift(b)
    b = b.real.copy()
    if zero_nyquist:
        sl = [slice(None)] * d
        for t in range(d):
            s = list(sl)
            s[t] = 0  # index 0 <-> k_t = -M/2
            b[tuple(s)] = 0.0
    return b


def fastsum_exact(alpha: np.ndarray, x: np.ndarray, b: np.ndarray, h: float) -> np.ndarray:
    """Eq. fastsum with exact sums: s_i = sum_k b_k ghat_k exp(2 pi i k.x~_i),
    ghat = adjoint NDFT of alpha at x~ = x/h.  Returns the real part."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    M = b.shape[0]
    xt = x / h
    g = adjoint_ndft(alpha, xt, M)
    s = ndft(b * g, xt, M)
    return s.real


def kb_beta(m: int, sigma_os: float) -> float:
    """Kaiser-Bessel shape parameter b = pi m (2 - 1/sigma)."""
    return math.pi * m * (2.0 - 1.0 / sigma_os)


def kb_window(t: np.ndarray, m: int, b: float) -> np.ndarray:
    """phi0(t) = I0(b sqrt(1 - (t/m)^2)) for |t| <= m, else 0 (grid units)."""
    t = np.asarray(t, dtype=np.float64)
    inside = np.abs(t) <= m
    arg = np.sqrt(np.clip(1.0 - (t / m) ** 2, 0.0, None))
    return np.where(inside, scipy.special.i0(b * arg), 0.0)


def kb_window_hat(xi: np.ndarray, m: int, b: float) -> np.ndarray:
    """int phi0(t) exp(-2 pi i xi t) dt = 2m sinh(s)/s, s = sqrt(b^2 - (2 pi m xi)^2)
    (sin form past the root, limit 2m at the root)."""
    xi = np.asarray(xi, dtype=np.float64)
    q = b * b - (2.0 * math.pi * m * xi) ** 2
    out = np.empty_like(q)
    pos = q > 1e-12
    neg = q < -1e-12
    zer = ~(pos | neg)
    s = np.sqrt(q[pos])
    out[pos] = 2 * m * np.sinh(s) / s
    s = np.sqrt(-q[neg])
    out[neg] = 2 * m * np.sin(s) / s
    out[zer] = 2 * m
    return out
