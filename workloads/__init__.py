"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only draws random numbers and assembles arrays; it contains none
of the method's arithmetic (no kernel evaluation, no Fourier coefficients, no
solver).  Every workload stands in for the paper's benchmark datasets, which
are not available: the shapes (N points, d features split into feature
windows of at most three features, equal weights 1/P) follow the
extended Gaussian ANOVA kernel of the paper (Sec. 3, eq.
extended_Gaussian_ANOVA_kernel; Sec. 5, combined kernel K = sum eta_l K_l)
and the numerical-experiments section (Sec. 6).

All generators use numpy's PCG64 (``numpy.random.default_rng``) with the
fixed seeds listed below, so both sides see bit-identical inputs.

Workloads
---------
``plain_fp64``      N=2000, d=3, one window {0,1,2}, ell=0.1, beta=1.
``feature_grouped`` N=100000 (or any N), d=9, windows {0,1,2},{3,4,5},{6,7,8},
                    eta=1/3, ell=0.2, beta=1.  N=1e6 is the headline size.
``batched``         64 problems, N log-uniform in [5000, 200000], d=6, windows
                    {0,1,2},{3,4},{5}, 4 right-hand sides, ell in {0.1,0.2,0.4}.
``large``           N=2e6, d=15 from a 16-component Gaussian mixture clamped to
                    [-1/4, 1/4), 5 windows of consecutive triples, ell=0.15,
                    beta=0.5.
``serving``         Poisson stream of requests with N uniform in [1000, 500000],
                    d in {6, 9, 12}, ell uniform in [0.1, 0.4], 1..8 RHS.
``train_test``      a feature-grouped training problem and Nz test points
                    from the same distribution (or a wider box), for
                    prediction at new points.
``labelled``        raw (unscaled) features with +-1 labels that depend on
                    three of them, split into training and test sets.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

LO, HI = -0.25, 0.25


@dataclass
class Window:
    """One feature window W_l: 0-based feature indices and weight eta_l."""

    feat: Tuple[int, ...]
    eta: float

    @property
    def d_A(self) -> int:
        return len(self.feat)


@dataclass
class Problem:
    """A KRR problem: points X (N x d, row-major float64), windows, ell, beta,
    coefficients alpha (N x nrhs, column-major storage in a (nrhs, N) array
    transposed view) and right-hand sides y (same layout)."""

    name: str
    X: np.ndarray
    windows: List[Window]
    ell: float
    beta: float
    alpha: np.ndarray  # shape (N, nrhs), Fortran order
    y: np.ndarray      # shape (N, nrhs), Fortran order
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.X.shape[0]

    @property
    def d(self) -> int:
        return self.X.shape[1]

    @property
    def nrhs(self) -> int:
        return self.alpha.shape[1]


def consecutive_windows(d: int, group: int = 3) -> List[Window]:
    """Split features 0..d-1 into consecutive groups of `group` (the last
    group holds the remainder), equal weights 1/P."""
    feats = [tuple(range(s, min(s + group, d))) for s in range(0, d, group)]
    P = len(feats)
    return [Window(f, 1.0 / P) for f in feats]


def _uniform_points(rng: np.random.Generator, N: int, d: int) -> np.ndarray:
    return np.ascontiguousarray(rng.uniform(LO, HI, size=(N, d)))


def _smooth_target(u: np.ndarray, freq: float = 4.0) -> np.ndarray:
    """g(u) = sin(freq*pi*u1) cos(freq*pi*u2) + u3, truncated to the columns
    present (a synthetic label, not part of the method)."""
    out = np.sin(freq * math.pi * u[:, 0])
    if u.shape[1] > 1:
        out = out * np.cos(freq * math.pi * u[:, 1])
    if u.shape[1] > 2:
        out = out + u[:, 2]
    return out


def plain_fp64(N: int = 2000) -> Problem:
    """Small double-precision case: N points uniform in [-1/4,1/4)^3, one
    window of three features, ell = 0.1, beta = 1.  Seeds: X 0, alpha 100,
    noise 200."""
    X = _uniform_points(np.random.default_rng(0), N, 3)
    alpha = np.random.default_rng(100).standard_normal(N)
    noise = np.random.default_rng(200).normal(0.0, 0.1, size=N)
    y = np.sin(4 * math.pi * X[:, 0]) * np.cos(4 * math.pi * X[:, 1]) + X[:, 2] + noise
    return Problem(
        "plain_fp64", X, [Window((0, 1, 2), 1.0)], 0.1, 1.0,
        np.asfortranarray(alpha[:, None]), np.asfortranarray(y[:, None]),
        extra=dict(M=32, m=4, sigma_os=2.0, h=1.0),
    )


def feature_grouped(N: int = 100_000, seed: int = 1, nrhs: int = 1) -> Problem:
    """Nine features uniform in [-1/4,1/4), three windows of three features
    with weights 1/3, ell = 0.2, beta = 1.  y = sum over windows of g(x^W) +
    N(0, 0.1^2).  Seed 1 for N = 1e5, seed 2 for the 1e6 headline size."""
    rng = np.random.default_rng(seed)
    X = _uniform_points(rng, N, 9)
    wins = consecutive_windows(9)
    alpha = rng.standard_normal((N, nrhs))
    y = np.zeros((N, nrhs))
    for r in range(nrhs):
        base = sum(_smooth_target(X[:, list(w.feat)]) for w in wins)
        y[:, r] = base + rng.normal(0.0, 0.1, size=N)
    return Problem(f"feature_grouped_N{N}", X, wins, 0.2, 1.0,
                   np.asfortranarray(alpha), np.asfortranarray(y),
                   extra=dict(M=64, m=6, sigma_os=2.0))


def headline(N: int = 1_000_000) -> Problem:
    return feature_grouped(N, seed=2)


def batched(n_problems: int = 64, nrhs: int = 4, n_lo: int = 5000,
            n_hi: int = 200_000, seed: int = 3) -> List[Problem]:
    """64 independent problems with N log-uniform in [5000, 200000], d = 6 in
    windows {0,1,2} (d_A=3), {3,4} (d_A=2), {5} (d_A=1), 4 right-hand sides
    g_r(u) = sin(2 pi (2+r) u1) cos(2 pi (2+r) u2) (+u3) + noise, ell drawn from
    {0.1, 0.2, 0.4}.  Problem p uses seed 3000+p."""
    meta = np.random.default_rng(seed)
    Ns = np.rint(np.exp(meta.uniform(math.log(n_lo), math.log(n_hi), n_problems))).astype(int)
    ells = meta.choice([0.1, 0.2, 0.4], size=n_problems)
    wins = [Window((0, 1, 2), 1 / 3), Window((3, 4), 1 / 3), Window((5,), 1 / 3)]
    out = []
    for p in range(n_problems):
        rng = np.random.default_rng(3000 + p)
        N = int(Ns[p])
        X = _uniform_points(rng, N, 6)
        alpha = rng.standard_normal((N, nrhs))
        y = np.zeros((N, nrhs))
        for r in range(nrhs):
            f = 2.0 * (2 + r)
            y[:, r] = sum(_smooth_target(X[:, list(w.feat)], f) for w in wins) \
                + rng.normal(0.0, 0.1, size=N)
        out.append(Problem(f"batched_{p}", X, wins, float(ells[p]), 1.0,
                           np.asfortranarray(alpha), np.asfortranarray(y)))
    return out


def large(N: int = 2_000_000, seed: int = 4) -> Problem:
    """N points in R^15 from a 16-component isotropic Gaussian mixture (equal
    weights, means U[-0.2,0.2)^15, std U[0.03,0.08]), clamped to
    [-1/4, nextafter(1/4, 0)]; five windows of consecutive triples, eta=1/5,
    ell = 0.15, beta = 0.5."""
    rng = np.random.default_rng(seed)
    d, K = 15, 16
    means = rng.uniform(-0.2, 0.2, size=(K, d))
    stds = rng.uniform(0.03, 0.08, size=K)
    comp = rng.integers(0, K, size=N)
    X = means[comp] + stds[comp, None] * rng.standard_normal((N, d))
    np.clip(X, LO, np.nextafter(HI, 0.0), out=X)
    X = np.ascontiguousarray(X)
    wins = consecutive_windows(d)
    alpha = rng.standard_normal((N, 1))
    y = sum(_smooth_target(X[:, list(w.feat)]) for w in wins) + rng.normal(0.0, 0.1, size=N)
    return Problem(f"large_N{N}", X, wins, 0.15, 0.5, np.asfortranarray(alpha),
                   np.asfortranarray(y[:, None]), extra=dict(M=64, m=6, sigma_os=2.0))


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after stream start
    problem: Problem


def serving_stream(n_requests: int, rate: float, n_lo: int = 1000, n_hi: int = 500_000,
                   seed: int = 5, rhs_max: int = 8) -> List[Request]:
    """Poisson arrivals (exponential gaps with mean 1/rate seconds); request r
    draws from seed 5000+r: N uniform in [n_lo, n_hi], d in {6, 9, 12} with
    consecutive-triple windows, ell uniform in [0.1, 0.4], 1..rhs_max RHS."""
    meta = np.random.default_rng(seed)
    gaps = meta.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps)
    reqs = []
    for r in range(n_requests):
        rng = np.random.default_rng(5000 + r)
        N = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.choice([6, 9, 12]))
        ell = float(rng.uniform(0.1, 0.4))
        nrhs = int(rng.integers(1, rhs_max + 1))
        X = _uniform_points(rng, N, d)
        wins = consecutive_windows(d)
        y = np.zeros((N, nrhs))
        for c in range(nrhs):
            f = 2.0 * (2 + c)
            y[:, c] = sum(_smooth_target(X[:, list(w.feat)], f) for w in wins) \
                + rng.normal(0.0, 0.1, size=N)
        alpha = np.zeros((N, nrhs))
        reqs.append(Request(r, float(t[r]), Problem(f"req_{r}", X, wins, ell, 1.0,
                                                    np.asfortranarray(alpha),
                                                    np.asfortranarray(y))))
    return reqs


def random_problem(N: int, d: int, windows: Sequence[Tuple[int, ...]], ell: float,
                   beta: float = 1.0, nrhs: int = 1, seed: int = 0,
                   eta: Optional[Sequence[float]] = None, lo: float = LO, hi: float = HI) -> Problem:
    """Generic seeded problem for tests: uniform points in [lo, hi)^d."""
    rng = np.random.default_rng(seed)
    X = np.ascontiguousarray(rng.uniform(lo, hi, size=(N, d)))
    P = len(windows)
    etas = list(eta) if eta is not None else [1.0 / P] * P
    wins = [Window(tuple(w), float(e)) for w, e in zip(windows, etas)]
    alpha = np.asfortranarray(rng.standard_normal((N, nrhs)))
    y = np.asfortranarray(rng.standard_normal((N, nrhs)))
    return Problem(f"random_N{N}_d{d}_s{seed}", X, wins, ell, beta, alpha, y)


def train_test(N: int, Nz: int, d: int = 9, seed: int = 6, ell: float = 0.2,
               test_lo: float = LO, test_hi: float = HI) -> Tuple[Problem, np.ndarray]:
    """Training problem shaped like ``feature_grouped`` (d features uniform in
    [-1/4, 1/4), consecutive triples as windows with weights 1/P, beta = 1)
    and Nz test points uniform in [test_lo, test_hi)^d drawn after it from the
    same generator; the paper's experiments split each sample into training
    and test halves (Sec. 6).  Returns (problem, Z)."""
    rng = np.random.default_rng(seed)
    X = _uniform_points(rng, N, d)
    wins = consecutive_windows(d)
    alpha = rng.standard_normal((N, 1))
    y = (sum(_smooth_target(X[:, list(w.feat)]) for w in wins)
         + rng.normal(0.0, 0.1, size=N))[:, None]
    Z = np.ascontiguousarray(rng.uniform(test_lo, test_hi, size=(Nz, d)))
    prob = Problem(f"train_test_N{N}_Nz{Nz}_s{seed}", X, wins, ell, 1.0,
                   np.asfortranarray(alpha), np.asfortranarray(y))
    return prob, Z


def labelled(N: int, Nz: int, d: int = 9, informative: Tuple[int, int, int] = (2, 5, 7),
             seed: int = 50, flip: float = 0.05):
    """Binary classification data in raw units: feature j uniform on
    [0, scale_j) with scales from 0.1 to 100 (so that z-scoring matters),
    label sign(sin(pi u_a) + 0.7 u_b + 0.5 u_c) on the informative features
    u = (x - mean) / std (population statistics), each label flipped with
    probability `flip` (each term is informative on its own: the paper's
    score is univariate, Sec. 5).  The paper classifies z-scored data with labels in
    {-1, 1} (Sec. 2, Sec. 6).  Returns (X, y, Z, yz) for N training and Nz
    test points."""
    rng = np.random.default_rng(seed)
    scales = np.exp(rng.uniform(math.log(0.1), math.log(100.0), size=d))
    def draw(n):
        X = rng.uniform(0.0, 1.0, size=(n, d)) * scales
        u = (X / scales - 0.5) * math.sqrt(12.0)
        a, b, c = informative
        g = np.sin(math.pi * u[:, a]) + 0.7 * u[:, b] + 0.5 * u[:, c]
        y = np.where(g >= 0.0, 1.0, -1.0)
        y = np.where(rng.uniform(size=n) < flip, -y, y)
        return np.ascontiguousarray(X), y
    X, y = draw(N)
    Z, yz = draw(Nz)
    return X, y, Z, yz
