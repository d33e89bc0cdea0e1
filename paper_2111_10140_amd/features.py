"""Host-side preprocessing ahead of the fast product: z-score scaling and the
grouping of features into windows by mutual information score.

Sec. 6 (data preprocessing): every feature is scaled to mean 0 and standard
deviation 1 with statistics taken from the training data only; test data
are scaled with the same statistics.

Sec. 5 (multiple kernel learning): features are ranked by their mutual
information score with the label; features scoring below a threshold are
dropped; the rest go to windows in rank order, three per window (the last
window holds the remaining one, two or three), and every window gets the
weight 1/P.

The paper does not fix how the score is estimated.  Here it is the plug-in
estimate on a binned feature: the feature's values are cut into B bins of
(nearly) equal counts at its empirical quantiles, B = clamp(ceil(N^(1/3)),
2, 64), and I(X; Y) = sum_{b, c} p(b, c) log(p(b, c) / (p(b) p(c))) in nats
over the joint histogram of bin and label.  Labels are discrete (class
labels); a real-valued target is first cut into the same kind of quantile
bins.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np


def zscore_fit(X: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Per-feature mean and standard deviation of training data X (N, d); a
    constant feature gets standard deviation 1 (it is only centred)."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim != 2 or X.shape[0] < 1:
        raise ValueError("X must be (N, d) with N >= 1")
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std = np.where(std > 0.0, std, 1.0)
    return mean, std


def zscore_apply(X: np.ndarray, mean: np.ndarray, std: np.ndarray) -> np.ndarray:
    """(X - mean) / std with the training statistics."""
    X = np.asarray(X, dtype=np.float64)
    return np.ascontiguousarray((X - mean) / std)


def quantile_bins(x: np.ndarray, n_bins: int) -> np.ndarray:
    """Bin index in [0, n_bins) of every value: the value's rank r (the
    number of values strictly below it, so equal values share a rank) gives
    bin floor(r n_bins / N).  Distinct values split into n_bins runs of
    equal length up to one; equal values always share a bin, so a binned
    feature carries no information about where its rows sit."""
    x = np.asarray(x)
    N = x.shape[0]
    if N == 0:
        return np.zeros(0, dtype=np.int64)
    order = np.argsort(x, kind="stable")
    srt = x[order]
    # a value's rank is the sorted position where its run of equal values starts
    starts = np.empty(N, dtype=bool)
    starts[0] = True
    np.not_equal(srt[1:], srt[:-1], out=starts[1:])
    run_start = np.maximum.accumulate(np.where(starts, np.arange(N, dtype=np.int64), 0))
    ranks = np.empty(N, dtype=np.int64)
    ranks[order] = run_start
    return (ranks * n_bins) // N


def default_bins(N: int) -> int:
    return int(min(64, max(2, math.ceil(N ** (1.0 / 3.0)))))


def _labels(y: np.ndarray, n_bins: int) -> np.ndarray:
    y = np.asarray(y)
    if y.dtype.kind in "iub":
        _, inv = np.unique(y, return_inverse=True)
        return inv.astype(np.int64)
    vals = np.unique(y)
    if vals.size <= 64 and np.all(vals == np.round(vals)):
        return np.searchsorted(vals, y).astype(np.int64)
    return quantile_bins(y, n_bins)


def _binned_mi(bx: np.ndarray, cy: np.ndarray, B: int, C: int) -> float:
    """Plug-in mutual information (nats) of bin indices bx in [0, B) and
    label indices cy in [0, C) from their joint counts."""
    N = bx.shape[0]
    joint = np.bincount(bx * C + cy, minlength=B * C).reshape(B, C).astype(np.float64)
    pj = joint / N
    pb = pj.sum(axis=1, keepdims=True)
    pc = pj.sum(axis=0, keepdims=True)
    nz = pj > 0
    return float(np.sum(pj[nz] * np.log(pj[nz] / (pb @ pc)[nz])))


def mutual_information(x: np.ndarray, y: np.ndarray, n_bins: int = 0) -> float:
    """Plug-in mutual information (nats) between feature values x and labels
    y after cutting x into n_bins quantile bins (0: default_bins(N))."""
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    if N == 0:
        return 0.0
    B = n_bins or default_bins(N)
    cy = _labels(y, B)
    return _binned_mi(quantile_bins(x, B), cy, B, int(cy.max()) + 1)


def mis_scores(X: np.ndarray, y: np.ndarray, n_bins: int = 0) -> np.ndarray:
    """Mutual information score of every feature (column) of X with y (the
    labels are binned once for all features)."""
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[0]
    if N == 0:
        return np.zeros(X.shape[1])
    B = n_bins or default_bins(N)
    cy = _labels(y, B)
    C = int(cy.max()) + 1
    return np.array([_binned_mi(quantile_bins(X[:, j], B), cy, B, C) for j in range(X.shape[1])])


def group_windows(scores: Sequence[float], threshold: float = 0.0,
                  size: int = 3) -> List[Tuple[Tuple[int, ...], float]]:
    """Windows from scores: features with score >= threshold, ranked by
    descending score (ties: lower index first), cut into consecutive groups
    of `size` (the last may be shorter), weights 1/P.  Returns
    [(features, eta), ...]; empty if no feature passes."""
    if not 1 <= size <= 3:
        raise ValueError("a window holds 1, 2 or 3 features")
    s = np.asarray(scores, dtype=np.float64)
    keep = [j for j in range(s.size) if s[j] >= threshold]
    keep.sort(key=lambda j: (-s[j], j))
    groups = [tuple(keep[k:k + size]) for k in range(0, len(keep), size)]
    P = len(groups)
    return [(g, 1.0 / P) for g in groups]
