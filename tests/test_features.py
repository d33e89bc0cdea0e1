"""Preprocessing pins (CPU): z-score scaling with training statistics
(Sec. 6) and the grouping of features into windows by mutual information
score (Sec. 5).  The score is checked against scikit-learn's contingency
mutual information on the same bins, against closed forms, and on data
whose label depends on known features."""
import math

import numpy as np
import pytest
from sklearn.metrics import mutual_info_score

import workloads
from paper_2111_10140_amd import features as F


def test_zscore_uses_training_statistics():
    rng = np.random.default_rng(0)
    X = rng.normal(3.0, 2.0, (500, 4))
    X[:, 2] = 7.0  # constant feature
    Z = rng.normal(-1.0, 5.0, (200, 4))
    mean, std = F.zscore_fit(X)
    Xs = F.zscore_apply(X, mean, std)
    np.testing.assert_allclose(Xs.mean(axis=0), 0.0, atol=1e-12)
    np.testing.assert_allclose(Xs[:, [0, 1, 3]].std(axis=0), 1.0, rtol=1e-12)
    assert np.all(Xs[:, 2] == 0.0)
    # test data scaled with the training statistics, not their own
    Zs = F.zscore_apply(Z, mean, std)
    np.testing.assert_allclose(Zs, (Z - X.mean(axis=0)) / np.where(X.std(axis=0) > 0, X.std(axis=0), 1))
    assert abs(Zs[:, 0].mean()) > 0.5


def test_quantile_bins_equal_counts():
    x = np.random.default_rng(1).standard_normal(1000)
    b = F.quantile_bins(x, 7)
    counts = np.bincount(b, minlength=7)
    assert counts.max() - counts.min() <= 1
    # monotone in x
    o = np.argsort(x)
    assert np.all(np.diff(b[o]) >= 0)


def test_mutual_information_matches_contingency_library():
    rng = np.random.default_rng(2)
    x = rng.standard_normal(3000)
    y = np.where(x + 0.8 * rng.standard_normal(3000) > 0, 1, -1)
    for B in (4, 10, 15):
        ref = mutual_info_score(y, F.quantile_bins(x, B))
        assert F.mutual_information(x, y, B) == pytest.approx(ref, rel=1e-12, abs=1e-15)


def test_mutual_information_closed_forms():
    # every bin holds both classes equally: I = 0
    x = np.arange(400, dtype=np.float64)
    y = np.where(np.arange(400) % 2 == 0, 1, -1)
    assert abs(F.mutual_information(x, y, 8)) < 1e-15
    # the label is the bin parity, classes balanced: I = H(Y) = log 2
    b = F.quantile_bins(x, 8)
    y2 = np.where(b % 2 == 0, 1, -1)
    assert F.mutual_information(x, y2, 8) == pytest.approx(math.log(2.0), rel=1e-14)
    # three balanced classes fixed by the bin: log 3
    y3 = b % 3
    x3 = np.arange(480, dtype=np.float64)
    y3 = F.quantile_bins(x3, 6) % 3
    assert F.mutual_information(x3, y3, 6) == pytest.approx(math.log(3.0), rel=1e-14)


def test_group_windows_rank_threshold_and_weights():
    s = [0.1, 0.5, 0.0, 0.5, 0.3, 0.02, 0.4]
    w = F.group_windows(s, threshold=0.0)
    assert [g for g, _ in w] == [(1, 3, 6), (4, 0, 5), (2,)]  # ties: lower index first
    assert all(e == pytest.approx(1 / 3) for _, e in w)
    w = F.group_windows(s, threshold=0.05)
    assert [g for g, _ in w] == [(1, 3, 6), (4, 0)]
    assert all(e == 0.5 for _, e in w)
    assert F.group_windows(s, threshold=1.0) == []
    assert [g for g, _ in F.group_windows([0.2, 0.1], size=1)] == [(0,), (1,)]
    with pytest.raises(ValueError):
        F.group_windows(s, size=4)


def test_informative_features_rank_first():
    X, y, _, _ = workloads.labelled(20000, 10)
    mean, std = F.zscore_fit(X)
    sc = F.mis_scores(F.zscore_apply(X, mean, std), y)
    top = set(np.argsort(-sc)[:3])
    assert top == {2, 5, 7}
    w = F.group_windows(sc)
    assert set(w[0][0]) == {2, 5, 7} and len(w) == 3


def test_tied_values_share_a_bin():
    # equal values must land in one bin whatever the rows' order
    x = np.repeat(np.array([0.0, 1.0, 2.0, 3.0]), [10, 300, 40, 250])
    b = F.quantile_bins(x, 8)
    for v in (0.0, 1.0, 2.0, 3.0):
        assert np.unique(b[x == v]).size == 1
    assert np.all(F.quantile_bins(np.full(77, 4.2), 5) == 0)


def test_rows_sorted_by_label_give_no_spurious_information():
    # rows ordered by class: a constant feature and a feature independent of
    # the label must score about 0 (position-based tie-breaks once split
    # the tied values by row and scored them near log 2)
    rng = np.random.default_rng(4)
    N = 3000
    y = np.sort(np.where(rng.random(N) < 0.5, -1, 1))
    const = np.full(N, 3.0)
    indep = (rng.random(N) < 0.5).astype(np.float64)
    informative = y + 2.0 * rng.standard_normal(N)
    assert F.mutual_information(const, y) == 0.0
    assert F.mutual_information(indep, y) < 5e-3
    assert F.mutual_information(informative, y) > 10 * F.mutual_information(indep, y)
    sc = F.mis_scores(np.stack([const, indep, informative], axis=1), y)
    assert int(np.argmax(sc)) == 2
