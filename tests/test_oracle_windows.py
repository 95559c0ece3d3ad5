"""Pins of the oracle's window selection by mutual-information ranking
(Section 3): closed forms of the mutual information, agreement with an
independent library routine on the same contingency tables, the bin rule at
its edges, and recovery of a known relevance order."""
import numpy as np
import pytest

import oracle
import workloads


def test_mi_of_a_copy_of_balanced_labels_is_log2():
    y = np.where(np.arange(1000) % 2 == 0, 1.0, -1.0)
    W, mi, counts = oracle.mi_windows(y[:, None].copy(), y, bins=2, P=1)
    assert mi[0] == pytest.approx(np.log(2.0), rel=1e-15)
    assert counts[0].tolist() == [[500, 0], [0, 500]]


def test_mi_is_zero_when_both_classes_have_the_same_histogram():
    x = np.concatenate([np.arange(50.0), np.arange(50.0)])
    y = np.concatenate([np.ones(50), -np.ones(50)])
    _, mi, _ = oracle.mi_windows(x[:, None], y, bins=7, P=1)
    assert mi[0] == 0.0


@pytest.mark.parametrize("bins", [2, 9, 32])
def test_mi_matches_an_independent_contingency_routine(bins):
    from sklearn.metrics import mutual_info_score
    p = workloads.graded_features(seed=3, N=3000, d=5)
    _, mi, _ = oracle.mi_windows(p.X, p.labels, bins=bins, P=2)
    B = oracle.mi_bins(p.X, bins)
    for f in range(5):
        assert mi[f] == pytest.approx(mutual_info_score(p.labels > 0, B[:, f]), rel=1e-12, abs=1e-15)


def test_bin_rule_at_the_edges():
    # range [0, 1], 4 bins: 0 -> 0, 0.25 k -> k, 1 -> 3 (clamped); a constant feature -> 0
    X = np.array([[0.0, 5.0], [0.25, 5.0], [0.5, 5.0], [0.7499, 5.0], [1.0, 5.0]])
    B = oracle.mi_bins(X, 4)
    assert B[:, 0].tolist() == [0, 1, 2, 2, 3]
    assert B[:, 1].tolist() == [0, 0, 0, 0, 0]


def test_windows_follow_the_relevance_order():
    order = np.random.default_rng(1).permutation(14)
    p = workloads.graded_features(seed=2, N=20000, d=14, order=order)
    W, mi, _ = oracle.mi_windows(p.X, p.labels, bins=32, P=5)
    ranked = np.argsort(order)               # feature of rank 0, 1, ...
    expect = np.full((5, 3), -1)
    for l in range(5):
        f = ranked[3 * l: 3 * l + 3]
        expect[l, :len(f)] = f
    assert W.tolist() == expect.tolist()
    assert np.all(np.diff(mi[ranked]) < 0)
    # fewer windows take the top-ranked features only
    W2, _, _ = oracle.mi_windows(p.X, p.labels, bins=32, P=2)
    assert W2.tolist() == expect[:2].tolist()


def test_ties_go_to_the_lower_index():
    p = workloads.graded_features(seed=4, N=2000, d=3)
    X = np.concatenate([p.X[:, [1]], p.X, p.X[:, [1]]], axis=1)   # features 0, 2 and 4 are identical
    W, mi, _ = oracle.mi_windows(X, p.labels, bins=16, P=2)
    assert mi[0] == mi[2] == mi[4]
    ranked = [f for f in W.reshape(-1) if f >= 0]
    assert ranked.index(0) < ranked.index(2) < ranked.index(4)
