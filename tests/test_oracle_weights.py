"""Pins for oracle.weights (eq_weighting): kNN relation i ~_k j, Gaussian
kernel, ties to the lower index, the median rule for phi, normalisation."""
import itertools
import math

import numpy as np
import pytest

from oracle import weights


def _brute_edges(X, k):
    n = len(X)
    rel = set()
    for i in range(n):
        cand = []
        for j in range(n):
            if j != i:
                d2 = math.fsum((a - b) ** 2 for a, b in zip(X[i], X[j]))
                cand.append((d2, j))
        cand.sort()
        for _, j in cand[:k]:
            rel.add((min(i, j), max(i, j)))
    return sorted(rel)


@pytest.mark.parametrize("n,p,k", [(6, 2, 1), (9, 3, 2), (12, 4, 3), (15, 2, 5)])
def test_knn_bruteforce(rng, n, p, k):
    X = rng.normal(size=(n, p))
    edges, w, phi = weights.knn_weights(X, None, k, 0.7)
    assert [tuple(e) for e in edges.tolist()] == _brute_edges(X.tolist(), k)
    for (i, j), we in zip(edges.tolist(), w):
        d2 = math.fsum((a - b) ** 2 for a, b in zip(X[i], X[j]))
        assert we == pytest.approx(math.exp(-0.7 * d2), rel=1e-14)


def test_ties_to_lower_index():
    # points 0..4 on a line at unit spacing: from point 2, points 1 and 3 tie
    X = np.arange(5, dtype=float)[:, None]
    lists = weights.knn_lists(X, 1)
    assert lists[2, 0] == 1          # tie 1 vs 3 -> lower index
    assert lists[0, 0] == 1 and lists[4, 0] == 3
    lists2 = weights.knn_lists(X, 2)
    assert lists2[0].tolist() == [1, 2]
    assert lists2[2].tolist() == [1, 3]


def test_uniform_phi_zero_and_union(rng):
    X = rng.normal(size=(20, 3))
    edges, w, _ = weights.knn_weights(X, None, 3, 0.0)
    assert (w == 1.0).all()
    assert (edges[:, 0] < edges[:, 1]).all()
    key = edges[:, 0] * 20 + edges[:, 1]
    assert (np.diff(key) > 0).all()
    # each point has at least k neighbours after the union
    deg = np.bincount(edges.reshape(-1), minlength=20)
    assert (deg >= 3).all()


def test_median_rule_and_normalize(rng):
    X = rng.normal(size=(30, 5))
    edges, w, phi = weights.knn_weights(X, None, 4, -0.5)
    d2 = -np.log(w) / phi
    srt = np.sort(d2)
    assert phi * srt[(len(srt) - 1) // 2] == pytest.approx(0.5, rel=1e-12)
    _, wn, _ = weights.knn_weights(X, None, 4, -0.5, normalize=True)
    assert wn.sum() == pytest.approx(1.0, rel=1e-14)
    assert np.allclose(wn / w, wn[0] / w[0])


def test_missing_uses_mean_imputation():
    X = np.array([[0.0, 0.0], [1.0, np.nan], [10.0, 4.0], [11.0, 4.0]])
    M = ~np.isnan(X)
    # column-1 observed mean = 8/3 fills (1, 1)
    edges, d2 = weights.knn_edges(np.where(M, X, 8.0 / 3.0), 1)
    e2, w2, _ = weights.knn_weights(X, M, 1, 1.0)
    assert np.array_equal(edges, e2)
    assert np.allclose(np.exp(-d2), w2)
