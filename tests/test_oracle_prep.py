"""Pins for oracle.prep: observed-column means, imputation, standardisation
(Methods: standardise predictors with widely different scales)."""
import numpy as np

from oracle import prep


def test_observed_means_by_hand():
    X = np.array([[1.0, 2.0, np.nan], [3.0, np.nan, np.nan], [5.0, 8.0, np.nan]])
    M = ~np.isnan(X)
    mu = prep.observed_column_means(X, M)
    assert mu.tolist() == [3.0, 5.0, 0.0]  # all-missing column -> 0
    Xt = prep.impute_column_means(X, M)
    assert Xt.tolist() == [[1, 2, 0], [3, 5, 0], [5, 8, 0]]


def test_standardize_by_hand():
    X = np.array([[1.0, 4.0, 7.0], [3.0, 4.0, np.nan], [5.0, 4.0, 9.0]])
    M = ~np.isnan(X)
    Z = prep.standardize_columns(X, M)
    # column 0: mean 3, population sd sqrt(8/3)
    sd = np.sqrt(8.0 / 3.0)
    assert np.allclose(Z[:, 0], [-2 / sd, 0.0, 2 / sd], atol=1e-15)
    assert (Z[:, 1] == 0).all()  # constant column -> 0
    assert np.allclose(Z[[0, 2], 2], [-1.0, 1.0])  # mean 8, sd 1
    assert np.isnan(Z[1, 2])


def test_standardize_moments(rng):
    X = rng.normal(3.0, 5.0, size=(50, 7))
    M = rng.random(X.shape) > 0.2
    Z = prep.standardize_columns(np.where(M, X, np.nan), M)
    for f in range(7):
        z = Z[M[:, f], f]
        assert abs(z.mean()) < 1e-13
        assert abs((z ** 2).mean() - 1.0) < 1e-12
