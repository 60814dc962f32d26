"""Pins of the oracle's extras (principal components, path projection,
smallest connected k, composite-distance weights) against values fixed by
construction or by closed forms."""
import math

import numpy as np
import pytest

from oracle import extras, weights


def _orthonormal_zero_mean(rng, n, r, zero_row=None):
    """n x r with orthonormal columns summing to 0; row zero_row all zero."""
    M = rng.normal(size=(n, r))
    rows = np.ones(n, dtype=bool)
    if zero_row is not None:
        M[zero_row] = 0.0
        rows[zero_row] = False
    M[rows] -= M[rows].mean(axis=0)
    Q, _ = np.linalg.qr(M)
    return Q


def _known_spectrum(seed=7, n=40, p=12, zero_row=None):
    rng = np.random.default_rng(seed)
    sig = np.array([9.0, 4.0, 1.5])
    A = _orthonormal_zero_mean(rng, n, 3, zero_row)
    B, _ = np.linalg.qr(rng.normal(size=(p, 3)))
    off = rng.normal(size=p) * 3.0
    return A @ np.diag(sig) @ B.T + off, sig, B, off


def test_pca_recovers_constructed_components():
    X, sig, B, off = _known_spectrum()
    V, S, c = extras.pca(X, None, 3)
    assert np.allclose(S, sig, rtol=1e-12)
    assert np.allclose(V, extras.sign_fix(B), atol=1e-12)
    assert np.allclose(c, off, atol=1e-12)
    # the largest-magnitude entry of every column is positive
    for k in range(3):
        assert V[np.argmax(np.abs(V[:, k])), k] > 0


def test_pca_ignores_missing_entries_through_mean_imputation():
    # row 0 of the centred matrix is zero, so its entries equal the column
    # means: masking them (and storing garbage there) changes nothing
    X, sig, B, off = _known_spectrum(zero_row=0)
    M = np.ones(X.shape, dtype=bool)
    M[0, ::2] = False
    Xg = X.copy()
    Xg[0, ::2] = 1e6
    V, S, c = extras.pca(Xg, M, 3)
    assert np.allclose(S, sig, rtol=1e-10)
    assert np.allclose(V, extras.sign_fix(B), atol=1e-10)
    assert np.allclose(c, off, atol=1e-10)


def test_projection_of_the_data_has_the_singular_values_as_norms():
    X, sig, B, off = _known_spectrum(seed=9)
    V, S, c = extras.pca(X, None, 2)
    P = extras.project(X, V, c)
    assert np.allclose(np.linalg.norm(P, axis=0), sig[:2], rtol=1e-12)
    assert np.allclose(P.mean(axis=0), 0.0, atol=1e-12)


def _two_clusters(a, b, seed=3):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(a, 3)) * 0.1
    Bc = rng.normal(size=(b, 3)) * 0.1 + 100.0
    return np.vstack([A, Bc])


@pytest.mark.parametrize("a,b", [(5, 9), (7, 7), (3, 12)])
def test_min_k_of_two_separated_clusters_is_the_smaller_size(a, b):
    # a point of the smaller cluster has a-1 neighbours inside it; its a-th
    # nearest neighbour lies in the other cluster
    X = _two_clusters(a, b)
    k, c = extras.min_connected_k(X, None, a + 2)
    assert k == min(a, b) and c == 1
    k, c = extras.min_connected_k(X, None, min(a, b) - 1)
    assert k == -1 and c == 2


def test_min_k_of_a_geometric_chain_is_one():
    X = (2.0 ** np.arange(12))[:, None]
    k, c = extras.min_connected_k(X, None, 3)
    assert k == 1 and c == 1


def test_coordinate_distances_closed_forms():
    assert extras.coord_distance([10.0], [350.0], period=[360.0]) == pytest.approx(20.0, abs=1e-12)
    assert extras.coord_distance([10.0, 1.0], [350.0, 4.0], period=[360.0, 0.0]) == pytest.approx(
        math.hypot(20.0, 3.0), abs=1e-12)
    assert extras.coord_distance([-170.0], [170.0], period=[360.0]) == pytest.approx(20.0, abs=1e-12)
    R = 6371.0
    assert extras.coord_distance([0, 0], [0, 90], geodesic=True, radius=R) == pytest.approx(R * math.pi / 2, rel=1e-12)
    assert extras.coord_distance([90, 0], [0, 45], geodesic=True) == pytest.approx(math.pi / 2, rel=1e-12)
    assert extras.coord_distance([0, 0], [0, 180], geodesic=True) == pytest.approx(math.pi, rel=1e-12)
    assert extras.coord_distance([45, 10], [45, 10], geodesic=True) == 0.0


def test_composite_distance_blend_and_alpha_one_reduces_to_knn_weights():
    X = np.array([[0.0, 0.0], [4.0, 0.0]])
    Y = np.array([[0.0], [8.0]])
    w, _ = extras.composite_weights(X, Y, np.array([[0, 1]]), alpha=0.25, phi=0.01)
    assert w[0] == pytest.approx(math.exp(-0.01 * 7.0 ** 2), rel=1e-14)  # d = 0.25*4 + 0.75*8
    rng = np.random.default_rng(11)
    X = rng.normal(size=(30, 6))
    edges, wk, phik = weights.knn_weights(X, None, 4, -0.5)
    wc, phic = extras.composite_weights(X, rng.normal(size=(30, 2)), edges, alpha=1.0, phi=-0.5)
    assert phic == pytest.approx(phik, rel=1e-14)
    assert np.allclose(wc, wk, rtol=1e-13)


def test_composite_distance_with_missing_entries_uses_the_knn_imputation():
    # alpha = 1 with a mask gives the kNN weights of the same masked data
    rng = np.random.default_rng(12)
    X = rng.normal(size=(40, 7))
    M = rng.random(X.shape) > 0.1
    Xn = np.where(M, X, np.nan)
    edges, wk, phik = weights.knn_weights(Xn, M, 5, -0.5)
    wc, phic = extras.composite_weights(np.where(M, X, 123.0), np.zeros((40, 1)), edges, alpha=1.0, phi=-0.5,
                                        mask=M)
    assert phic == pytest.approx(phik, rel=1e-14)
    assert np.allclose(wc, wk, rtol=1e-13)
