"""k-nearest-neighbour Gaussian-kernel weights (oracle, FP64).  Test
infrastructure only.

Definition (Methods, "Calibration of Weights", eq_weighting):
  d_ij  = ||x_i - x_j||  (Euclidean, on the mean-imputed matrix X-tilde when
          entries are missing; the paper fills them by multiple imputation,
          which is replaced here by observed-column-mean imputation)
  i ~_k j  iff  j is among the k nearest neighbours of i, or i among those of j
  w_ij  = 1{i ~_k j} exp(-phi d_ij^2)
Readings where the paper is silent:
  * a point is not its own neighbour; distance ties are broken towards the
    lower index;
  * phi < 0 means phi = |phi| / median(d^2 over the edge set), taking the
    lower median (element floor((E-1)/2) of the sorted values);
  * optional normalisation makes the weights over the edge set (each
    unordered pair once) sum to 1, which the paper notes only rescales mu.

Distances are computed straight from their definition, one row at a time, in
FP64.  Pins: tests/test_oracle_weights.py (brute force on tiny inputs, ties,
symmetry, phi = 0 uniform weights, the median rule).
"""
from __future__ import annotations

import numpy as np

from .prep import impute_column_means


def sq_distances_row(Xt: np.ndarray, i: int) -> np.ndarray:
    """d_ij^2 for all j, from the definition sum_f (x_jf - x_if)^2."""
    diff = Xt - Xt[i][None, :]
    return (diff * diff).sum(axis=1)


def knn_rows(Xt: np.ndarray, k: int, rows) -> np.ndarray:
    """(len(rows), k) neighbour indices of the given points, nearest first,
    ties to the lower index, self excluded."""
    n = Xt.shape[0]
    if not (1 <= k < n):
        raise ValueError("need 1 <= k < n")
    rows = np.asarray(rows, dtype=np.int64).reshape(-1)
    out = np.empty((rows.size, k), dtype=np.int64)
    idx = np.arange(n)
    for r, i in enumerate(rows.tolist()):
        d2 = sq_distances_row(Xt, i)
        d2[i] = np.inf
        order = np.lexsort((idx, d2))  # primary d2, secondary index
        out[r] = order[:k]
    return out


def knn_lists(Xt: np.ndarray, k: int) -> np.ndarray:
    """(n, k) neighbour indices of each point, nearest first, ties to the
    lower index, self excluded."""
    return knn_rows(Xt, k, np.arange(Xt.shape[0]))


def knn_edges(Xt: np.ndarray, k: int):
    """Symmetrised kNN edge set, sorted by (i, j) with i < j, and the squared
    distance of each edge."""
    n = Xt.shape[0]
    nb = knn_lists(Xt, k)
    a = np.repeat(np.arange(n), k)
    b = nb.reshape(-1)
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    key = np.unique(lo * n + hi)
    edges = np.stack([key // n, key % n], axis=1)
    d2 = np.empty(edges.shape[0])
    for e, (i, j) in enumerate(edges.tolist()):
        diff = Xt[j] - Xt[i]
        d2[e] = (diff * diff).sum()
    return edges, d2


def lower_median(v: np.ndarray) -> float:
    v = np.sort(np.asarray(v, dtype=np.float64))
    return float(v[(v.size - 1) // 2])


def knn_weights(X: np.ndarray, mask, k: int, phi: float, normalize: bool = False):
    """Return (edges, w, phi_used): edges (E, 2) with i < j sorted
    lexicographically, w (E,) float64."""
    Xt = impute_column_means(X, mask)
    edges, d2 = knn_edges(Xt, k)
    if phi < 0:
        med = lower_median(d2)
        phi_used = (-phi) / med if med > 0 else 0.0
    else:
        phi_used = float(phi)
    w = np.exp(-phi_used * d2)
    if normalize:
        w = w / w.sum()
    return edges, w, phi_used
