"""Extras around the solver (oracle, FP64).  Test infrastructure only.

* Principal components of the original data (Evaluation of Clusters: the
  cluster path is viewed on principal components of X): X-tilde = X with
  missing entries replaced by observed column means, centred by those means;
  the components are the right singular vectors of the centred matrix (a
  library SVD serves as the step), the singular values come with them.
  Sign convention: each vector's entry of largest magnitude (the first one on
  ties) is positive.
* Projection of a path (Discussion: project before any transfer):
  (U - center) V for each gamma's U.
* Smallest k with a connected kNN graph (Results, "Impact of the Constants
  k and phi"): by definition, the first k = 1, 2, ... whose symmetrised kNN
  graph (the same graph as the weights use) has one component; -1 when
  there is none up to k_max.  A linear scan, so no monotonicity is assumed.
* Composite distance (composite_distance):
  d_ij = alpha ||x_i - x_j|| + (1 - alpha) dist(y_i, y_j), with dist
  Euclidean over coordinates, a coordinate with a period taken modulo it
  (the shorter way round), or the great-circle distance of (latitude,
  longitude) in degrees times a radius; then w = exp(-phi d^2) as in
  eq_weighting, phi < 0 meaning |phi| / lower median of d^2.

Pins: tests/test_oracle_extras.py (a matrix built with known singular
vectors and values, missing-entry imputation, two separated clusters whose
smallest connected k is their size, a geometric chain connected at k = 1,
wrap-around and great-circle distances with known values, alpha = 1
reducing to the kNN weights).
"""
from __future__ import annotations

import math

import numpy as np

from . import graph, weights
from .prep import impute_column_means


def sign_fix(V: np.ndarray) -> np.ndarray:
    """Flip each column so its entry of largest magnitude (first on ties) is
    positive."""
    V = np.array(V, dtype=np.float64, copy=True)
    for c in range(V.shape[1]):
        k = int(np.argmax(np.abs(V[:, c])))  # argmax returns the first maximum
        if V[k, c] < 0:
            V[:, c] = -V[:, c]
    return V


def pca(X: np.ndarray, mask, r: int):
    """(V (p, r), singular values (r,), column means (p,)) of the centred,
    mean-imputed data."""
    Xt = impute_column_means(X, mask)
    center = Xt.mean(axis=0)
    C = Xt - center[None, :]
    _, S, Vt = np.linalg.svd(C, full_matrices=False)
    return sign_fix(Vt[:r].T), S[:r].copy(), center


def project(U: np.ndarray, V: np.ndarray, center=None) -> np.ndarray:
    """(U - center) V."""
    U = np.asarray(U, dtype=np.float64)
    c = np.zeros(U.shape[-1]) if center is None else np.asarray(center, dtype=np.float64)
    return (U - c) @ np.asarray(V, dtype=np.float64)


def min_connected_k(X: np.ndarray, mask, k_max: int):
    """(smallest k <= k_max whose kNN graph is connected, or -1; components
    at k_max)."""
    Xt = impute_column_means(X, mask)
    n = Xt.shape[0]
    found = -1
    ncomp = None
    for k in range(1, k_max + 1):
        edges, _ = weights.knn_edges(Xt, k)
        _, c = graph.components(n, edges)
        if c == 1 and found < 0:
            found = k
        if k == k_max:
            ncomp = c
    return found, ncomp


def coord_distance(yi, yj, period=None, geodesic=False, radius=1.0) -> float:
    """dist(y_i, y_j): periodic Euclidean, or great-circle (haversine) for
    (latitude, longitude) in degrees."""
    yi = np.asarray(yi, dtype=np.float64)
    yj = np.asarray(yj, dtype=np.float64)
    if geodesic:
        la1, lo1 = math.radians(yi[0]), math.radians(yi[1])
        la2, lo2 = math.radians(yj[0]), math.radians(yj[1])
        h = math.sin((la2 - la1) / 2) ** 2 + math.cos(la1) * math.cos(la2) * math.sin((lo2 - lo1) / 2) ** 2
        h = min(max(h, 0.0), 1.0)
        return (radius if radius > 0 else 1.0) * 2.0 * math.atan2(math.sqrt(h), math.sqrt(1.0 - h))
    d = np.abs(yj - yi)
    if period is not None:
        P = np.asarray(period, dtype=np.float64)
        wrap = P > 0
        dm = np.where(wrap, np.mod(d, np.where(wrap, P, 1.0)), d)
        d = np.where(wrap, np.minimum(dm, P - dm), d)
    return float(np.sqrt((d * d).sum()))


def composite_weights(X: np.ndarray, Y: np.ndarray, edges: np.ndarray, alpha: float, phi: float,
                      period=None, geodesic=False, radius=1.0, normalize=False, mask=None):
    """(w (E,), phi_used) over the given edges; with a mask, distances of X
    on its mean-imputed copy (as the kNN weights)."""
    X = np.asarray(X, dtype=np.float64)
    if mask is not None:
        X = impute_column_means(X, mask)
    Y = np.asarray(Y, dtype=np.float64).reshape(X.shape[0], -1)
    E = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    d2 = np.empty(E.shape[0])
    for e, (i, j) in enumerate(E.tolist()):
        dx = math.sqrt(float(((X[j] - X[i]) ** 2).sum())) if X.shape[1] else 0.0
        dy = coord_distance(Y[i], Y[j], period, geodesic, radius)
        d = alpha * dx + (1.0 - alpha) * dy
        d2[e] = d * d
    if phi < 0:
        med = weights.lower_median(d2) if d2.size else 0.0
        phi_used = (-phi) / med if med > 0 else 0.0
    else:
        phi_used = float(phi)
    w = np.exp(-phi_used * d2)
    if normalize and w.size:
        w = w / w.sum()
    return w, phi_used
