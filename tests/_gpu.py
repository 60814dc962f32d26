"""Helpers shared by the GPU parity tests: seeded inputs, the oracle's
reference run, and comparison metrics."""
import numpy as np
import torch

import gen
from oracle import mm, weights


def as_f32_values(X):
    """The FP32 values of X as float64 (the exact inputs both sides see)."""
    return np.asarray(X, dtype=np.float32).astype(np.float64)


def plain_problem():
    wl = gen.plain()
    X = wl.X  # f64 config
    edges, w, _ = weights.knn_weights(X, None, wl.k, wl.phi)
    return X, None, edges, w


def reduced_expression(n=300, p=64, seed=1002):
    wl = gen.expression(seed=seed, n=n, p=p, n_clusters=6, n_gamma=6)
    X = as_f32_values(wl.X)
    edges, w, _ = weights.knn_weights(X, wl.mask, wl.k, wl.phi)
    return X, wl.mask, edges, w, wl.gammas


def to_dev(X, mask, edges, w, dtype):
    Xt = torch.tensor(np.nan_to_num(X, nan=0.0), dtype=dtype, device="cuda")
    m = None if mask is None else torch.tensor(mask.astype(np.uint8), device="cuda")
    e = torch.tensor(np.asarray(edges, dtype=np.int32), device="cuda")
    wt = torch.tensor(np.asarray(w, dtype=np.float64), device="cuda")
    return Xt, m, e, wt


def rel_max(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def oracle_jacobi(X, mask, edges, w):
    return mm.Problem(X, mask, edges, w)
