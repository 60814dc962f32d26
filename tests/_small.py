"""Small seeded problems shared by the CPU oracle tests (inputs only)."""
import numpy as np

import gen
from oracle import weights


def mixture_problem(seed, n=16, p=3, clusters=3, k=4, phi=0.0, missing=0.0):
    rng = np.random.default_rng(seed)
    X, _ = gen.gaussian_mixture(rng, n, p, clusters)
    mask = None
    if missing > 0:
        mask = rng.random((n, p)) >= missing
        mask[:, :] |= ~mask.any(axis=0, keepdims=True)  # keep every column observed somewhere
        X = np.where(mask, X, np.nan)
    edges, w, _ = weights.knn_weights(X, mask, k, phi)
    return X, mask, edges, w
