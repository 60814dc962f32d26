"""Input preparation for the oracle (FP64).  Test infrastructure only.

* ``observed_column_means``: mean of each column over its observed entries.
* ``impute_column_means``: X-tilde, missing entries replaced by the observed
  column mean.  Used for the initial iterate and for the weight distances.
* ``standardize_columns``: each column to mean 0 and variance 1 over its
  observed entries (population variance, divisor = number observed); a
  constant column becomes 0.  The paper recommends standardising predictors
  whose scales differ widely (Methods, after eq_lindsten).

Pins: tests/test_oracle_prep.py (hand-computed columns, constant columns,
all-missing columns, invariance of the observed pattern).
"""
from __future__ import annotations

import numpy as np


def _mask_of(X: np.ndarray, mask) -> np.ndarray:
    if mask is None:
        return np.ones(X.shape, dtype=bool)
    return np.asarray(mask, dtype=bool)


def observed_column_means(X: np.ndarray, mask=None) -> np.ndarray:
    """Column means over observed entries; 0 for a column with none observed."""
    X = np.asarray(X, dtype=np.float64)
    M = _mask_of(X, mask)
    cnt = M.sum(axis=0)
    tot = np.where(M, X, 0.0).sum(axis=0)
    out = np.zeros(X.shape[1])
    nz = cnt > 0
    out[nz] = tot[nz] / cnt[nz]
    return out


def impute_column_means(X: np.ndarray, mask=None) -> np.ndarray:
    """X with every missing entry replaced by its observed column mean."""
    X = np.asarray(X, dtype=np.float64)
    M = _mask_of(X, mask)
    mu = observed_column_means(X, M)
    return np.where(M, X, mu[None, :])


def standardize_columns(X: np.ndarray, mask=None) -> np.ndarray:
    """Observed entries of each column mapped to (x - mean)/sd, where mean and
    sd (divisor = observed count) are taken over the observed entries; sd == 0
    gives 0.  Missing entries are returned as NaN."""
    X = np.asarray(X, dtype=np.float64)
    M = _mask_of(X, mask)
    mu = observed_column_means(X, M)
    cnt = M.sum(axis=0)
    dev = np.where(M, X - mu[None, :], 0.0)
    var = np.zeros(X.shape[1])
    nz = cnt > 0
    var[nz] = (dev[:, nz] ** 2).sum(axis=0) / cnt[nz]
    sd = np.sqrt(var)
    inv = np.zeros_like(sd)
    inv[sd > 0] = 1.0 / sd[sd > 0]
    Z = dev * inv[None, :]
    return np.where(M, Z, np.nan)
