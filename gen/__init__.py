"""Seeded synthetic inputs for the convex-clustering workloads.

This module is shared by the FP64 oracle and by the GPU path.  It holds only
random-number recipes: data matrices, missing-data masks, and the settings
(k, phi rule, regularisation path) that each workload is run with.  It holds
none of the clustering method's arithmetic: no distances, weights,
standardisation, projections or updates.

Every generator uses numpy's ``default_rng(seed)`` (PCG64) and draws its
random numbers in the fixed order written in each function.

Workloads (sizes follow the paper's data shapes; the paper's own data sets are
not available, so these stand in for them):

* ``plain``     n=200,  p=10,    4 isotropic Gaussian clusters, no missing data
* ``expression`` n=2000, p=500,  20 clusters, log-normal feature scales, 5% MCAR
* ``genotype``  n=1000, p=20000, Balding-Nichols {0,1,2} codes over 12 groups
* ``batched``   256 small Gaussian-mixture instances
* ``served``    a Poisson request stream of mixed-size instances, 10% MCAR

Missing entries of X are set to NaN so that any accidental use of them shows.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "Workload",
    "gaussian_mixture",
    "plain",
    "expression",
    "genotype",
    "batched_instance",
    "served_arrivals",
    "served_instance",
    "gamma_path",
    "WORKLOADS",
    "make",
]


@dataclass
class Workload:
    """One synthetic problem instance.

    X      : (n, p) float64, rows are cases; missing entries are NaN.
    mask   : (n, p) bool, True = observed; None means fully observed.
    k      : nearest-neighbour count for the weights.
    phi    : Gaussian-kernel constant.  A value >= 0 is used literally; a
             negative value -c asks for phi = c / median(d^2 over the kNN
             edge set) (the reading used for wide data, where a literal
             constant underflows every weight).
    gammas : regularisation path, processed in the given order.
    standardize : whether columns are standardised before clustering.
    name, seed : identification.
    labels_true : generating cluster of each case (for reporting only).
    """

    name: str
    seed: int
    X: np.ndarray
    mask: Optional[np.ndarray]
    k: int
    phi: float
    gammas: np.ndarray
    standardize: bool = False
    labels_true: Optional[np.ndarray] = field(default=None, repr=False)

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def p(self) -> int:
        return int(self.X.shape[1])


def gamma_path(lo: float, hi: float, count: int) -> np.ndarray:
    """``count`` log-spaced values from lo to hi (inclusive)."""
    return np.logspace(np.log10(lo), np.log10(hi), count)


def _mcar(rng: np.random.Generator, n: int, p: int, frac: float) -> np.ndarray:
    """Missing completely at random: each entry observed with prob 1-frac."""
    return rng.random((n, p)) >= frac


def gaussian_mixture(rng: np.random.Generator, n: int, p: int, n_clusters: int,
                     centre_sd: float = 3.0, noise_sd: float = 1.0):
    """Centres c_k ~ N(0, centre_sd^2 I); case i belongs to cluster i mod C;
    x_i = c_{z_i} + N(0, noise_sd^2 I).  Draw order: centres, then noise."""
    centres = rng.normal(0.0, centre_sd, size=(n_clusters, p))
    z = np.arange(n) % n_clusters
    X = centres[z] + rng.normal(0.0, noise_sd, size=(n, p))
    return X, z


def plain(seed: int = 1001, n: int = 200, p: int = 10) -> Workload:
    """Plain method workload: 4 isotropic Gaussian clusters, no missing data,
    k=10, literal phi=0.5, single gamma=1.0."""
    rng = np.random.default_rng(seed)
    X, z = gaussian_mixture(rng, n, p, 4)
    return Workload("plain", seed, X, None, k=10, phi=0.5,
                    gammas=np.array([1.0]), labels_true=z)


def expression(seed: int = 1002, n: int = 2000, p: int = 500,
               n_clusters: int = 20, missing: float = 0.05,
               n_gamma: int = 30) -> Workload:
    """Expression-like workload: 20 latent clusters, log-normal feature scales
    sigma_f ~ LogNormal(0,1), x_if = sigma_f (c_{z_i f} + N(0,1)), 5% of the
    entries missing completely at random, k=15, gamma path of 30 log-spaced
    values in [1e-3, 1e2].  Not standardised (keeps the feature scales).
    Draw order: centres, noise, feature scales, mask."""
    rng = np.random.default_rng(seed)
    X, z = gaussian_mixture(rng, n, p, n_clusters)
    sigma = rng.lognormal(0.0, 1.0, size=p)
    X = X * sigma[None, :]
    mask = _mcar(rng, n, p, missing)
    X = np.where(mask, X, np.nan)
    return Workload("expression", seed, X, mask, k=15, phi=-0.5,
                    gammas=gamma_path(1e-3, 1e2, n_gamma), labels_true=z)


def genotype(seed: int = 1003, n: int = 1000, p: int = 20000,
             n_groups: int = 12, fst: float = 0.05,
             n_gamma: int = 40) -> Workload:
    """Genotype-like workload (Balding-Nichols): ancestral frequency
    q_l ~ U(0.05, 0.95); group frequency f_gl ~ Beta(q_l (1-F)/F,
    (1-q_l)(1-F)/F) with F = F_ST; genotype g_il ~ Binomial(2, f_{z_i l}),
    z_i = i mod 12.  Columns are to be standardised before clustering;
    k=20, gamma path of 40 log-spaced values in [1e-3, 1e2].
    Draw order: q, f, g."""
    rng = np.random.default_rng(seed)
    q = rng.uniform(0.05, 0.95, size=p)
    a = q * (1.0 - fst) / fst
    b = (1.0 - q) * (1.0 - fst) / fst
    f = rng.beta(a[None, :], b[None, :], size=(n_groups, p))
    z = np.arange(n) % n_groups
    G = rng.binomial(2, f[z]).astype(np.float64)
    return Workload("genotype", seed, G, None, k=20, phi=-0.5,
                    gammas=gamma_path(1e-3, 1e2, n_gamma), standardize=True,
                    labels_true=z)


def batched_instance(b: int) -> Workload:
    """Instance b of the batched workload: seed 4000+b; n ~ U{50..800},
    p ~ U{20..200}, C ~ U{2..10} Gaussian clusters as in ``plain``, k=10,
    phi by the median rule, 16 log-spaced gammas in [1e-3, 1e2].
    Draw order: n, p, C, then the mixture."""
    rng = np.random.default_rng(4000 + b)
    n = int(rng.integers(50, 801))
    p = int(rng.integers(20, 201))
    C = int(rng.integers(2, 11))
    X, z = gaussian_mixture(rng, n, p, C)
    return Workload(f"batched[{b}]", 4000 + b, X, None, k=10, phi=-0.5,
                    gammas=gamma_path(1e-3, 1e2, 16), labels_true=z)


def served_arrivals(rate: float = 200.0, count: int = 2000,
                    seed: int = 5999) -> np.ndarray:
    """Poisson arrival times (seconds) of the served workload."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def served_instance(r: int) -> Workload:
    """Request r of the served workload: seed 5000+r; n log-uniform in
    [100, 5000]; p ~ U{10..1000}; C ~ U{2..10}; 10% MCAR; k=10; phi by the
    median rule; path of U{8..32} log-spaced gammas in [1e-3, 1e2].
    Draw order: n, p, C, path length, mixture, mask."""
    rng = np.random.default_rng(5000 + r)
    n = int(np.exp(rng.uniform(np.log(100), np.log(5000))))
    p = int(rng.integers(10, 1001))
    C = int(rng.integers(2, 11))
    g = int(rng.integers(8, 33))
    X, z = gaussian_mixture(rng, n, p, C)
    mask = _mcar(rng, n, p, 0.10)
    X = np.where(mask, X, np.nan)
    return Workload(f"served[{r}]", 5000 + r, X, mask, k=10, phi=-0.5,
                    gammas=gamma_path(1e-3, 1e2, g), labels_true=z)


WORKLOADS = {
    "plain": plain,
    "expression": expression,
    "genotype": genotype,
}


def make(name: str, **kw) -> Workload:
    """Build a named workload; keyword arguments shrink or reseed it."""
    return WORKLOADS[name](**kw)
