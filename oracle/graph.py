"""Graph helpers for the oracle (FP64 / integer).  Test infrastructure only.

The edge set E holds each unordered pair {i, j} with positive weight once, as
(i, j) with i < j (Methods, block-descent projection: E is the union of the
neighbourhoods N_i = L_i u R_i).  The incidence matrix D (|E| x n) has row e =
(i, j) equal to e_i - e_j, so (D U)_e = u_i - u_j is the constraint
v_ij = u_i - u_j of eq_proxdist, and L = D^T D is the unweighted Laplacian.

``components`` labels the connected components of a subgraph (the fused
edges) by the smallest point index in each, using union-find.  Pinned against
brute-force reachability in tests/test_oracle_graph.py.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def validate_edges(n: int, edges: np.ndarray) -> np.ndarray:
    """Return edges as an (E, 2) int64 array, checking 0 <= i < j < n and that
    no pair repeats."""
    E = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if E.size:
        if (E[:, 0] < 0).any() or (E[:, 1] >= n).any():
            raise ValueError("edge endpoint out of range")
        if (E[:, 0] >= E[:, 1]).any():
            raise ValueError("edges must satisfy i < j")
        key = E[:, 0] * n + E[:, 1]
        if np.unique(key).size != key.size:
            raise ValueError("duplicate edge")
    return E


def incidence(n: int, edges: np.ndarray) -> sp.csr_matrix:
    """D with (D U)_e = u_i - u_j for e = (i, j)."""
    E = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    m = E.shape[0]
    rows = np.repeat(np.arange(m), 2)
    cols = E.reshape(-1)
    vals = np.tile(np.array([1.0, -1.0]), m)
    return sp.csr_matrix((vals, (rows, cols)), shape=(m, n))


def adjacency(n: int, edges: np.ndarray) -> sp.csr_matrix:
    """Unweighted symmetric adjacency of E (n x n)."""
    E = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    r = np.concatenate([E[:, 0], E[:, 1]])
    c = np.concatenate([E[:, 1], E[:, 0]])
    return sp.csr_matrix((np.ones(r.size), (r, c)), shape=(n, n))


def degrees(n: int, edges: np.ndarray) -> np.ndarray:
    """|N_i| for each point."""
    E = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return np.bincount(E.reshape(-1), minlength=n).astype(np.int64)


def components(n: int, edges: np.ndarray, keep=None):
    """Connected components of the subgraph made of the edges with keep[e]
    true (all edges if keep is None).  Returns (labels, n_components) where
    labels[i] is the smallest point index in i's component."""
    E = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if keep is not None:
        E = E[np.asarray(keep, dtype=bool)]
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for i, j in E.tolist():
        ri, rj = find(i), find(j)
        if ri != rj:
            # keep the smaller index as the root so a root is its set's min
            if ri < rj:
                parent[rj] = ri
            else:
                parent[ri] = rj
    labels = np.array([find(i) for i in range(n)], dtype=np.int64)
    return labels, int(np.unique(labels).size)
