"""Pins for oracle.graph: incidence matrix D (v_ij = u_i - u_j, eq_proxdist),
the Laplacian, and connected components labelled by their minimum index."""
import numpy as np
import pytest
from scipy.sparse.csgraph import connected_components

from oracle import graph


def _random_edges(rng, n, m):
    pairs = set()
    while len(pairs) < m:
        i, j = sorted(rng.choice(n, 2, replace=False).tolist())
        pairs.add((i, j))
    return np.array(sorted(pairs), dtype=np.int64)


def test_incidence_and_laplacian(rng):
    n = 9
    E = _random_edges(rng, n, 14)
    D = graph.incidence(n, E).toarray()
    U = rng.normal(size=(n, 3))
    for e, (i, j) in enumerate(E):
        assert np.array_equal((D @ U)[e], U[i] - U[j])
    L = D.T @ D
    deg = graph.degrees(n, E)
    A = graph.adjacency(n, E).toarray()
    assert np.array_equal(L, np.diag(deg) - A)


def test_validate_edges():
    with pytest.raises(ValueError):
        graph.validate_edges(3, [[1, 0]])
    with pytest.raises(ValueError):
        graph.validate_edges(3, [[0, 3]])
    with pytest.raises(ValueError):
        graph.validate_edges(3, [[0, 1], [0, 1]])


def _bfs_labels(n, E):
    adj = [[] for _ in range(n)]
    for i, j in E:
        adj[i].append(j)
        adj[j].append(i)
    lab = [-1] * n
    for s in range(n):
        if lab[s] >= 0:
            continue
        stack = [s]
        lab[s] = s
        while stack:
            a = stack.pop()
            for b in adj[a]:
                if lab[b] < 0:
                    lab[b] = s
                    stack.append(b)
    return np.array(lab)


@pytest.mark.parametrize("m", [0, 5, 20, 60])
def test_components_vs_bfs(rng, m):
    n = 40
    E = _random_edges(rng, n, m) if m else np.zeros((0, 2), dtype=np.int64)
    keep = rng.random(len(E)) < 0.7
    lab, k = graph.components(n, E, keep)
    ref = _bfs_labels(n, E[keep])  # BFS from increasing s labels by the min
    assert np.array_equal(lab, ref)
    ncc, _ = connected_components(graph.adjacency(n, E[keep]), directed=False)
    assert k == ncc
