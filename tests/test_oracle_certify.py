"""Pins tying the oracle's proximal-distance fixed point to the exact
minimiser of the convex-clustering objective (eq_lindsten), through
certificates that share nothing with the MM iteration:

  * closed forms: n = 2 (fused iff ||x1 - x2|| <= 2 mu w), and p = 1 on the
    complete graph with unit weights (u_i = x_i - mu (2 r_i - n - 1));
  * brute force over all partitions for n <= 5 (the optimum's fusion
    pattern and value);
  * a dual solver with a duality-gap bound ||U - U*|| <= sqrt(2 gap);
  * full coalescence at large mu on a connected graph (all u_i = xbar);
  * for missing data (eq_missing_analog): the minimiser is a fixed point of
    "fill the missing entries from U, then solve the complete-data problem".

The proximal-distance fixed point lies O(eta) from U*; the bounds below are
stated in units of eta.
"""
import numpy as np
import pytest

import gen
from oracle import certify, graph, mm, weights
from tests._small import mixture_problem


def _pd(X, M, E, w, mu, eta=1e-2, tol=1e-7, **kw):
    prob = mm.Problem(X, M, E, w)
    st, info = prob.solve(mu, mm.Opts(eta=eta, tol=tol, **kw))
    return prob, st, info


# ------------------------------------------------ dual solver vs closed forms
@pytest.mark.parametrize("mu", [0.2, 0.9, 3.0])
def test_dual_two_point(mu):
    x = np.array([[0.0, 1.0, 2.0], [1.5, -0.5, 2.5]])
    E = np.array([[0, 1]])
    U, gap = certify.dual_solve(x, E, [0.8], mu)
    assert gap < 1e-12
    assert np.allclose(U, certify.two_point(x[0], x[1], 0.8, mu), atol=1e-6)


def test_dual_line_complete():
    x = np.array([0.0, 1.0, 2.5, 4.0, 7.0])
    E = certify.complete_edges(5)
    mu = 0.2  # min gap 1.0 > 2 mu
    U, gap = certify.dual_solve(x[:, None], E, np.ones(len(E)), mu)
    assert np.allclose(U[:, 0], certify.line_complete(x, mu), atol=1e-6)


@pytest.mark.parametrize("seed,mu", [(21, 0.3), (22, 0.8), (23, 2.0)])
def test_dual_matches_brute_force(seed, mu):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(5, 2)) * 1.5
    W = np.exp(-0.2 * ((X[:, None] - X[None]) ** 2).sum(-1))
    E = certify.complete_edges(5)
    w = W[E[:, 0], E[:, 1]]
    fstar, lab, Ub = certify.brute_force(X, W, mu)
    U, gap = certify.dual_solve(X, E, w, mu)
    assert certify.convex_objective(X, None, U, E, w, mu) == pytest.approx(fstar, abs=1e-8)
    assert np.abs(U - Ub).max() < 1e-5


# ------------------------------------------------ PD fixed point vs optimum
@pytest.mark.parametrize("mu", [0.3, 1.0, 2.5])
def test_pd_two_point(mu):
    x = np.array([[0.0, 1.0], [2.0, 0.5]])
    _, st, info = _pd(x, None, np.array([[0, 1]]), np.array([1.0]), mu, eta=1e-3)
    ref = certify.two_point(x[0], x[1], 1.0, mu)
    assert np.linalg.norm(st.U - ref) <= 1.5e-3 * np.linalg.norm(x)
    fused_ref = np.linalg.norm(x[0] - x[1]) <= 2 * mu
    assert bool(info.fused[0]) == fused_ref
    assert np.allclose(st.U.mean(axis=0), x.mean(axis=0), atol=1e-12)


def test_pd_line_complete():
    x = np.array([0.0, 1.0, 2.5, 4.0, 7.0])
    E = certify.complete_edges(5)
    _, st, info = _pd(x[:, None], None, E, np.ones(len(E)), 0.2, eta=1e-3)
    assert np.abs(st.U[:, 0] - certify.line_complete(x, 0.2)).max() <= 2e-3 * np.abs(x).max()
    assert info.n_clusters == 5


@pytest.mark.parametrize("seed,mu", [(31, 0.25), (32, 0.7), (33, 1.5), (34, 4.0)])
def test_pd_matches_brute_force_partition(seed, mu):
    rng = np.random.default_rng(seed)
    X = np.vstack([rng.normal(0, 0.3, (2, 2)), rng.normal(3, 0.3, (3, 2))])
    W = np.exp(-0.1 * ((X[:, None] - X[None]) ** 2).sum(-1))
    E = certify.complete_edges(5)
    w = W[E[:, 0], E[:, 1]]
    fstar, lab, Ub = certify.brute_force(X, W, mu)
    _, st, info = _pd(X, None, E, w, mu, eta=3e-3)
    assert np.array_equal(info.labels, lab)
    f_pd = certify.convex_objective(X, None, st.U, E, w, mu)
    assert fstar - 1e-9 <= f_pd <= fstar + 3e-3 * abs(fstar) + 1e-9
    assert np.linalg.norm(st.U - Ub) <= 3e-3 * np.linalg.norm(X)


@pytest.mark.parametrize("seed,mu", [(41, 0.3), (42, 1.0), (43, 2.0)])
def test_pd_within_eta_of_dual_certificate(seed, mu):
    X, M, E, w = mixture_problem(seed, n=24, p=3, k=4)
    eta = 1e-2
    _, st, info = _pd(X, M, E, w, mu, eta=eta)
    Ustar, gap = certify.dual_solve(X, E, w, mu)
    cert = np.sqrt(2 * gap)
    assert cert < 1e-5 * np.linalg.norm(X)
    assert np.linalg.norm(st.U - Ustar) <= 0.8 * eta * np.linalg.norm(X) + cert
    dd = np.linalg.norm(Ustar[E[:, 0]] - Ustar[E[:, 1]], axis=1)
    lab_star, _ = graph.components(X.shape[0], E, dd < 1e-6 * np.abs(X).max())
    assert np.array_equal(info.labels, lab_star)


def _fully_fused_fixed_point(prob, d, rho, X):
    """With every s_e = 0 the MM map is linear: A = (I+L)^{-1} U and
    U = A + theta (X - A), theta = d/(d+rho), whose fixed point is
    U = theta (I - (1-theta)(I+L)^{-1})^{-1} X."""
    n = prob.n
    L = (prob.D.T @ prob.D).toarray()
    theta = d / (d + rho)
    G = np.linalg.inv(np.eye(n) + L)
    return theta * np.linalg.solve(np.eye(n) - (1 - theta) * G, X)


def test_full_coalescence_on_connected_graph():
    rng = np.random.default_rng(51)
    X = rng.normal(size=(12, 2))
    E = certify.complete_edges(12)
    w = np.ones(len(E))
    Ustar, gap = certify.dual_solve(X, E, w, 5.0)
    assert np.abs(Ustar - X.mean(axis=0)).max() < 1e-9   # U* = 1 xbar^T
    devs = []
    for eta in (1e-2, 1e-3):
        prob, st, info = _pd(X, None, E, w, 5.0, eta=eta, tol=1e-9)
        assert info.n_clusters == 1 and info.fused.all()
        assert np.allclose(st.U.mean(axis=0), X.mean(axis=0), atol=1e-12)
        # U - xbar shrinks in proportion to eta (complete graph: lambda = n)
        dev = np.linalg.norm(st.U - X.mean(axis=0)) / np.linalg.norm(X - X.mean(axis=0))
        assert dev <= 1.5 * eta
        devs.append(dev)
        ref = _fully_fused_fixed_point(prob, info.d, info.rho, X)
        assert np.abs(st.U - ref).max() < 1e-7 * np.abs(X).max()
    assert devs[1] < 0.2 * devs[0]


def test_disconnected_graph_collapses_per_component():
    X, M, E, w = mixture_problem(52, n=18, clusters=3, k=2)
    comp, ncomp = graph.components(X.shape[0], E)
    assert ncomp >= 2
    prob, st, info = _pd(X, M, E, w, 50.0, tol=1e-9)
    assert info.fused.all() and info.n_clusters == ncomp
    assert np.array_equal(info.labels, comp)
    for c in np.unique(comp):
        sel = comp == c
        assert np.allclose(st.U[sel].mean(axis=0), X[sel].mean(axis=0), atol=1e-12)
    ref = _fully_fused_fixed_point(prob, info.d, info.rho, X)
    assert np.abs(st.U - ref).max() < 1e-7 * np.abs(X).max()


def test_missing_data_self_consistency():
    X, M, E, w = mixture_problem(61, n=20, p=3, k=4, missing=0.15)
    mu = 0.8
    _, st, info = _pd(X, M, E, w, mu, eta=3e-3, tol=1e-8)
    Y = np.where(M, X, st.U)
    Ustar_Y, gap = certify.dual_solve(Y, E, w, mu)
    assert np.linalg.norm(st.U - Ustar_Y) <= 0.8 * 3e-3 * np.linalg.norm(Y) + np.sqrt(2 * gap)
    # and the missing-data objective is no larger than at the complete-data
    # optimum of the mean-imputed matrix
    Ut, _ = certify.dual_solve(np.where(M, X, 0.0) + np.where(M, 0.0, mm.Problem(X, M, E, w).Xt), E, w, mu)
    fm = certify.convex_objective(np.where(M, X, 0.0), M, st.U, E, w, mu)
    ft = certify.convex_objective(np.where(M, X, 0.0), M, Ut, E, w, mu)
    assert fm <= ft + 1e-6 * abs(ft)
