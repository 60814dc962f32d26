"""Pins for the oracle's MM solver (oracle.mm).

Each test checks the MM iteration against a fact the paper or the
mathematics fixes, not against a retyped copy of the same formula:
  * the U and V updates are the exact minimisers of their blocks of the
    separable surrogate (second_surrogate): checked by numerical minimisation;
  * the projection is the least-squares projection onto C = {(A, D A)}:
    checked with a generic least-squares solver on the stacked system, the
    paper's block-descent cycle, many Jacobi sweeps, and the complete-graph
    closed form;
  * mu = 0 and an empty edge set leave U = X (P:Methods, f_mu at mu = 0);
  * column means are invariant without missing data (D 1 = 0);
  * translation, scaling and permutation equivariance;
  * the MM descent property of the objective (sqrt_root_majorization);
  * the K = 1 Jacobi variant has the exact variant's fixed point.
"""
import numpy as np
import pytest
import scipy.optimize as so

from oracle import certify, mm
from tests._small import mixture_problem


# ---------------------------------------------------------------- updates
@pytest.mark.parametrize("case", range(6))
def test_v_update_is_group_prox(case):
    rng = np.random.default_rng(100 + case)
    b = rng.normal(size=3) * (0.0 if case == 5 else 1.0)
    mu_w = [0.3, 1.0, 5.0, 0.05, 2.0, 1.0][case]
    d, rho = 0.7, 2.0
    s = mm.shrink_factor(np.array([np.linalg.norm(b)]), np.array([mu_w]), d, rho)[0]
    v_closed = s * b
    v_num, f_num = certify.group_shrink_bruteforce(b, mu_w, rho / d)
    f = lambda v: mu_w * np.linalg.norm(v) + 0.5 * (rho / d) * ((v - b) ** 2).sum()
    assert f(v_closed) <= f_num + 1e-10
    assert np.allclose(v_closed, v_num, atol=1e-5)


def test_u_update_minimises_block():
    rng = np.random.default_rng(7)
    y, a = rng.normal(size=4), rng.normal(size=4)
    d, rho = 0.3, 1.7
    f = lambda u: 0.5 * ((y - u) ** 2).sum() + 0.5 * (rho / d) * ((u - a) ** 2).sum()
    res = so.minimize(f, np.zeros(4), method="BFGS", options=dict(gtol=1e-12))
    assert np.allclose(mm.u_update(y, a, d, rho), res.x, atol=1e-7)


# ------------------------------------------------------------- projection
def _rhs(prob, rng):
    U = rng.normal(size=(prob.n, prob.p))
    V = rng.normal(size=(prob.E, prob.p))
    return U, V, U + prob.DT @ V


def test_projection_is_least_squares():
    X, M, E, w = mixture_problem(1, n=14, p=2)
    prob = mm.Problem(X, M, E, w)
    rng = np.random.default_rng(3)
    U, V, rhs = _rhs(prob, rng)
    A = prob.project(rhs, U, "exact")
    # minimise ||A - U||^2 + ||D A - V||^2 with a generic least-squares solver
    K = np.vstack([np.eye(prob.n), prob.D.toarray()])
    A_ls = np.linalg.lstsq(K, np.vstack([U, V]), rcond=None)[0]
    assert np.allclose(A, A_ls, atol=1e-12)


def test_projection_block_descent_and_jacobi_agree():
    X, M, E, w = mixture_problem(2, n=12, p=2)
    prob = mm.Problem(X, M, E, w)
    rng = np.random.default_rng(4)
    U, V, rhs = _rhs(prob, rng)
    A_ex = prob.project(rhs, U, "exact")
    A_gs = prob.project(rhs, U, "gauss_seidel")
    A_j = prob.project(rhs, U, "jacobi:4000")
    assert np.abs(A_gs - A_ex).max() < 1e-12
    assert np.abs(A_j - A_ex).max() < 1e-10


def test_projection_complete_graph_closed_form():
    n, p = 7, 3
    rng = np.random.default_rng(5)
    E = certify.complete_edges(n)
    prob = mm.Problem(rng.normal(size=(n, p)), None, E, np.ones(len(E)))
    U, V, rhs = _rhs(prob, rng)
    assert np.allclose(prob.project(rhs, U, "exact"), certify.complete_projection(rhs), atol=1e-13)


def test_projection_fixes_points_of_C():
    X, M, E, w = mixture_problem(3)
    prob = mm.Problem(X, M, E, w)
    U = np.random.default_rng(6).normal(size=X.shape)
    rhs = U + prob.DT @ (prob.D @ U)
    assert np.allclose(prob.project(rhs, U, "exact"), U, atol=1e-12)
    assert np.allclose(prob.project(rhs, U, "jacobi:1"), U, atol=1e-12)


# --------------------------------------------------------- special cases
def test_mu_zero_and_empty_graph_leave_X():
    X, M, E, w = mixture_problem(4)
    prob = mm.Problem(X, M, E, w)
    st, info = prob.solve(0.0, mm.Opts(tol=0, max_iter=50))
    assert np.abs(st.U - X).max() < 1e-12
    assert info.n_clusters == X.shape[0]
    prob0 = mm.Problem(X, M, np.zeros((0, 2), int), np.zeros(0))
    st0, info0 = prob0.solve(5.0, mm.Opts(tol=0, max_iter=20))
    assert np.abs(st0.U - X).max() < 1e-12


def test_mu_zero_with_missing_keeps_observed():
    X, M, E, w = mixture_problem(5, missing=0.2)
    prob = mm.Problem(X, M, E, w)
    st, _ = prob.solve(0.0, mm.Opts(tol=0, max_iter=30))
    assert np.abs(np.where(M, st.U - X, 0.0)).max() < 1e-12
    # missing entries keep their initial observed-column-mean value
    assert np.abs(np.where(M, 0.0, st.U - prob.Xt)).max() < 1e-12


def test_all_observed_mask_is_no_mask_path():
    X, _, E, w = mixture_problem(6)
    a, ia = mm.Problem(X, None, E, w).solve(0.8, mm.Opts(tol=0, max_iter=200))
    b, ib = mm.Problem(X, np.ones(X.shape, bool), E, w).solve(0.8, mm.Opts(tol=0, max_iter=200))
    assert np.array_equal(a.U, b.U) and np.array_equal(a.s, b.s)


def test_column_means_invariant_every_iteration():
    X, M, E, w = mixture_problem(7, n=20)
    prob = mm.Problem(X, M, E, w)
    rho, eps = prob.constants(1.5, mm.Opts())
    st = prob.initial_state()
    xbar = X.mean(axis=0)
    for _ in range(60):
        st, _ = prob.iterate(1.5, rho, eps, st, "exact")
        assert np.abs(st.U.mean(axis=0) - xbar).max() < 1e-12
        assert np.abs(st.A.mean(axis=0) - xbar).max() < 1e-12


# ---------------------------------------------------------- equivariance
def _fixed(prob, mu, iters=300, proj="exact", **kw):
    return prob.solve(mu, mm.Opts(tol=0, max_iter=iters, proj=proj, **kw))


def test_translation_equivariance():
    X, M, E, w = mixture_problem(8)
    c = np.array([5.0, -3.0, 100.0])
    a, _ = _fixed(mm.Problem(X, M, E, w), 1.2)
    b, _ = _fixed(mm.Problem(X + c, M, E, w), 1.2)
    assert np.abs(b.U - c - a.U).max() < 1e-9
    assert np.array_equal(a.s == 0, b.s == 0)


def test_scaling_equivariance():
    X, M, E, w = mixture_problem(9)
    alpha = 3.5
    a, ia = _fixed(mm.Problem(X, M, E, w), 0.9)
    b, ib = _fixed(mm.Problem(alpha * X, M, E, w), alpha * 0.9)
    assert ib.rho == pytest.approx(alpha * ia.rho, rel=1e-13)
    assert np.abs(b.U - alpha * a.U).max() < 1e-10 * alpha
    assert np.allclose(a.s, b.s, atol=1e-10)


def test_permutation_equivariance():
    X, M, E, w = mixture_problem(10, n=15)
    n = X.shape[0]
    perm = np.random.default_rng(11).permutation(n)      # new index of point i
    Xp = np.empty_like(X)
    Xp[perm] = X
    Ep = np.sort(perm[E], axis=1)
    order = np.lexsort((Ep[:, 1], Ep[:, 0]))
    a, _ = _fixed(mm.Problem(X, M, E, w), 1.1)
    b, _ = _fixed(mm.Problem(Xp, M, Ep[order], w[order]), 1.1)
    assert np.abs(b.U[perm] - a.U).max() < 1e-10
    fperm = np.array([2, 0, 1])
    c, _ = _fixed(mm.Problem(X[:, fperm], M, E, w), 1.1)
    assert np.abs(c.U - a.U[:, fperm]).max() < 1e-10


# ------------------------------------------------------------ MM descent
@pytest.mark.parametrize("missing", [0.0, 0.25])
def test_objective_descends(missing):
    X, M, E, w = mixture_problem(12, n=18, missing=missing)
    prob = mm.Problem(X, M, E, w)
    _, info = prob.solve(1.0, mm.Opts(tol=0, max_iter=400, record=True))
    F = np.array(info.trace_F)
    assert (np.diff(F) <= 1e-12 * np.abs(F[:-1])).all()
    assert F[-1] < F[0]


# ------------------------------------------------------- objective values
def test_objective_value_at_initial_state():
    """The initial state (U_0 = X-tilde, s = 1, A' = U_0) lies in C: its
    projection is itself, so d_0 = sqrt(eps), the loss vanishes on the
    observed entries, and F_0 = mu sum_e w_e ||x~_i - x~_j|| + rho sqrt(eps);
    at mu = 0 that is rho sqrt(eps)."""
    import math
    X, M, E, w = mixture_problem(17, n=15, p=3, missing=0.2)
    prob = mm.Problem(X, M, E, w)
    Xt = prob.Xt
    for mu in (0.0, 0.7, 3.0):
        rho, eps = prob.constants(mu, mm.Opts())
        _, dg = prob.iterate(mu, rho, eps, prob.initial_state(), "exact")
        pen = math.fsum(w[e] * math.sqrt(math.fsum((Xt[E[e, 0], f] - Xt[E[e, 1], f]) ** 2 for f in range(3)))
                        for e in range(len(E)))
        assert dg["d"] == pytest.approx(math.sqrt(eps), rel=1e-12)
        assert dg["F"] == pytest.approx(mu * pen + rho * math.sqrt(eps), rel=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_objective_value_two_points(seed):
    """n = 2, one edge.  The projection keeps the mean of the two rows and
    sets beta = a_1 - a_2 to the minimiser of ||delta - beta||^2/2 +
    ||v - beta||^2, delta = u_1 - u_2, i.e. beta = (delta + 2 v)/3; so
    dist^2 = ||delta - v||^2 / 3 with v = s (a'_1 - a'_2), and
    F = 1/2 ||X - U||^2 + mu w ||v|| + rho sqrt(||delta - v||^2/3 + eps)."""
    import math
    rng = np.random.default_rng(300 + seed)
    p = 4
    X = rng.normal(size=(2, p))
    E = np.array([[0, 1]])
    w = np.array([rng.uniform(0.2, 2.0)])
    prob = mm.Problem(X, None, E, w)
    U, Ap = rng.normal(size=(2, p)), rng.normal(size=(2, p))
    s = np.array([[0.0, 1.0, rng.uniform(0.05, 0.95), 0.5][seed]])
    mu, rho, eps = rng.uniform(0.1, 3.0), rng.uniform(1.0, 5.0), rng.uniform(1e-4, 1e-1)
    v = s[0] * (Ap[0] - Ap[1])
    delta = U[0] - U[1]
    d = math.sqrt(((delta - v) ** 2).sum() / 3.0 + eps)
    F = 0.5 * ((X - U) ** 2).sum() + mu * w[0] * math.sqrt((v ** 2).sum()) + rho * d
    for proj in ("exact", "gauss_seidel", "jacobi:200"):
        _, dg = prob.iterate(mu, rho, eps, mm.State(U.copy(), s.copy(), Ap.copy()), proj)
        assert dg["d"] == pytest.approx(d, rel=1e-12), proj
        assert dg["F"] == pytest.approx(F, rel=1e-12), proj


def test_stopping_rule_semantics():
    X, M, E, w = mixture_problem(13)
    prob = mm.Problem(X, M, E, w)
    _, info = prob.solve(1.0, mm.Opts(tol=0, max_iter=37))
    assert info.iters == 37 and not info.converged
    _, info2 = prob.solve(1.0, mm.Opts(tol=1e-3))
    assert info2.converged and info2.iters >= mm.MIN_TEST_ITER + 1
    assert info2.iters % mm.DEFAULT_TEST_EVERY == 0
    _, info3 = prob.solve(1.0, mm.Opts(tol=1e-3, test_every=1))
    assert info3.converged and info3.iters >= mm.MIN_TEST_ITER + 1


def test_window_test_equals_one_step_test_for_k1():
    """K = 1 is the plain test sqrt(||U_{m+1}-U_m||^2 + ||A_m-A_{m-1}||^2)."""
    X, M, E, w = mixture_problem(16)
    prob = mm.Problem(X, M, E, w)
    rho, eps = prob.constants(1.0, mm.Opts())
    eta = np.sqrt(eps) / rho
    st = prob.initial_state()
    expect = None
    for m in range(5000):
        st2, dg = prob.iterate(1.0, rho, eps, st, "exact")
        r = np.sqrt(dg["dU2"] + dg["dA2"])
        if m >= mm.MIN_TEST_ITER and r <= 1e-4 * eta * max(1.0, np.linalg.norm(st2.U)):
            expect = m + 1
            break
        st = st2
    _, info = prob.solve(1.0, mm.Opts(tol=1e-4, test_every=1))
    assert info.converged and info.iters == expect


def test_jacobi_fixed_point_equals_exact():
    X, M, E, w = mixture_problem(14, n=16)
    prob = mm.Problem(X, M, E, w)
    a, ia = prob.solve(1.0, mm.Opts(tol=1e-9))
    b, ib = prob.solve(1.0, mm.Opts(tol=1e-9, proj="jacobi:1"))
    assert ia.converged and ib.converged
    sc = np.abs(a.U).max()
    assert np.abs(a.U - b.U).max() / sc < 1e-7
    assert np.array_equal(ia.labels, ib.labels)


def test_path_warm_start_matches_cold_solves():
    X, M, E, w = mixture_problem(15, n=16, missing=0.1)
    prob = mm.Problem(X, M, E, w)
    mus = [0.1, 0.5, 2.0]
    _, infos, Us = prob.solve_path(mus, mm.Opts(tol=1e-9))
    for mu, info, U in zip(mus, infos, Us):
        st, ic = prob.solve(mu, mm.Opts(tol=1e-9))
        assert np.abs(st.U - U).max() / np.abs(U).max() < 1e-6
        assert np.array_equal(info.labels, ic.labels)
