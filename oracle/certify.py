"""Independent certificates for convex clustering (FP64).  Test infrastructure
only.  None of these functions runs the MM iteration; they pin it from
outside.

* ``convex_objective``   f_mu(U) of eq_lindsten, or its missing-data form
                         eq_missing_analog when a mask is given.
* ``dual_solve``         the optimum U* of eq_lindsten (complete data) by
                         accelerated projected gradient on the dual
                           max_{||lambda_e|| <= mu w_e}
                               1/2 ||X||^2 - 1/2 ||X - D^T Lambda||^2,
                         with U(Lambda) = X - D^T Lambda.  Returns the duality
                         gap; since f_mu is 1-strongly convex,
                         ||U(Lambda) - U*||_F <= sqrt(2 gap).
* ``brute_force``        for n <= 5 and a complete graph: the minimum of
                         f_mu over every partition of the points into fused
                         groups (Bell(5) = 52), each group sharing one centre,
                         each restricted problem minimised by BFGS.  The best
                         partition is the fusion pattern of U*.
* ``two_point``          n = 2 closed form: the centroid stays fixed and
                         u_1 - u_2 = max(1 - 2 mu w / ||x_1 - x_2||, 0)(x_1 - x_2).
* ``line_complete``      p = 1, complete graph with unit weights: before any
                         fusion u_i = x_i - mu (2 r_i - n - 1), r_i the rank
                         of x_i (valid while every gap exceeds 2 mu).
* ``complete_projection``  (I + L)^{-1} for the complete graph is
                         (I + 1 1^T)/(n + 1).
* ``group_shrink_bruteforce``  numerical minimiser of
                         mu w ||v|| + rho/(2 d) ||v - b||^2 (the V update's
                         block problem), for checking the closed form.

The derivations are written out in the design notes; each is checked in
tests/test_oracle_certify.py.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.optimize as so

from .graph import incidence


def convex_objective(X, mask, U, edges, w, mu) -> float:
    X = np.asarray(X, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    M = np.ones(X.shape, dtype=bool) if mask is None else np.asarray(mask, dtype=bool)
    loss = 0.5 * (np.where(M, X - U, 0.0) ** 2).sum()
    E = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if E.shape[0] == 0:
        return float(loss)
    diff = U[E[:, 0]] - U[E[:, 1]]
    pen = mu * (np.asarray(w) * np.sqrt((diff ** 2).sum(axis=1))).sum()
    return float(loss + pen)


def _project_ball(Lam, radius):
    nrm = np.sqrt((Lam ** 2).sum(axis=1))
    scale = np.ones_like(nrm)
    big = nrm > radius
    scale[big] = radius[big] / nrm[big]
    return Lam * scale[:, None]


def dual_solve(X, edges, w, mu, iters: int = 20000, gap_tol: float = 1e-13):
    """Return (U, gap): U = X - D^T Lambda for the best dual iterate found.

    Accelerated projected gradient (FISTA with gradient-based restart) on
    phi(Lambda) = 1/2 ||X - D^T Lambda||^2 over the product of balls
    ||lambda_e|| <= mu w_e; step 1/lambda_max(L)."""
    X = np.asarray(X, dtype=np.float64)
    n, p = X.shape
    E = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if E.shape[0] == 0 or mu == 0:
        return X.copy(), 0.0
    D = incidence(n, E)
    L = (D.T @ D).toarray()
    step = 1.0 / float(np.linalg.eigvalsh(L).max())
    radius = mu * np.asarray(w, dtype=np.float64)
    Lam = np.zeros((E.shape[0], p))
    Y = Lam.copy()
    t = 1.0
    half_x2 = 0.5 * (X ** 2).sum()
    best_gap, best_U = np.inf, X.copy()
    for it in range(iters):
        Lam_new = _project_ball(Y + step * (D @ (X - D.T @ Y)), radius)
        if np.sum((Y - Lam_new) * (Lam_new - Lam)) > 0:
            t = 1.0                                   # restart momentum
            Y = Lam_new.copy()
        else:
            t_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
            Y = Lam_new + ((t - 1.0) / t_new) * (Lam_new - Lam)
            t = t_new
        Lam = Lam_new
        if it % 25 == 0 or it == iters - 1:
            U = X - D.T @ Lam
            primal = convex_objective(X, None, U, E, w, mu)
            dual = half_x2 - 0.5 * (U ** 2).sum()
            gap = primal - dual
            if gap < best_gap:
                best_gap, best_U = gap, U.copy()
            if gap <= gap_tol * max(1.0, abs(primal)):
                break
    return best_U, float(max(best_gap, 0.0))


def _set_partitions(items):
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in _set_partitions(rest):
        for k in range(len(part)):
            yield part[:k] + [[first] + part[k]] + part[k + 1:]
        yield [[first]] + part


def brute_force(X, w_matrix, mu):
    """X (n, p) with n <= 5; w_matrix (n, n) symmetric, positive off the
    diagonal.  Returns (f_star, best_partition as labels by min index,
    U_star)."""
    X = np.asarray(X, dtype=np.float64)
    n, p = X.shape
    if n > 5:
        raise ValueError("brute force is for n <= 5")
    W = np.asarray(w_matrix, dtype=np.float64)
    best = (np.inf, None, None)
    for part in _set_partitions(list(range(n))):
        K = len(part)
        grp = np.empty(n, dtype=np.int64)
        for k, blk in enumerate(part):
            grp[blk] = k
        cross = [(i, j, W[i, j]) for i in range(n) for j in range(i + 1, n)
                 if grp[i] != grp[j] and W[i, j] > 0]

        def fval(c):
            C = c.reshape(K, p)
            val = 0.5 * ((X - C[grp]) ** 2).sum()
            g = np.zeros_like(C)
            for i in range(n):
                g[grp[i]] += C[grp[i]] - X[i]
            for i, j, wij in cross:
                dvec = C[grp[i]] - C[grp[j]]
                nrm = np.sqrt((dvec ** 2).sum())
                val += mu * wij * nrm
                if nrm > 0:
                    g[grp[i]] += mu * wij * dvec / nrm
                    g[grp[j]] -= mu * wij * dvec / nrm
            return val, g.reshape(-1)

        c0 = np.stack([X[blk].mean(axis=0) for blk in part])
        res = so.minimize(fval, c0.reshape(-1), jac=True, method="BFGS",
                          options=dict(gtol=1e-12, maxiter=10000))
        if res.fun < best[0]:
            C = res.x.reshape(K, p)
            lab = np.empty(n, dtype=np.int64)
            for blk in part:
                lab[blk] = min(blk)
            best = (float(res.fun), lab, C[grp].copy())
    return best


def two_point(x1, x2, w, mu):
    """Closed-form optimum for n = 2 (eq_lindsten)."""
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    c = 0.5 * (x1 + x2)
    delta = x1 - x2
    nrm = np.sqrt((delta ** 2).sum())
    fac = max(1.0 - 2.0 * mu * w / nrm, 0.0) if nrm > 0 else 0.0
    return np.stack([c + 0.5 * fac * delta, c - 0.5 * fac * delta])


def line_complete(x, mu):
    """p = 1, unit weights on every pair: u_i = x_i - mu (2 r_i - n - 1) with
    r_i the 1-based rank; valid while min gap > 2 mu."""
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    n = x.size
    r = np.empty(n)
    r[np.argsort(x, kind="stable")] = np.arange(1, n + 1)
    return x - mu * (2.0 * r - n - 1.0)


def complete_projection(rhs):
    """(I + L)^{-1} rhs for the complete graph on the rows of rhs."""
    rhs = np.asarray(rhs, dtype=np.float64)
    n = rhs.shape[0]
    return (rhs + rhs.sum(axis=0, keepdims=True)) / (n + 1.0)


def complete_edges(n):
    return np.array(list(itertools.combinations(range(n), 2)), dtype=np.int64).reshape(-1, 2)


def group_shrink_bruteforce(b, mu_w, rho_over_d):
    """Numerically minimise mu_w ||v|| + rho_over_d/2 ||v - b||^2."""
    b = np.asarray(b, dtype=np.float64)

    def f(v):
        return mu_w * np.sqrt((v ** 2).sum() + 1e-300) + 0.5 * rho_over_d * ((v - b) ** 2).sum()

    best = None
    for v0 in (b.copy(), np.zeros_like(b), 0.5 * b):
        res = so.minimize(f, v0, method="Nelder-Mead",
                          options=dict(xatol=1e-12, fatol=1e-15, maxiter=40000))
        if best is None or res.fun < best.fun:
            best = res
    return best.x, best.fun
