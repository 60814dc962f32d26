"""The proximal-distance MM algorithm for convex clustering (oracle, FP64).
Test infrastructure only.

What is computed (Methods, "The Proximal Distance Algorithm" and "Missing
Data"):

  Split v_ij = u_i - u_j (eq_proxdist); C = {(U, V): V = D U}.  With the
  smoothed distance dist_eps = sqrt(dist^2 + eps) and the two majorisations
  (first_surrogate, sqrt_root_majorization) one MM iteration from (U_m, V_m) is

    1. projection   (A_m, B_m) = P_C(U_m, V_m), i.e. (I + D^T D) A_m =
                    U_m + D^T V_m and B_m = D A_m (block-descent section);
    2. distance     d_m = sqrt(||U_m - A_m||^2 + ||V_m - B_m||^2 + eps)
                    (second_surrogate);
    3. V update     v_{m+1,e} = max(1 - mu w_e d_m / (rho ||b_e||), 0) b_e,
                    and 0 when b_e = 0 (group soft-threshold);
    4. U update     u_{m+1,i} = (d_m y_i + rho a_i) / (d_m + rho), where
                    Y = X on observed entries and U_m elsewhere
                    (eq_missing_analog majorisation; Y = X without missing data).

  V is kept in factored form: after any V update V = diag(s) D A' with A' the
  projection it was shrunk from, so the state is (U, s, A').  This is exact,
  not an approximation: step 3 multiplies each b_e = (D A_m)_e by a scalar.

Projection modes:
  * "exact"        Cholesky solve of (I + L) A = U + D^T V (what the paper's
                   block descent converges to);
  * "gauss_seidel" the paper's block descent itself: cycle i = 1..n through
                   a_i = (u_i + sum_R v_ij - sum_L v_ji + sum_N a_j)/(1+|N_i|)
                   until the iterates stop changing (pure Python, tiny inputs);
  * "jacobi:K"     K Jacobi sweeps of the same block update, started from the
                   previous projection A' (what the GPU path runs, K = 1).
                   Its fixed points are those of the exact mode.

Readings where the paper is silent (each listed in the design notes):
  * rho = 2 sqrt(||M o (X - xbar)||^2 + mu^2 sum_e w_e^2): an upper bound on
    the norm of the multiplier at the optimum, so the exact-penalty condition
    "rho bigger than a Lipschitz constant" holds;
  * eps = (eta rho)^2 with eta = 1e-2 by default;
  * initial state U_0 = X-tilde (missing -> observed column mean), s_0 = 1,
    A' = U_0, so V_0 = D U_0 lies in C;
  * a path warm-starts each mu from the previous mu's final state;
  * stopping: the test is taken after iterations m >= 2 with (m+1) a
    multiple of the window K (test_every, default 64), on the mean
    displacement over the window,
      r = sqrt(||U_{m+1} - U_{m+1-K}||^2 + ||A_m - A_{m-K}||^2) / K
          <= tol * eta * max(1, ||U_{m+1}||_F),      eta = sqrt(eps)/rho,
    or the solve ends after max_iter iterations; tol = 0 turns the test
    off.  K = 1 is the plain one-step test.  The window makes the decision
    insensitive to rounding-level jitter of reduced-precision state;
  * the reported solution is U_{m+1}; edge e is fused when s_{m+1,e} = 0; the
    clusters are the connected components of the fused edges, each labelled
    by its smallest point index.

Objective reported per iteration (the quantity the MM drives downhill):
  F_m = 1/2 sum_{observed} (x - u_m)^2 + mu sum_e w_e ||v_{m,e}|| + rho d_m.

Parity pins: tests/test_oracle_mm.py and tests/test_oracle_certify.py.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .graph import adjacency, components, degrees, incidence, validate_edges
from .prep import impute_column_means, observed_column_means

DEFAULT_ETA = 1e-2
DEFAULT_TOL = 1e-6
DEFAULT_MAX_ITER = 200_000
DEFAULT_TEST_EVERY = 64
MIN_TEST_ITER = 2


def shrink_factor(nb, mu_w, d, rho):
    """V update (group soft-threshold): v = s b with
    s = max(1 - mu w d / (rho ||b||), 0), and s = 0 when b = 0."""
    nb = np.asarray(nb, dtype=np.float64)
    tau = np.asarray(mu_w, dtype=np.float64) * d / rho
    s = np.zeros(nb.shape)
    pos = nb > 0
    s[pos] = np.maximum(1.0 - tau[pos] / nb[pos], 0.0)
    return s


def u_update(Y, A, d, rho):
    """U update: u_i = (d y_i + rho a_i) / (d + rho)."""
    return (d * Y + rho * A) / (d + rho)


@dataclass
class Opts:
    eta: float = DEFAULT_ETA
    rho: Optional[float] = None   # None -> default rule
    eps: Optional[float] = None   # None -> (eta * rho)^2
    tol: float = DEFAULT_TOL
    max_iter: int = DEFAULT_MAX_ITER
    test_every: int = DEFAULT_TEST_EVERY  # stop-test window K
    proj: str = "exact"           # "exact" | "gauss_seidel" | "jacobi:K"
    record: bool = False          # keep per-iteration F and d


@dataclass
class State:
    U: np.ndarray   # (n, p) centres
    s: np.ndarray   # (E,)  shrink factors: V = diag(s) D A
    A: np.ndarray   # (n, p) projection the current V was shrunk from

    def copy(self) -> "State":
        return State(self.U.copy(), self.s.copy(), self.A.copy())


@dataclass
class Info:
    iters: int = 0
    converged: bool = False
    objective: float = np.nan
    d: float = np.nan
    rel_change: float = np.nan
    rho: float = np.nan
    eps: float = np.nan
    n_clusters: int = 0
    labels: Optional[np.ndarray] = None
    fused: Optional[np.ndarray] = None
    trace_F: List[float] = field(default_factory=list)
    trace_d: List[float] = field(default_factory=list)


class Problem:
    """X (n, p) with optional mask (True = observed), edges (E, 2) with i < j,
    weights w (E,) > 0."""

    def __init__(self, X, mask, edges, w):
        X = np.asarray(X, dtype=np.float64)
        if X.ndim != 2 or X.shape[0] < 1 or X.shape[1] < 1:
            raise ValueError("X must be (n, p) with n, p >= 1")
        self.n, self.p = X.shape
        self.M = (np.ones(X.shape, dtype=bool) if mask is None
                  else np.asarray(mask, dtype=bool).copy())
        if self.M.shape != X.shape:
            raise ValueError("mask shape")
        if not np.isfinite(X[self.M]).all():
            raise ValueError("observed X must be finite")
        self.has_missing = not self.M.all()
        self.X = np.where(self.M, X, 0.0)           # missing entries unused
        self.Xt = impute_column_means(X, self.M)    # X-tilde
        self.edges = validate_edges(self.n, edges)
        self.w = np.asarray(w, dtype=np.float64).reshape(-1)
        if self.w.shape[0] != self.edges.shape[0]:
            raise ValueError("one weight per edge")
        if not (np.isfinite(self.w).all() and (self.w > 0).all()):
            raise ValueError("weights must be finite and > 0")
        self.E = self.edges.shape[0]
        self.D = incidence(self.n, self.edges)
        self.DT = self.D.T.tocsr()
        self.Adj = adjacency(self.n, self.edges)
        self.deg = degrees(self.n, self.edges).astype(np.float64)
        self._chol = None

    # ---- defaults (readings of the paper's "rho large", "eps small") ----
    def default_rho(self, mu: float) -> float:
        xbar = observed_column_means(np.where(self.M, self.X, np.nan), self.M)
        dev = np.where(self.M, self.X - xbar[None, :], 0.0)
        val = 2.0 * np.sqrt((dev ** 2).sum() + mu * mu * (self.w ** 2).sum())
        return float(val) if val > 0 else 1.0

    def constants(self, mu: float, opts: Opts):
        rho = opts.rho if (opts.rho is not None and opts.rho > 0) else self.default_rho(mu)
        eps = opts.eps if (opts.eps is not None and opts.eps > 0) else (opts.eta * rho) ** 2
        return rho, eps

    def initial_state(self) -> State:
        return State(self.Xt.copy(), np.ones(self.E), self.Xt.copy())

    # ---- projection onto C ----
    def _cholesky(self):
        if self._chol is None:
            L = (self.D.T @ self.D).toarray()
            self._chol = sla.cho_factor(np.eye(self.n) + L, lower=True)
        return self._chol

    def project(self, rhs: np.ndarray, A0: np.ndarray, mode: str) -> np.ndarray:
        """Solve (I + L) A = rhs (exact), or approximate it from A0."""
        if mode == "exact":
            if self.E == 0:
                return rhs.copy()
            return sla.cho_solve(self._cholesky(), rhs)
        if mode.startswith("jacobi"):
            K = int(mode.split(":")[1]) if ":" in mode else 1
            A = A0.copy()
            for _ in range(K):
                A = (rhs + self.Adj @ A) / (1.0 + self.deg)[:, None]
            return A
        if mode == "gauss_seidel":
            return self._gauss_seidel(rhs, A0)
        raise ValueError(f"unknown projection mode {mode!r}")

    def _gauss_seidel(self, rhs, A0, tol=1e-15, max_cycles=100_000):
        nbrs = [[] for _ in range(self.n)]
        for i, j in self.edges.tolist():
            nbrs[i].append(j)
            nbrs[j].append(i)
        A = A0.copy()
        scale = max(1.0, float(np.abs(rhs).max()))
        for _ in range(max_cycles):
            change = 0.0
            for i in range(self.n):
                new = (rhs[i] + A[nbrs[i]].sum(axis=0)) / (1.0 + len(nbrs[i]))
                change = max(change, float(np.abs(new - A[i]).max()))
                A[i] = new
            if change <= tol * scale:
                break
        return A

    # ---- one MM iteration ----
    def iterate(self, mu: float, rho: float, eps: float, st: State, proj: str):
        """One MM iteration from st = (U_m, s_m, A_{m-1}).  Returns the next
        state (U_{m+1}, s_{m+1}, A_m) and a dict of diagnostics."""
        U, s, Ap = st.U, st.s, st.A
        Bp = self.D @ Ap                       # (D A_{m-1})
        V = s[:, None] * Bp                    # V_m
        rhs = U + self.DT @ V                  # U_m + D^T V_m
        A = self.project(rhs, Ap, proj)        # A_m
        B = self.D @ A                         # B_m = D A_m
        dist2 = ((U - A) ** 2).sum() + ((V - B) ** 2).sum()
        d = np.sqrt(dist2 + eps)               # d_m
        nb = np.sqrt((B ** 2).sum(axis=1))     # ||b_e||
        s_new = shrink_factor(nb, mu * self.w, d, rho)
        Y = np.where(self.M, self.X, U)
        U_new = u_update(Y, A, d, rho)
        loss = 0.5 * (np.where(self.M, self.X - U, 0.0) ** 2).sum()
        pen = mu * (self.w * np.sqrt((V ** 2).sum(axis=1))).sum()
        F = loss + pen + rho * d
        diag = dict(d=float(d), F=float(F), nb=nb, dist2=float(dist2),
                    dU2=float(((U_new - U) ** 2).sum()),
                    dA2=float(((A - Ap) ** 2).sum()))
        return State(U_new, s_new, A), diag

    # ---- solve at one mu ----
    def solve(self, mu: float, opts: Optional[Opts] = None,
              state: Optional[State] = None):
        opts = opts or Opts()
        rho, eps = self.constants(mu, opts)
        eta = np.sqrt(eps) / rho
        st = self.initial_state() if state is None else state.copy()
        info = Info(rho=rho, eps=eps)
        K = max(1, int(opts.test_every))
        U_snap = st.U.copy()   # U_{m+1-K} at the next test
        A_snap = st.A.copy()   # A_{m-K} at the next test
        for m in range(opts.max_iter):
            st, dg = self.iterate(mu, rho, eps, st, opts.proj)
            info.iters = m + 1
            info.objective, info.d = dg["F"], dg["d"]
            if opts.record:
                info.trace_F.append(dg["F"])
                info.trace_d.append(dg["d"])
            if (m + 1) % K != 0:
                continue
            r = np.sqrt(((st.U - U_snap) ** 2).sum() + ((st.A - A_snap) ** 2).sum()) / K
            U_snap = st.U.copy()
            A_snap = st.A.copy()
            unorm = max(1.0, float(np.sqrt((st.U ** 2).sum())))
            info.rel_change = r / unorm
            if opts.tol > 0 and m >= MIN_TEST_ITER and r <= opts.tol * eta * unorm:
                info.converged = True
                break
        fused = st.s == 0.0
        labels, ncl = components(self.n, self.edges, fused)
        info.fused, info.labels, info.n_clusters = fused, labels, ncl
        return st, info

    def solve_path(self, mus, opts: Optional[Opts] = None,
                   state: Optional[State] = None, keep_U: bool = True):
        """Solve along mus in the given order, warm-starting each from the
        previous final state.  Returns (final state, [info], [U per mu])."""
        st = self.initial_state() if state is None else state.copy()
        infos, Us = [], []
        for mu in mus:
            st, info = self.solve(float(mu), opts, st)
            infos.append(info)
            if keep_U:
                Us.append(st.U.copy())
        return st, infos, Us


def solve(X, mask, edges, w, mu, opts: Optional[Opts] = None):
    """Convenience: build the problem and solve at one mu from the initial
    state.  Returns (U, info)."""
    prob = Problem(X, mask, edges, w)
    st, info = prob.solve(mu, opts)
    return st.U, info


def with_opts(opts: Optional[Opts], **kw) -> Opts:
    return replace(opts or Opts(), **kw)
