"""The oracle's pins have teeth: each plausible mistake planted in the MM
iteration (a dropped term, a wrong sign, swapped operands, an ignored mask)
makes at least one certificate check fail.  Mistakes are planted in
subclasses of the oracle on the CPU; the oracle itself is untouched."""
import numpy as np
import pytest

from oracle import certify, mm
from tests._small import mixture_problem


def _iterate_variant(self, mu, rho, eps, st, proj, bug):
    U, s, Ap = st.U, st.s, st.A
    Bp = self.D @ Ap
    V = s[:, None] * Bp
    rhs = U - self.DT @ V if bug == "rhs_sign" else U + self.DT @ V
    A = self.project(rhs, Ap, proj)
    B = self.D @ A
    dist2 = ((U - A) ** 2).sum()
    if bug != "drop_v_distance":
        dist2 += ((V - B) ** 2).sum()
    d = np.sqrt(dist2 + eps)
    nb = np.sqrt((B ** 2).sum(axis=1))
    if bug == "shrink_without_d":
        s_new = mm.shrink_factor(nb, mu * self.w, 1.0, rho)
    else:
        s_new = mm.shrink_factor(nb, mu * self.w, d, rho)
    Y = self.X if bug == "ignore_mask" else np.where(self.M, self.X, U)
    if bug == "swap_d_rho":
        U_new = mm.u_update(Y, A, rho, d)
    else:
        U_new = mm.u_update(Y, A, d, rho)
    loss = 0.5 * (np.where(self.M, self.X - U, 0.0) ** 2).sum()
    pen = mu * (self.w * np.sqrt((V ** 2).sum(axis=1))).sum()
    F = loss + pen + rho * d
    return mm.State(U_new, s_new, A), dict(
        d=float(d), F=float(F), nb=nb, dist2=float(dist2),
        dU2=float(((U_new - U) ** 2).sum()), dA2=float(((A - Ap) ** 2).sum()))


def _make(bug):
    class P(mm.Problem):
        def iterate(self, mu, rho, eps, st, proj):
            return _iterate_variant(self, mu, rho, eps, st, proj, bug)
    return P


def _battery(P):
    """Return the list of checks that fail for problem class P."""
    failed = []
    X, M, E, w = mixture_problem(71, n=16, p=3, k=4)
    prob = P(X, M, E, w)
    st, info = prob.solve(1.0, mm.Opts(tol=1e-7, max_iter=30000, record=True))
    Ustar, gap = certify.dual_solve(X, E, w, 1.0)
    if not np.linalg.norm(st.U - Ustar) <= 0.8e-2 * np.linalg.norm(X) + np.sqrt(2 * gap):
        failed.append("certificate")
    F = np.array(info.trace_F)
    if not (np.diff(F) <= 1e-12 * np.abs(F[:-1])).all():
        failed.append("descent")
    Xm, Mm, Em, wm = mixture_problem(72, n=16, p=3, k=4, missing=0.2)
    pm = P(Xm, Mm, Em, wm)
    st0, _ = pm.solve(0.0, mm.Opts(tol=0, max_iter=40))
    if not (np.abs(np.where(Mm, st0.U - Xm, 0.0)).max() < 1e-12
            and np.abs(np.where(Mm, 0.0, st0.U - pm.Xt)).max() < 1e-12):
        failed.append("mu0_missing")
    return failed


def test_correct_oracle_passes_battery():
    assert _battery(mm.Problem) == []
    assert _battery(_make(None)) == []


@pytest.mark.parametrize("bug", ["rhs_sign", "drop_v_distance", "shrink_without_d",
                                 "ignore_mask", "swap_d_rho"])
def test_planted_mistake_is_caught(bug):
    assert _battery(_make(bug)) != []
