"""Served solves (continuous batching): requests that arrive while others
run share the launches and give the same results as when solved alone,
within the stated tolerance; admission follows the HBM budget."""
import numpy as np
import pytest
import torch

import gen

from _gpu import rel_max

pytestmark = pytest.mark.gpu

GAMMAS = [1e-2, 1.0, 10.0, 100.0]
OPTS = dict(max_iter=20000, tol=1e-6)


@pytest.fixture(scope="module")
def cc():
    import paper_1409_2065_amd as cc
    cc.load()
    return cc


def request(seed, n, p, clusters, missing):
    rng = np.random.default_rng(seed)
    X, _ = gen.gaussian_mixture(rng, n, p, clusters)
    X = np.asarray(X, dtype=np.float32)
    mask = (rng.random((n, p)) >= missing).astype(np.uint8) if missing > 0 else None
    return X, mask


def alone(cc, X, mask, k=10, phi=-0.5, precision="mixed"):
    Xt = torch.tensor(X * (mask if mask is not None else 1), dtype=torch.float32, device="cuda")
    M = None if mask is None else torch.tensor(mask, device="cuda")
    e, w, _ = cc.build_knn_weights(Xt, M, k=k, phi=phi)
    with cc.Problem(Xt, M, e, w, precision=precision) as pr:
        infos, lab, _ = pr.solve_path(GAMMAS, labels=True, **OPTS)
        U = pr.U().cpu().numpy()
    return lab.cpu().numpy(), infos, U


# (seed, n, p, clusters, missing): features per lane 1, 8, 16 and 1
SPECS = [(11, 60, 20, 3, 0.0), (12, 150, 300, 4, 0.1), (13, 90, 700, 3, 0.1), (14, 200, 40, 5, 0.0)]


@pytest.mark.parametrize("precision", ["mixed", "f64"])
def test_server_mix_equals_alone(cc, precision):
    reqs = [request(*s) for s in SPECS]
    with cc.Server(precision, hbm_budget=8 << 30, round_iters=32, **OPTS) as srv:
        tickets = [srv.submit(X, m, k=10, phi=-0.5, gammas=GAMMAS) for X, m in reqs[:2]]
        srv.step()
        srv.step()
        # two more arrive while the first two run
        tickets += [srv.submit(X, m, k=10, phi=-0.5, gammas=GAMMAS) for X, m in reqs[2:]]
        states = {}
        for _ in range(100000):
            a, w, d = srv.step()
            if a == 0 and w == 0:
                break
        for t in tickets:
            st = srv.status(t)
            assert st["state"] == 2, st
            assert st["t_submit"] <= st["t_admit"] <= st["t_done"]
            states[t] = srv.result(t, U=True)
        for t in tickets:
            srv.release(t)
    for (X, m), t in zip(reqs, tickets):
        lab, infos, U = states[t]
        rlab, rinf, rU = alone(cc, X, m, precision=precision)
        for k in range(len(GAMMAS)):
            assert infos[k]["converged"] == rinf[k]["converged"], (t, k)
            if rinf[k]["converged"]:
                assert np.array_equal(lab[k].cpu().numpy(), rlab[k]), (t, k)
                assert infos[k]["n_clusters"] == rinf[k]["n_clusters"]
        if rinf[-1]["converged"]:
            assert rel_max(U.cpu().numpy(), rU) < 1e-5, t


def test_server_budget_admission(cc):
    reqs = [request(20 + s, 80, 30, 3, 0.0) for s in range(3)]
    with cc.Server("mixed", hbm_budget=1, round_iters=16, **OPTS) as srv:
        tickets = [srv.submit(X, m, k=8, gammas=GAMMAS[:2]) for X, m in reqs]
        a, w, _ = srv.step()
        assert a == 1 and w == 2  # one at a time within a 1-byte budget
        seen_active = {a}
        for _ in range(100000):
            a, w, d = srv.step()
            seen_active.add(a)
            if a == 0 and w == 0:
                break
        assert seen_active <= {0, 1}
        t_admit = [srv.status(t)["t_admit"] for t in tickets]
        assert t_admit == sorted(t_admit)  # first come, first served
        for t in tickets:
            lab, infos, _ = srv.result(t)
            assert lab.shape == (2, 80) and all(i["iters"] > 0 for i in infos)
            srv.release(t)


def test_server_rejects_bad_requests(cc):
    with cc.Server("mixed") as srv:
        with pytest.raises(cc.CCError):
            srv.submit(np.zeros((10, 1100), np.float32), gammas=[1.0])  # p > 1024
        with pytest.raises(cc.CCError):
            srv.submit(np.zeros((10, 5), np.float32), k=10, gammas=[1.0])  # k >= n
        with pytest.raises(cc.CCError):
            srv.submit(np.zeros((10, 5), np.float32), gammas=[])
        with pytest.raises(cc.CCError):
            srv.release(12345)


def test_server_memory_accounting_and_failed_admission(cc):
    """Bytes counted against the budget rise with admissions and return to
    zero once every request is released; a request whose admission fails
    (observed X not finite: the weights refuse it) ends FAILED, reports its
    error through the result call and is never counted."""
    import ctypes as C
    from paper_1409_2065_amd import _lib
    reqs = [request(30 + s, 70, 25, 3, 0.0) for s in range(2)]
    gam = np.asarray(GAMMAS[:2], dtype=np.float64)
    with cc.Server("mixed", hbm_budget=8 << 30, round_iters=16, **OPTS) as srv:
        assert srv.memory() == (0, 8 << 30)
        bad = np.ascontiguousarray(reqs[0][0].copy())
        bad[3, 4] = np.nan
        t = C.c_int64()
        # straight through the C ABI: the Python wrapper would replace the NaN
        st = _lib.load().cc_server_submit(srv._h, 70, 25, bad.ctypes.data_as(C.c_void_p), None, 8, -0.5,
                                          gam.size, gam.ctypes.data_as(_lib.P_f64), C.byref(t))
        assert st == _lib.CC_OK
        tb = t.value
        srv._shape[tb] = (70, 25, gam.size)
        tickets = [srv.submit(X, m, k=8, gammas=gam) for X, m in reqs]
        a, w, _ = srv.step()
        assert srv.status(tb)["state"] == _lib.CC_REQ_FAILED
        assert a == 2 and w == 0
        used = srv.memory()[0]
        assert used > 0
        with pytest.raises(cc.CCError) as ei:
            srv.result(tb)
        assert ei.value.status == _lib.CC_ERR_INVALID_ARG and "non-finite" in str(ei.value)
        srv.release(tb)
        assert srv.memory()[0] == used
        for _ in range(100000):
            a, w, d = srv.step()
            if a == 0 and w == 0:
                break
        assert srv.memory()[0] == used  # finished requests keep their results
        for tk in tickets:
            assert srv.status(tk)["state"] == _lib.CC_REQ_DONE
            srv.release(tk)
        assert srv.memory()[0] == 0


def test_served_requests_match_oracle(cc):
    """Served requests (continuous batching, the second joining while the
    first runs) against the FP64 oracle on its own kNN weights of the same
    data and mask: every gamma the oracle's stopping test passes is also
    converged on the server, with the same labels; the centres after the
    path agree within 1e-5.  Both sides stop at tol 1e-4 or 5000 MM
    iterations per gamma (tighter than the benchmark's tol 1e-3 and
    1000-iteration cap)."""
    from oracle import mm, weights
    specs = [(41, 60, 20, 3, 0.1), (42, 120, 30, 4, 0.1), (43, 90, 50, 3, 0.0)]
    gam = [1e-2, 1.0, 10.0, 100.0]
    opts = dict(max_iter=5000, tol=1e-4)
    reqs = [request(*s) for s in specs]
    with cc.Server("mixed", hbm_budget=8 << 30, round_iters=32, **opts) as srv:
        tickets = [srv.submit(reqs[0][0], reqs[0][1], k=10, phi=-0.5, gammas=gam)]
        srv.step()
        tickets += [srv.submit(X, m, k=10, phi=-0.5, gammas=gam) for X, m in reqs[1:]]
        for _ in range(100000):
            a, w, _ = srv.step()
            if a == 0 and w == 0:
                break
        res = [srv.result(t, U=True) for t in tickets]
    for (X, m), (lab, infos, U) in zip(reqs, res):
        Xd = X.astype(np.float64)
        M = None if m is None else m.astype(bool)
        Xn = Xd if M is None else np.where(M, Xd, np.nan)
        E, w, _ = weights.knn_weights(Xn, M, 10, -0.5)
        _, oinf, oU = mm.Problem(Xn, M, E, w).solve_path(gam, mm.Opts(proj="jacobi:1", **opts))
        assert any(i.converged for i in oinf)
        for k, oi in enumerate(oinf):
            if oi.converged:
                assert infos[k]["converged"] == 1, (k, infos[k])
                assert np.array_equal(lab[k].cpu().numpy(), oi.labels), k
                assert infos[k]["n_clusters"] == oi.n_clusters
        assert oinf[-1].converged
        assert rel_max(U.cpu().numpy(), oU[-1]) < 1e-5
