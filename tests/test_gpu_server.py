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


def alone(cc, X, mask, k=10, phi=-0.5):
    Xt = torch.tensor(X * (mask if mask is not None else 1), dtype=torch.float32, device="cuda")
    M = None if mask is None else torch.tensor(mask, device="cuda")
    e, w, _ = cc.build_knn_weights(Xt, M, k=k, phi=phi)
    with cc.Problem(Xt, M, e, w, precision="mixed") as pr:
        infos, lab, _ = pr.solve_path(GAMMAS, labels=True, **OPTS)
        U = pr.U().cpu().numpy()
    return lab.cpu().numpy(), infos, U


# (seed, n, p, clusters, missing): features per lane 1, 8, 16 and 1
SPECS = [(11, 60, 20, 3, 0.0), (12, 150, 300, 4, 0.1), (13, 90, 700, 3, 0.1), (14, 200, 40, 5, 0.0)]


def test_server_mix_equals_alone(cc):
    reqs = [request(*s) for s in SPECS]
    with cc.Server("mixed", hbm_budget=8 << 30, round_iters=32, **OPTS) as srv:
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
        rlab, rinf, rU = alone(cc, X, m)
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
