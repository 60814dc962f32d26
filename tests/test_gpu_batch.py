"""Batched solves (many instances along their own gamma paths in the same
launches) against the plain per-problem path: the same labels, infos and
final state, bitwise when both use the same tile shapes."""
import numpy as np
import pytest
import torch

import gen
from oracle import weights

from _gpu import rel_max, to_dev

pytestmark = pytest.mark.gpu

OPTS = dict(max_iter=3000, tol=1e-6)


@pytest.fixture(scope="module")
def cc():
    import paper_1409_2065_amd as cc
    cc.load()
    return cc


def instance(b):
    wl = gen.batched_instance(b)
    X = np.asarray(wl.X, dtype=np.float32).astype(np.float64)
    edges, w, _ = weights.knn_weights(X, None, wl.k, wl.phi)
    return X, edges, w, [float(g) for g in wl.gammas[::5]]


def make(cc, X, edges, w, precision="mixed"):
    Xt, _, e, wt = to_dev(X, None, edges, w, torch.float32)
    return cc.Problem(Xt, None, e, wt, precision=precision)


def alone(cc, X, edges, w, gammas, precision="mixed"):
    with make(cc, X, edges, w, precision) as pr:
        infos, lab, _ = pr.solve_path(gammas, labels=True, **OPTS)
        U, A, s = (t.cpu().numpy() for t in pr.get_state())
    return infos, lab.cpu().numpy(), U, A, s


@pytest.mark.parametrize("precision", ["f32", "mixed", "f64"])
def test_batch_equals_alone_bitwise(cc, monkeypatch, precision):
    # p in (128, 256]: both sweeps take 4 features per lane alone and batched
    ids = [31, 33, 37, 22]
    inst = [instance(b) for b in ids]
    monkeypatch.setenv("CCMI_VEC", "4")
    monkeypatch.setenv("CCMI_EDGE_IPW", "4")  # the batched edge sweep's items per wave
    ref = [alone(cc, X, e, w, g, precision) for X, e, w, g in inst]
    probs = [make(cc, X, e, w, precision) for X, e, w, _ in inst]
    with cc.Batch(probs, [g for *_, g in inst], autotune=False, **OPTS) as bt:
        assert bt.config()["vec"] == 4
        labs, infos, lat = bt.run()
    assert np.all(lat > 0)
    for b, (pr, (rinf, rlab, rU, rA, rs)) in enumerate(zip(probs, ref)):
        U, A, s = (t.cpu().numpy() for t in pr.get_state())
        assert np.array_equal(labs[b].cpu().numpy(), rlab), ids[b]
        assert np.array_equal(U, rU) and np.array_equal(A, rA) and np.array_equal(s, rs), ids[b]
        for k, (i1, i2) in enumerate(zip(infos[b], rinf)):
            for key in ("iters", "converged", "n_clusters", "objective", "d", "rho", "eps"):
                assert i1[key] == i2[key], (ids[b], k, key, i1[key], i2[key])
        assert max(i["seconds"] for i in infos[b]) <= lat[b] / 1e3 + 1e-9
        pr.close()


def test_batch_mixed_shapes_autotuned(cc):
    # different widths and sizes in one batch, tile width picked by the autotuner
    ids = [14, 24, 3, 30, 11]
    inst = [instance(b) for b in ids]
    ref = [alone(cc, X, e, w, g) for X, e, w, g in inst]
    probs = [make(cc, X, e, w) for X, e, w, _ in inst]
    with cc.Batch(probs, [g for *_, g in inst], autotune=True, **OPTS) as bt:
        cfg = bt.config()
        assert cfg["vec"] in (1, 2, 4) and cfg["items_per_wave"] in (1, 4, 16)
        assert len(cfg["tune_us"]) == 9 and all(t > 0 for t in cfg["tune_us"])
        classes, of = bt.tuning()
        # one class per (row width, work) group; every instance in exactly one
        assert sum(c["instances"] for c in classes) == len(ids)
        assert sorted(set(of)) == list(range(len(classes)))
        for c in classes:
            assert c["vec"] in (1, 2, 4) and c["items_per_wave"] in (1, 4, 16) and c["us_per_iteration"] > 0
        for b, (X, *_rest) in enumerate(inst):
            p = X.shape[1]
            assert classes[of[b]]["width_class"] == (0 if p <= 64 else 1 if p <= 128 else 2 if p <= 256 else 3)
        labs, infos, lat = bt.run()
    for b, (pr, (rinf, rlab, rU, rA, rs)) in enumerate(zip(probs, ref)):
        U = pr.get_state()[0].cpu().numpy()
        for k in range(len(rinf)):
            assert infos[b][k]["converged"] == rinf[k]["converged"], (ids[b], k)
            if rinf[k]["converged"]:
                assert np.array_equal(labs[b][k].cpu().numpy(), rlab[k]), (ids[b], k)
        assert rel_max(U, rU) < 1e-5, ids[b]
        pr.close()


def test_batch_rejects_bad_input(cc):
    X, e, w, g = instance(14)
    pr = make(cc, X, e, w)
    with pytest.raises(cc.CCError):
        cc.Batch([pr, pr], [g, g], autotune=False)  # the same problem twice
    with pytest.raises(cc.CCError):
        cc.Batch([pr], [[]], autotune=False)  # empty path
    pr64 = make(cc, X, e, w, precision="f64")
    with pytest.raises(cc.CCError):
        cc.Batch([pr, pr64], [g, g], autotune=False)  # mixed precisions
    pr.close()
    pr64.close()


def test_batched_instances_match_oracle(cc):
    """Batched instances (in shared launches with others) against the FP64
    oracle on the same edges and weights: every gamma the oracle's stopping
    test passes is converged in the batch too, with the same labels and
    iteration count within one test window; the centres after each gamma
    (from the same instance solved alone, which the batch equals bitwise)
    and after the path agree within 1e-5.  Both sides stop at tol 1e-4 or
    5000 MM iterations per gamma (tighter than the benchmark's tol 1e-3 and
    1000-iteration cap)."""
    from oracle import mm
    opts = dict(max_iter=5000, tol=1e-4)
    ids = [14, 3, 24, 31, 2]
    inst = []
    for b in ids:
        X, e, w, _ = instance(b)
        inst.append((X, e, w, [float(g) for g in gen.batched_instance(b).gammas[::3]]))
    probs = [make(cc, X, e, w) for X, e, w, _ in inst]
    with cc.Batch(probs, [g for *_, g in inst], autotune=False, **opts) as bt:
        labs, infos, _ = bt.run()
    finals = [pr.get_state()[0].cpu().numpy() for pr in probs]
    for pr in probs:
        pr.close()
    for b, (X, e, w, g) in enumerate(inst[:3]):
        _, oinf, oU = mm.Problem(X, None, e, w).solve_path(g, mm.Opts(proj="jacobi:1", **opts))
        with make(cc, X, e, w) as pr:
            _, _, Up = pr.solve_path(g, labels=False, U_path=True, **opts)
        Up = Up.cpu().numpy()
        assert sum(i.converged for i in oinf) >= len(g) - 1
        for k, oi in enumerate(oinf):
            if oi.converged:
                assert infos[b][k]["converged"] == 1, (ids[b], k)
                assert abs(infos[b][k]["iters"] - oi.iters) <= mm.DEFAULT_TEST_EVERY, (ids[b], k)
                assert np.array_equal(labs[b][k].cpu().numpy(), oi.labels), (ids[b], k)
                assert rel_max(Up[k], oU[k]) < 1e-5, (ids[b], k)
        assert rel_max(finals[b], oU[-1]) < 1e-5, ids[b]
