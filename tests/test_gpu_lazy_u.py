"""U stored lazily.  With one projection sweep the point sweep keeps U only
at missing entries (a side array) and the solve rebuilds U from the last
sweep's A' and theta when it ends.  The MM update of U (Missing Data) is a
function of X, A' and, at missing entries, the previous U, so the result
is the same bits as storing U every iteration (CCMI_LAZY_U=0).  The tests
force the lazy path (CCMI_LAZY_U=2) also where the solver would not take
it by default (missing data with one item per wave)."""
import numpy as np
import pytest
import torch

from tests._gpu import plain_problem, reduced_expression, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cc():
    import paper_1409_2065_amd as P
    P.load()
    assert torch.cuda.is_available()
    return P


def _gpu(cc, X, mask, edges, w, precision):
    dtype = torch.float64 if precision == "f64" else torch.float32
    Xt, m, e, wt = to_dev(X, mask, edges, w, dtype)
    return cc.Problem(Xt, m, e, wt, precision=precision)


def _run(cc, prob, precision, steps, monkeypatch, lazy):
    monkeypatch.setenv("CCMI_LAZY_U", lazy)
    X, M, E, w = prob
    out = []
    with _gpu(cc, X, M, E, w, precision) as g:
        for gamma, kw in steps:
            info = g.solve(gamma, **kw)
            out.append(np.array([info["iters"], info["converged"], info["objective"], info["d"]]))
            out.extend(t.cpu().numpy() for t in g.get_state())
            out.append(g.U(torch.float64).cpu().numpy())
    return out


def _same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


# a cold start, then warm starts that begin from the rebuilt U
STEPS = [(3.0, dict(tol=0.0, max_iter=1)), (3.0, dict(tol=0.0, max_iter=2)),
         (5.0, dict(tol=0.0, max_iter=37)), (8.0, dict(tol=1e-5, max_iter=3000))]


@pytest.mark.parametrize("precision", ["f32", "mixed", "f64"])
@pytest.mark.parametrize("masked", [True, False])
def test_lazy_u_is_bitwise_the_stored_u(cc, precision, masked, monkeypatch):
    X, M, E, w, _ = reduced_expression(n=300, p=300)
    prob = (X, M if masked else None, E, w)
    _same(_run(cc, prob, precision, STEPS, monkeypatch, "0"),
          _run(cc, prob, precision, STEPS, monkeypatch, "2"))


@pytest.mark.parametrize("vec", ["1", "2"])
def test_lazy_u_narrow_tiles(cc, vec, monkeypatch):
    """1 and 2 features per lane: the missing-entry ranks follow the tile."""
    monkeypatch.setenv("CCMI_VEC", vec)
    X, M, E, w, _ = reduced_expression(n=200, p=150)
    prob = (X, M, E, w)
    _same(_run(cc, prob, "mixed", STEPS[:3], monkeypatch, "0"),
          _run(cc, prob, "mixed", STEPS[:3], monkeypatch, "2"))


@pytest.mark.parametrize("waves", ["4", "8"])
def test_lazy_u_several_items_per_wave(cc, monkeypatch, waves):
    """3000 points x 3 tiles in blocks of 4 and 8 waves: waves take several
    items and prefetch (the default takes the lazy path here)."""
    monkeypatch.setenv("CCMI_POINT_WAVES", waves)
    X, M, E, w, _ = reduced_expression(n=3000, p=700)
    prob = (X, M, E, w)
    steps = [(5.0, dict(tol=0.0, max_iter=12)), (6.0, dict(tol=0.0, max_iter=5))]
    _same(_run(cc, prob, "mixed", steps, monkeypatch, "0"),
          _run(cc, prob, "mixed", steps, monkeypatch, "1"))


def test_lazy_u_after_a_batch_changed_the_tiles(cc, monkeypatch):
    """A batched solve picks its own tile width for the problem; the next
    single solve rebuilds the missing-entry index for that width."""
    X, M, E, w, _ = reduced_expression(n=150, p=100)
    res = []
    for lazy in ("0", "2"):
        monkeypatch.setenv("CCMI_LAZY_U", lazy)
        monkeypatch.setenv("CCMI_VEC", "4")
        out = []
        with _gpu(cc, X, M, E, w, "mixed") as g:
            g.solve(3.0, tol=0.0, max_iter=20)
            out.append(g.U(torch.float64).cpu().numpy())
            with cc.Batch([g], [[4.0, 6.0]], autotune=False, max_iter=200, tol=0.0) as bt:
                assert bt.config()["vec"] != 4
                bt.run()
            out.append(g.U(torch.float64).cpu().numpy())
            g.solve(7.0, tol=0.0, max_iter=20)
            out.extend(t.cpu().numpy() for t in g.get_state())
        res.append(out)
    _same(*res)


def test_lazy_u_no_mask_plain(cc, monkeypatch):
    X, M, E, w = plain_problem()
    prob = (X, M, E, w)
    _same(_run(cc, prob, "mixed", STEPS, monkeypatch, "0"),
          _run(cc, prob, "mixed", STEPS, monkeypatch, "1"))


@pytest.mark.parametrize("precision", ["f32", "mixed", "f64"])
def test_state_storage_rounding(cc, precision):
    """The state a problem stores: U in the state type; A in FP32 (f32), as
    an FP32 high half plus an FP32 low half (mixed: 48 significant bits, the
    high half being the nearest FP32 value), or in FP64.  Reading the state
    back and setting it again reproduces it bit for bit."""
    X, M, E, w, _ = reduced_expression(n=120, p=70)
    rng = np.random.default_rng(7)
    U0 = rng.standard_normal((120, 70)) * np.exp(rng.uniform(-20, 20, (120, 70)))
    A0 = rng.standard_normal((120, 70)) * np.exp(rng.uniform(-20, 20, (120, 70)))
    s0 = rng.uniform(0.0, 1.0, len(E))
    with _gpu(cc, X, M, E, w, precision) as g:
        g.set_state(torch.tensor(U0, device="cuda"), torch.tensor(A0, device="cuda"),
                    torch.tensor(s0, device="cuda"))
        U1, A1, s1 = (t.cpu().numpy() for t in g.get_state())
        g.set_state(torch.tensor(U1, device="cuda"), torch.tensor(A1, device="cuda"),
                    torch.tensor(s1, device="cuda"))
        U2, A2, s2 = (t.cpu().numpy() for t in g.get_state())
    assert np.array_equal(s1, s0)
    assert np.array_equal(U2, U1) and np.array_equal(A2, A1) and np.array_equal(s2, s1)
    if precision == "f32":
        assert np.array_equal(U1, U0.astype(np.float32).astype(np.float64))
        assert np.array_equal(A1, A0.astype(np.float32).astype(np.float64))
    elif precision == "f64":
        assert np.array_equal(U1, U0) and np.array_equal(A1, A0)
    else:
        assert np.array_equal(U1, U0)
        hi = A0.astype(np.float32).astype(np.float64)
        lo = (A0 - hi).astype(np.float32).astype(np.float64)
        assert np.array_equal(A1, hi + lo)
        assert np.array_equal(A1.astype(np.float32).astype(np.float64), hi)
        assert np.max(np.abs(A1 - A0) / np.abs(A0)) <= 2.0 ** -47
