"""GPU parity of the MM solver (libccmi through the C ABI) against the FP64
oracle, on the same seeded inputs.

Tolerances (stated per test): FP64 state tracks the oracle's Jacobi-1
trajectory to rounding; the mixed precision (FP64 point state, FP32 pair
sweep) stays within max|dU|/max|U| <= 1e-5 of the oracle's fixed point with
identical fusion partitions; the all-FP32 state stalls up to ~1e-4 away.
"""
import numpy as np
import pytest
import torch

from oracle import mm
from tests._gpu import (as_f32_values, oracle_jacobi, plain_problem, reduced_expression,
                        rel_max, to_dev)

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


# ------------------------------------------------------- trajectory parity
@pytest.mark.parametrize("iters", [1, 2, 3, 7, 60])
def test_fixed_iterations_f64_match_oracle_trajectory(cc, iters):
    X, M, E, w = plain_problem()
    prob = oracle_jacobi(X, M, E, w)
    st, info = prob.solve(10.0, mm.Opts(tol=0, max_iter=iters, proj="jacobi:1", record=True))
    with _gpu(cc, X, M, E, w, "f64") as g:
        gi = g.solve(10.0, tol=0.0, max_iter=iters, record_objective=1)
        U, A, s = (t.cpu().numpy() for t in g.get_state())
        F = g.trace()
    assert gi["iters"] == iters and gi["converged"] == 0
    assert rel_max(U, st.U) < 1e-11
    assert rel_max(A, st.A) < 1e-11
    assert np.abs(s - st.s).max() < 1e-9
    assert np.array_equal(s == 0, st.s == 0)
    assert np.allclose(F, info.trace_F, rtol=1e-10, atol=0)
    assert gi["d"] == pytest.approx(info.d, rel=1e-10)
    assert gi["objective"] == pytest.approx(info.objective, rel=1e-10)


@pytest.mark.parametrize("precision,tol", [("mixed", 2e-6), ("f32", 2e-5)])
def test_fixed_iterations_reduced_precision(cc, precision, tol):
    X, M, E, w, gam = reduced_expression()
    prob = oracle_jacobi(X, M, E, w)
    st, _ = prob.solve(3.0, mm.Opts(tol=0, max_iter=200, proj="jacobi:1"))
    with _gpu(cc, X, M, E, w, precision) as g:
        g.solve(3.0, tol=0.0, max_iter=200)
        U, A, s = (t.cpu().numpy() for t in g.get_state())
    assert rel_max(U, st.U) < tol
    assert rel_max(A, st.A) < tol


# ------------------------------------------------------ converged parity
def test_plain_config_f64_gamma_1(cc):
    """Plain workload (n=200, p=10, k=10, phi=0.5, gamma=1), FP64."""
    X, M, E, w = plain_problem()
    st, info = oracle_jacobi(X, M, E, w).solve(1.0, mm.Opts(proj="jacobi:1"))
    with _gpu(cc, X, M, E, w, "f64") as g:
        gi = g.solve(1.0)
        U = g.U(torch.float64).cpu().numpy()
        lab, ncl = g.labels()
    assert gi["converged"] == 1 and info.converged
    assert abs(gi["iters"] - info.iters) <= mm.DEFAULT_TEST_EVERY
    assert rel_max(U, st.U) < 1e-8
    assert np.array_equal(lab.cpu().numpy(), info.labels)
    assert ncl == info.n_clusters == gi["n_clusters"]


# gamma = 1000 fuses every edge of each kNN component (full coalescence)
@pytest.mark.parametrize("gamma", [1.0, 10.0, 100.0, 1000.0])
def test_plain_config_mixed_converged(cc, gamma):
    X, M, E, w = plain_problem()
    X = as_f32_values(X)
    st, info = oracle_jacobi(X, M, E, w).solve(gamma, mm.Opts(proj="jacobi:1"))
    with _gpu(cc, X, M, E, w, "mixed") as g:
        gi = g.solve(gamma)
        U = g.U(torch.float64).cpu().numpy()
        lab, ncl = g.labels()
        fused = g.fused_edges().cpu().numpy().astype(bool)
    assert gi["converged"] == 1
    assert rel_max(U, st.U) <= 1e-5
    assert np.array_equal(lab.cpu().numpy(), info.labels)
    assert ncl == info.n_clusters
    assert np.array_equal(fused, info.fused)


def test_reduced_expression_path_mixed(cc):
    """Expression-like recipe at n=100, p=150 (two feature tiles, the second
    ragged) with 5% missing entries: a
    warm-started path; every gamma matches within 1e-5 with equal labels."""
    X, M, E, w, gam = reduced_expression(n=100, p=150)
    gam = [0.3, 3.0, 30.0, 100.0]
    # missing entries at small gamma converge slowly (the loss is flat in
    # them); both sides stop at the same cap when the test has not passed
    cap = 4000
    _, infos, Us = oracle_jacobi(X, M, E, w).solve_path(gam, mm.Opts(proj="jacobi:1", max_iter=cap))
    with _gpu(cc, X, M, E, w, "mixed") as g:
        ginfos, lab, Up = g.solve_path(gam, labels=True, U_path=True, max_iter=cap)
    lab = lab.cpu().numpy()
    Up = Up.cpu().numpy()
    for k in range(len(gam)):
        assert ginfos[k]["converged"] == int(infos[k].converged)
        assert abs(ginfos[k]["iters"] - infos[k].iters) <= mm.DEFAULT_TEST_EVERY
        assert rel_max(Up[k], Us[k]) <= 1e-5, (gam[k], rel_max(Up[k], Us[k]))
        assert np.array_equal(lab[k], infos[k].labels), gam[k]
    assert len(set(i.n_clusters for i in infos)) > 1  # the path spans fusion


def test_f32_precision_plain(cc):
    X, M, E, w = plain_problem()
    X = as_f32_values(X)
    st, info = oracle_jacobi(X, M, E, w).solve(10.0, mm.Opts(proj="jacobi:1"))
    with _gpu(cc, X, M, E, w, "f32") as g:
        g.solve(10.0, max_iter=60000)
        U = g.U(torch.float64).cpu().numpy()
        lab, _ = g.labels()
    assert rel_max(U, st.U) <= 2e-4
    assert np.array_equal(lab.cpu().numpy(), info.labels)


# ------------------------------------------------------------ edge cases
def test_gamma_zero_and_isolated_points(cc):
    X, M, E, w, _ = reduced_expression(n=80, p=20)
    with _gpu(cc, X, M, E, w, "mixed") as g:
        g.solve(0.0, tol=0.0, max_iter=30)
        U = g.U(torch.float64).cpu().numpy()
    obs = M
    assert np.array_equal(U[obs], X[obs])
    # no edges at all: U = X for any gamma
    with _gpu(cc, X, M, np.zeros((0, 2), int), np.zeros(0), "mixed") as g:
        info = g.solve(5.0, tol=0.0, max_iter=10)
        U = g.U(torch.float64).cpu().numpy()
        lab, ncl = g.labels()
    assert np.array_equal(U[obs], X[obs])
    assert ncl == X.shape[0] and info["n_clusters"] == X.shape[0]


@pytest.mark.parametrize("n,p", [(1, 1), (1, 5), (2, 1), (3, 300), (9, 1)])
def test_tiny_shapes(cc, n, p):
    rng = np.random.default_rng(n * 100 + p)
    X = as_f32_values(rng.normal(size=(n, p)))
    E = np.array([(i, j) for i in range(n) for j in range(i + 1, n)], dtype=np.int64).reshape(-1, 2)
    w = np.ones(len(E))
    st, info = oracle_jacobi(X, None, E, w).solve(0.7, mm.Opts(proj="jacobi:1", tol=0, max_iter=40))
    with _gpu(cc, X, None, E, w, "f64") as g:
        g.solve(0.7, tol=0.0, max_iter=40)
        U = g.U(torch.float64).cpu().numpy()
        lab, ncl = g.labels()
    assert rel_max(U, st.U) < 1e-11
    assert np.array_equal(lab.cpu().numpy(), info.labels)


def test_all_observed_mask_equals_no_mask(cc):
    X, _, E, w = plain_problem()
    X = as_f32_values(X)
    with _gpu(cc, X, None, E, w, "mixed") as g:
        g.solve(10.0, tol=0.0, max_iter=100)
        a = g.U(torch.float64).cpu().numpy()
    with _gpu(cc, X, np.ones(X.shape, bool), E, w, "mixed") as g:
        g.solve(10.0, tol=0.0, max_iter=100)
        b = g.U(torch.float64).cpu().numpy()
    assert np.array_equal(a, b)


def test_deterministic_repeat(cc):
    X, M, E, w, _ = reduced_expression()
    outs = []
    for _ in range(2):
        with _gpu(cc, X, M, E, w, "mixed") as g:
            g.solve(5.0, tol=0.0, max_iter=300)
            outs.append(g.U(torch.float64).cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_state_export_import_resumes_path_bitwise(cc):
    X, M, E, w, _ = reduced_expression()
    gam = [0.5, 2.0, 8.0, 30.0]
    kw = dict(tol=1e-6, max_iter=5000)
    with _gpu(cc, X, M, E, w, "mixed") as g:
        _, lab_all, U_all = g.solve_path(gam, U_path=True, **kw)
    with _gpu(cc, X, M, E, w, "mixed") as g:
        g.solve_path(gam[:2], **kw)
        blob = g.export_state()
    with _gpu(cc, X, M, E, w, "mixed") as g2:
        g2.import_state(blob)
        _, lab2, U2 = g2.solve_path(gam[2:], U_path=True, **kw)
    assert torch.equal(U2, U_all[2:])
    assert torch.equal(lab2, lab_all[2:])


def test_invalid_inputs_rejected(cc):
    X, M, E, w = plain_problem()
    _, _, e, wt = to_dev(X, None, E, w, torch.float32)
    Xb = torch.tensor(X, dtype=torch.float32, device="cuda")
    Xb[3, 2] = float("nan")          # an observed non-finite entry
    with pytest.raises(cc.CCError) as ei:
        cc.Problem(Xb, None, e, wt)
    assert ei.value.status == 1
    mb = torch.ones(Xb.shape, dtype=torch.uint8, device="cuda")
    mb[3, 2] = 0                     # the same entry marked missing is fine
    with cc.Problem(Xb, mb, e, wt) as g:
        g.solve(1.0, max_iter=5)
        assert torch.isfinite(g.U()).all()
        # a path with an infinite or negative gamma is refused before any
        # gamma is solved: the state stays as it was
        U0 = [t.cpu().numpy() for t in g.get_state()]
        for bad in ([2.0, float("inf")], [2.0, -1.0], [2.0, float("nan")]):
            with pytest.raises(cc.CCError) as ei:
                g.solve_path(bad, max_iter=5)
            assert ei.value.status == 1
            assert all(np.array_equal(a, b) for a, b in zip(U0, (t.cpu().numpy() for t in g.get_state())))
    with pytest.raises(cc.CCError):
        _gpu(cc, X, None, E[:, ::-1].copy(), w, "mixed")   # i > j
    with pytest.raises(cc.CCError):
        _gpu(cc, X, None, np.vstack([E, E[:1]]), np.r_[w, w[:1]], "mixed")  # duplicate
    with pytest.raises(cc.CCError):
        _gpu(cc, X, None, E, -w, "mixed")


# ------------------------------------------------------- kernel variants
# The point sweep has a wave-per-(point, tile) form (CCMI_SLAB_F=0, tile
# width 64*CCMI_VEC) and an LDS-slab form (CCMI_SLAB_F = feature-tile width);
# wide rows (> 1024 features) switch the edge sweep to per-tile partials.
# Each variant must reproduce the oracle's FP64 trajectory.
@pytest.mark.parametrize("slab,vec", [("0", "1"), ("0", "2"), ("0", "4"),
                                      ("4", "0"), ("8", "0"), ("16", "0"), ("32", "0")])
def test_point_kernel_variants(cc, slab, vec, monkeypatch):
    monkeypatch.setenv("CCMI_SLAB_F", slab)
    monkeypatch.setenv("CCMI_VEC", vec)
    X, M, E, w, _ = reduced_expression(n=300, p=150)  # ragged last tile for every width
    st, _ = oracle_jacobi(X, M, E, w).solve(3.0, mm.Opts(tol=0, max_iter=80, proj="jacobi:1"))
    with _gpu(cc, X, M, E, w, "f64") as g:
        g.solve(3.0, tol=0.0, max_iter=80)
        U, A, s = (t.cpu().numpy() for t in g.get_state())
    assert rel_max(U, st.U) < 1e-11
    assert rel_max(A, st.A) < 1e-11
    assert np.abs(s - st.s).max() < 1e-9


@pytest.mark.parametrize("precision,tol", [("f64", 1e-11), ("mixed", 2e-6)])
def test_wide_rows_edge_tiles(cc, precision, tol):
    X, M, E, w, _ = reduced_expression(n=60, p=1100)  # 1100 > 1024: tiled edge sweep
    st, _ = oracle_jacobi(X, M, E, w).solve(20.0, mm.Opts(tol=0, max_iter=60, proj="jacobi:1"))
    with _gpu(cc, X, M, E, w, precision) as g:
        g.solve(20.0, tol=0.0, max_iter=60)
        U, A, s = (t.cpu().numpy() for t in g.get_state())
    assert rel_max(U, st.U) < tol
    assert rel_max(A, st.A) < tol


@pytest.mark.parametrize("p,precision,items", [
    (40, "f64", "1"), (100, "f64", "1"), (200, "f64", "1"), (200, "f64", "0"),
    (450, "mixed", "1"), (450, "mixed", "0"), (700, "mixed", "1")])
def test_edge_sweep_variants(cc, p, precision, items, monkeypatch):
    """Edge sweep by work items of edges sharing a lower end (1, 2, 4 and 8
    features per lane), its edge-parallel fallback (CCMI_EDGE_ITEMS=0) and
    the edge-parallel kernel for rows up to 1024 wide follow the oracle's
    trajectory."""
    monkeypatch.setenv("CCMI_EDGE_ITEMS", items)
    X, M, E, w, _ = reduced_expression(n=150, p=p)
    st, _ = oracle_jacobi(X, M, E, w).solve(3.0, mm.Opts(tol=0, max_iter=60, proj="jacobi:1"))
    with _gpu(cc, X, M, E, w, precision) as g:
        g.solve(3.0, tol=0.0, max_iter=60)
        U, A, s = (t.cpu().numpy() for t in g.get_state())
    tol = 1e-11 if precision == "f64" else 2e-6
    assert rel_max(U, st.U) < tol
    assert rel_max(A, st.A) < tol


def test_point_sweep_prefetch(cc):
    """More point-tile items than one per wave (3000 points x 3 tiles): the
    point sweep prefetches each wave's next item; trajectory parity."""
    X, M, E, w, _ = reduced_expression(n=3000, p=700)
    st, _ = oracle_jacobi(X, M, E, w).solve(5.0, mm.Opts(tol=0, max_iter=12, proj="jacobi:1"))
    with _gpu(cc, X, M, E, w, "f64") as g:
        g.solve(5.0, tol=0.0, max_iter=12)
        U, A, s = (t.cpu().numpy() for t in g.get_state())
    assert rel_max(U, st.U) < 1e-11
    assert rel_max(A, st.A) < 1e-11


@pytest.mark.parametrize("edge_slab,slab_items", [("0", "1"), ("1", "0"), ("1", "1")])
def test_wide_rows_edge_variants(cc, edge_slab, slab_items, monkeypatch):
    """Wide rows: the per-tile edge partials (CCMI_EDGE_SLAB=0) and the LDS
    slab edge sweep, by single edges (CCMI_EDGE_SLAB_ITEMS=0) or by work
    items of edges sharing a lower end, agree with the oracle's trajectory."""
    monkeypatch.setenv("CCMI_EDGE_SLAB", edge_slab)
    monkeypatch.setenv("CCMI_EDGE_SLAB_ITEMS", slab_items)
    X, M, E, w, _ = reduced_expression(n=60, p=1100)
    st, _ = oracle_jacobi(X, M, E, w).solve(20.0, mm.Opts(tol=0, max_iter=40, proj="jacobi:1"))
    with _gpu(cc, X, M, E, w, "f64") as g:
        g.solve(20.0, tol=0.0, max_iter=40)
        U, A, s = (t.cpu().numpy() for t in g.get_state())
    assert rel_max(U, st.U) < 1e-11
    assert np.abs(s - st.s).max() < 1e-9


@pytest.mark.parametrize("precision", ["f32", "mixed"])
def test_slab_edge_items_are_bitwise_the_edge_order(cc, precision, monkeypatch):
    """The slab edge sweep by work items adds each edge's features in the
    same order as the sweep by single edges: identical iterates."""
    X, M, E, w, _ = reduced_expression(n=60, p=1100)
    out = []
    for items in ("0", "1"):
        monkeypatch.setenv("CCMI_EDGE_SLAB_ITEMS", items)
        with _gpu(cc, X, M, E, w, precision) as g:
            g.solve(20.0, tol=0.0, max_iter=30)
            out.append([t.cpu().numpy() for t in g.get_state()])
    for a, b in zip(*out):
        assert np.array_equal(a, b)


# ------------------------------------------------------- sampled kernel timing
def test_kernel_stats_sample_every_kth_iteration(cc):
    """cc_profile samples every k-th MM iteration with events stamped by the
    kernels' own start and end; sampling leaves the iterates unchanged."""
    X, M, E, w = plain_problem()
    with _gpu(cc, X, M, E, w, "mixed") as g, _gpu(cc, X, M, E, w, "mixed") as h:
        g.profile(4)
        g.solve(10.0, tol=0.0, max_iter=64)
        ks = g.kernel_stats()
        g.profile(0)
        h.solve(10.0, tol=0.0, max_iter=64)
        Ug = g.U(torch.float64).cpu().numpy()
        Uh = h.U(torch.float64).cpu().numpy()
    assert np.array_equal(Ug, Uh)
    for name in ("point_sweep", "edge_stage"):
        assert ks[name]["launches"] >= 64 // 4 - 1
        assert 0.0 < ks[name]["avg_ms"] < 5.0


# ------------------------------------------- small eta: FP64 point state
@pytest.mark.parametrize("gamma", [1.0, 5.0])
def test_small_eta_mixed_converged(cc, gamma):
    """eta = 1e-3 puts the MM fixed point ten times closer to the minimiser
    of f_mu than the default, at about ten times the iterations (~8e4 here),
    where the MM contraction per iteration is ~1 - eta/14.  An FP32 point
    state would stall up to ulp / (1 - rate) away; the mixed precision
    (FP64 point state, FP32 neighbour gathers) still reaches the oracle's
    fixed point within 1e-5 with the same fused edges and labels."""
    import gen
    from oracle import weights
    wl = gen.plain(n=40, p=5)
    X = as_f32_values(wl.X)
    E, w, _ = weights.knn_weights(X, None, 6, 0.5)
    st, info = oracle_jacobi(X, None, E, w).solve(
        gamma, mm.Opts(proj="jacobi:1", eta=1e-3, max_iter=400000))
    with _gpu(cc, X, None, E, w, "mixed") as g:
        gi = g.solve(gamma, eta=1e-3, max_iter=400000)
        U = g.U(torch.float64).cpu().numpy()
        lab, ncl = g.labels()
        fused = g.fused_edges().cpu().numpy().astype(bool)
    assert info.converged and gi["converged"] == 1
    assert gi["iters"] > 40000
    assert rel_max(U, st.U) <= 1e-5
    assert np.array_equal(fused, info.fused)
    assert np.array_equal(lab.cpu().numpy(), info.labels)
    assert ncl == info.n_clusters


# ------------------------------------- several projection sweeps per iteration
# proj_sweeps = K runs K Jacobi sweeps of the paper's block update per MM
# iteration (the block-descent projection repeated towards stability), the
# first from the previous projection; the oracle's "jacobi:K" does the same.
@pytest.mark.parametrize("K,iters", [(2, 7), (2, 60), (4, 60), (3, 61)])
def test_proj_sweeps_f64_match_oracle_trajectory(cc, K, iters):
    X, M, E, w = plain_problem()
    st, info = oracle_jacobi(X, M, E, w).solve(
        10.0, mm.Opts(tol=0, max_iter=iters, proj=f"jacobi:{K}", record=True, test_every=4))
    with _gpu(cc, X, M, E, w, "f64") as g:
        gi = g.solve(10.0, tol=0.0, max_iter=iters, record_objective=1, proj_sweeps=K, test_every=4)
        U, A, s = (t.cpu().numpy() for t in g.get_state())
        F = g.trace()
    assert gi["iters"] == iters
    assert rel_max(U, st.U) < 1e-11
    assert rel_max(A, st.A) < 1e-11
    assert np.abs(s - st.s).max() < 1e-9
    assert np.array_equal(s == 0, st.s == 0)
    assert np.allclose(F, info.trace_F, rtol=1e-10, atol=0)
    assert gi["d"] == pytest.approx(info.d, rel=1e-10)


@pytest.mark.parametrize("vec", ["1", "2", "4"])
def test_proj_sweeps_tiles_and_missing_data(cc, vec, monkeypatch):
    """Two and five sweeps on a masked problem whose rows span several
    feature tiles (the last ragged) at every tile width; the window of the
    stopping test (K = 1) makes the last sweep compare with the previous
    projection itself."""
    monkeypatch.setenv("CCMI_VEC", vec)
    X, M, E, w, _ = reduced_expression(n=300, p=150)
    for K, win in ((2, 1), (5, 64)):
        st, info = oracle_jacobi(X, M, E, w).solve(
            3.0, mm.Opts(tol=0, max_iter=70, proj=f"jacobi:{K}", test_every=win))
        with _gpu(cc, X, M, E, w, "f64") as g:
            gi = g.solve(3.0, tol=0.0, max_iter=70, proj_sweeps=K, test_every=win)
            U, A, s = (t.cpu().numpy() for t in g.get_state())
        assert rel_max(U, st.U) < 1e-11, K
        assert rel_max(A, st.A) < 1e-11, K
        assert gi["rel_change"] == pytest.approx(info.rel_change, rel=1e-8), K


def test_proj_sweeps_prefetch_and_mixed(cc):
    """Several items per wave (3000 points x 3 tiles) with three sweeps:
    FP64 to rounding, the mixed precision within its fixed-iteration bar."""
    X, M, E, w, _ = reduced_expression(n=3000, p=700)
    st, _ = oracle_jacobi(X, M, E, w).solve(5.0, mm.Opts(tol=0, max_iter=12, proj="jacobi:3"))
    for precision, tol in (("f64", 1e-11), ("mixed", 2e-6)):
        with _gpu(cc, X, M, E, w, precision) as g:
            g.solve(5.0, tol=0.0, max_iter=12, proj_sweeps=3)
            U, A, s = (t.cpu().numpy() for t in g.get_state())
        assert rel_max(U, st.U) < tol, precision
        assert rel_max(A, st.A) < tol, precision


@pytest.mark.parametrize("K", [2, 4])
def test_proj_sweeps_mixed_converged(cc, K):
    """The converged mixed-precision solve with K sweeps reaches the
    oracle's fixed point (that of the exact projection) within 1e-5, with
    the same fused edges and labels."""
    X, M, E, w = plain_problem()
    X = as_f32_values(X)
    st, info = oracle_jacobi(X, M, E, w).solve(10.0, mm.Opts(proj=f"jacobi:{K}"))
    with _gpu(cc, X, M, E, w, "mixed") as g:
        gi = g.solve(10.0, proj_sweeps=K)
        U = g.U(torch.float64).cpu().numpy()
        lab, ncl = g.labels()
        fused = g.fused_edges().cpu().numpy().astype(bool)
    assert gi["converged"] == 1 and info.converged
    assert rel_max(U, st.U) <= 1e-5
    assert np.array_equal(fused, info.fused)
    assert np.array_equal(lab.cpu().numpy(), info.labels)


def test_proj_sweeps_rejected_where_unsupported(cc):
    X, M, E, w = plain_problem()
    with _gpu(cc, X, M, E, w, "mixed") as g:
        for bad in (0, 65):
            with pytest.raises(cc.CCError) as ei:
                g.solve(1.0, proj_sweeps=bad)
            assert ei.value.status == 1
        with pytest.raises(cc.CCError):
            cc.Batch([g], [[1.0]], autotune=False, proj_sweeps=2)


def test_f32_prefetch_path(cc):
    """FP32 state with several items per wave (the point sweep's prefetching
    form), where A is itself the array the next sweep gathers: trajectory
    within the FP32 bar."""
    X, M, E, w, _ = reduced_expression(n=3000, p=700)
    st, _ = oracle_jacobi(X, M, E, w).solve(5.0, mm.Opts(tol=0, max_iter=12, proj="jacobi:1"))
    with _gpu(cc, X, M, E, w, "f32") as g:
        g.solve(5.0, tol=0.0, max_iter=12)
        U, A, s = (t.cpu().numpy() for t in g.get_state())
    assert rel_max(U, st.U) < 2e-5
    assert rel_max(A, st.A) < 2e-5


# ------------------------------------------------------------ numeric errors
def test_non_finite_state_reports_numeric_error(cc):
    """A state with a non-finite entry makes d non-finite: the solve returns
    CC_ERR_NUMERIC (an ordinary status, no device fault), the next
    warm-started solve starts again from the initial state, and after
    cc_reset_state the problem solves as a fresh one does, bitwise."""
    X, M, E, w = plain_problem()
    X = as_f32_values(X)
    with _gpu(cc, X, M, E, w, "mixed") as ref:
        ref.solve(10.0, tol=0.0, max_iter=50)
        Uref = ref.U(torch.float64).cpu().numpy()
    with _gpu(cc, X, M, E, w, "mixed") as g:
        U, A, s = (t.cpu().numpy() for t in g.get_state())
        U[5, 3] = np.nan
        g.set_state(U, A, s)
        with pytest.raises(cc.CCError) as ei:
            g.solve(10.0, max_iter=100)
        assert ei.value.status == 4  # CC_ERR_NUMERIC
        g.solve(10.0, tol=0.0, max_iter=50)  # warm start falls back to the initial state
        assert np.array_equal(g.U(torch.float64).cpu().numpy(), Uref)
        U[5, 3] = np.inf
        g.set_state(U, A, s)
        with pytest.raises(cc.CCError) as ei:
            g.solve(10.0, max_iter=100)
        assert ei.value.status == 4
        g.reset_state()
        g.solve(10.0, tol=0.0, max_iter=50)
        assert np.array_equal(g.U(torch.float64).cpu().numpy(), Uref)


@pytest.mark.parametrize("waves", ["4", "8", "16"])
def test_point_sweep_prefetch_mixed_wide_blocks(cc, waves, monkeypatch):
    """The mixed precision with several items per wave (3000 points x 3
    tiles) in point-sweep blocks of 4, 8 and 16 waves: trajectory within the
    mixed bar with the same fused edges."""
    monkeypatch.setenv("CCMI_POINT_WAVES", waves)
    X, M, E, w, _ = reduced_expression(n=3000, p=700)
    st, _ = oracle_jacobi(X, M, E, w).solve(5.0, mm.Opts(tol=0, max_iter=12, proj="jacobi:1"))
    with _gpu(cc, X, M, E, w, "mixed") as g:
        g.solve(5.0, tol=0.0, max_iter=12)
        U, A, s = (t.cpu().numpy() for t in g.get_state())
    assert rel_max(U, st.U) < 2e-6
    assert rel_max(A, st.A) < 2e-6
    assert np.array_equal(s == 0, st.s == 0)
