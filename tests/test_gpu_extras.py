"""GPU parity of the extras (cc_pca, cc_solve_path_pc, cc_min_connected_k,
cc_composite_weights, through the C ABI) against the FP64 oracle on the same
seeded inputs.

Tolerances: principal components match the oracle's SVD to 1e-7 (vectors,
after the shared sign convention) and 1e-9 relative (singular values) at
the iteration counts used, where the spectral gaps make subspace iteration
converge far below that; projections of the GPU's own path equal the
host projection of the same U to rounding and the oracle's path within the
solver's 1e-5 bar; the smallest connected k and the component counts are
integers and must be equal; weights match to 1e-12 relative."""
import numpy as np
import pytest
import torch

import gen
from oracle import extras, mm, weights
from tests._gpu import as_f32_values, oracle_jacobi, reduced_expression, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cc():
    import paper_1409_2065_amd as P
    P.load()
    assert torch.cuda.is_available()
    return P


def _x_dev(X, mask, dtype=torch.float32):
    Xt = torch.tensor(np.nan_to_num(X, nan=0.0), dtype=dtype, device="cuda")
    m = None if mask is None else torch.tensor(mask.astype(np.uint8), device="cuda")
    return Xt, m


# ------------------------------------------------------------------ PCA
@pytest.mark.parametrize("n,p,r,with_mask", [(300, 64, 2, True), (300, 64, 5, False), (120, 5, 2, False),
                                              (90, 700, 3, True)])
def test_pca_matches_oracle(cc, n, p, r, with_mask):
    wl = gen.expression(seed=1002, n=n, p=p, n_clusters=6, n_gamma=2, missing=0.05 if with_mask else 0.0)
    X = as_f32_values(wl.X)
    M = wl.mask if with_mask else None
    V0, S0, c0 = extras.pca(X, M, r)
    Xt, m = _x_dev(X, M)
    V, S, c = cc.pca(Xt, m, r=r, iters=200)
    V = V.cpu().numpy()
    assert np.allclose(S, S0, rtol=1e-9, atol=0), (S, S0)
    assert np.abs(V - V0).max() < 1e-7
    assert np.abs(c.cpu().numpy() - c0).max() < 1e-12 * max(1.0, np.abs(c0).max())


def test_pca_f64_input_and_full_subspace(cc):
    # p = 6 < r + 8: the subspace is the whole space and one step is exact
    wl = gen.plain(n=80, p=6)
    V0, S0, _ = extras.pca(wl.X, None, 4)
    Xt = torch.tensor(wl.X, dtype=torch.float64, device="cuda")
    V, S, _ = cc.pca(Xt, None, r=4, iters=1)
    assert np.allclose(S, S0, rtol=1e-12)
    assert np.abs(V.cpu().numpy() - V0).max() < 1e-10


# ------------------------------------------------------ projected path
def test_solve_path_pc_projects_each_gamma(cc):
    X, M, E, w, _ = reduced_expression(n=100, p=150)
    gam = [0.3, 3.0, 30.0]
    cap = 4000
    V0, _, c0 = extras.pca(X, M, 2)
    _, infos, Us = oracle_jacobi(X, M, E, w).solve_path(gam, mm.Opts(proj="jacobi:1", max_iter=cap))
    Xt, m, e, wt = to_dev(X, M, E, w, torch.float32)
    Vd = torch.tensor(V0, device="cuda")
    cd = torch.tensor(c0, device="cuda")
    with cc.Problem(Xt, m, e, wt, precision="mixed") as g:
        gi, lab, proj = g.solve_path_pc(gam, Vd, cd, labels=True, max_iter=cap)
        U_last = g.U(torch.float64).cpu().numpy()
    with cc.Problem(Xt, m, e, wt, precision="mixed") as h:
        _, lab2, Up = h.solve_path(gam, labels=True, U_path=True, max_iter=cap)
    proj = proj.cpu().numpy()
    Up = Up.cpu().numpy().astype(np.float64)
    # the projection kernel reads the same U the plain path copies out
    assert np.abs(proj[-1] - extras.project(U_last, V0, c0)).max() < 1e-10 * max(1.0, np.abs(proj).max())
    assert np.array_equal(lab.cpu().numpy(), lab2.cpu().numpy())
    scale = np.abs(X[~np.isnan(X)]).max()
    for k in range(len(gam)):
        # Up is FP32: its rounding bounds the difference to the FP64 U
        assert np.abs(proj[k] - extras.project(Up[k], V0, c0)).max() < 1e-6 * scale * np.sqrt(X.shape[1])
        ref = extras.project(Us[k], V0, c0)
        assert np.abs(proj[k] - ref).max() <= 1e-5 * np.abs(Us[k]).max() * np.sqrt(X.shape[1])
        assert np.array_equal(lab.cpu().numpy()[k], infos[k].labels)
        assert gi[k]["converged"] == int(infos[k].converged)


# --------------------------------------------------- smallest connected k
def _two_clusters(a, b, seed=3):
    rng = np.random.default_rng(seed)
    return np.vstack([rng.normal(size=(a, 3)) * 0.1, rng.normal(size=(b, 3)) * 0.1 + 100.0])


@pytest.mark.parametrize("case", ["two_clusters", "expression", "disconnected", "plain_f64"])
def test_min_connected_k_matches_oracle(cc, case):
    if case == "two_clusters":
        X, M, kmax = as_f32_values(_two_clusters(6, 11)), None, 10
    elif case == "expression":
        wl = gen.expression(seed=1002, n=150, p=30, n_clusters=6, n_gamma=2)
        X, M, kmax = as_f32_values(wl.X), wl.mask, 24
    elif case == "disconnected":
        X, M, kmax = as_f32_values(_two_clusters(8, 9)), None, 5
    else:
        wl = gen.plain(n=120, p=10)
        X, M, kmax = wl.X, None, 30
    k0, c0 = extras.min_connected_k(X, M, kmax)
    dtype = torch.float64 if case == "plain_f64" else torch.float32
    Xt, m = _x_dev(X, M, dtype)
    k, c = cc.min_connected_k(Xt, m, k_max=kmax)
    assert (k, c) == (k0, c0)
    if case == "disconnected":
        assert k == -1 and c == 2


# ------------------------------------------------- composite distance
@pytest.mark.parametrize("alpha,phi,mode,normalize", [(1.0, 0.3, "euclid", False), (0.3, -0.5, "periodic", False),
                                                     (0.0, -0.5, "geodesic", True), (0.6, 0.02, "geodesic", False)])
def test_composite_weights_match_oracle(cc, alpha, phi, mode, normalize):
    rng = np.random.default_rng(21)
    n = 200
    X = rng.normal(size=(n, 40)).astype(np.float32).astype(np.float64)
    edges, _, _ = weights.knn_weights(X, None, 6, 0.5)
    period, geo = None, False
    if mode == "geodesic":
        Y = np.stack([rng.uniform(-80, 80, n), rng.uniform(-180, 180, n)], axis=1)
        geo = True
    else:
        Y = rng.uniform(0, 360, size=(n, 2))
        if mode == "periodic":
            period = [360.0, 0.0]
    w0, phi0 = extras.composite_weights(X, Y, edges, alpha, phi, period, geo, 6371.0 if geo else 1.0, normalize)
    w, phi_used = cc.composite_weights(torch.tensor(edges, dtype=torch.int32), torch.tensor(X, dtype=torch.float32),
                                       torch.tensor(Y), alpha, phi, period=period, geodesic=geo,
                                       radius=6371.0 if geo else 1.0, normalize=normalize)
    assert phi_used == pytest.approx(phi0, rel=1e-12)
    assert np.allclose(w.cpu().numpy(), w0, rtol=1e-12, atol=0)


def test_composite_weights_with_missing_entries_match_oracle(cc):
    wl = gen.expression(seed=1002, n=150, p=30, n_clusters=6, n_gamma=2)
    X = as_f32_values(wl.X)
    M = wl.mask
    edges, _, _ = weights.knn_weights(X, M, 8, -0.5)
    rng = np.random.default_rng(5)
    Y = np.stack([rng.uniform(-60, 60, X.shape[0]), rng.uniform(-180, 180, X.shape[0])], axis=1)
    w0, phi0 = extras.composite_weights(X, Y, edges, 0.5, -0.5, geodesic=True, radius=6371.0, mask=M)
    Xt, m = _x_dev(X, M)
    w, phi_used = cc.composite_weights(torch.tensor(edges, dtype=torch.int32), Xt, torch.tensor(Y), 0.5, -0.5,
                                       geodesic=True, radius=6371.0, mask=m)
    assert phi_used == pytest.approx(phi0, rel=1e-12)
    assert np.allclose(w.cpu().numpy(), w0, rtol=1e-12, atol=0)


def test_extras_reject_bad_arguments(cc):
    X = torch.zeros((10, 3), device="cuda")
    with pytest.raises(cc.CCError):
        cc.pca(X, r=17)
    with pytest.raises(cc.CCError):
        cc.min_connected_k(X, k_max=10)
    with pytest.raises(cc.CCError):
        cc.composite_weights(torch.tensor([[0, 10]], dtype=torch.int32), X, torch.zeros((10, 2)), 0.5, 0.1)
    with pytest.raises(cc.CCError):
        cc.composite_weights(torch.tensor([[0, 1]], dtype=torch.int32), X, torch.zeros((10, 3)), 0.5, 0.1,
                             geodesic=True)
