"""GPU parity of the weight builder, column standardisation and the
component labelling against the oracle (integer outputs bit-exact; weights
to FP64 rounding)."""
import numpy as np
import pytest
import torch

import gen
from oracle import graph, prep, weights
from tests._gpu import as_f32_values

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cc():
    import paper_1409_2065_amd as P
    P.load()
    return P


def _check(cc, X, mask, k, phi, normalize=False):
    E_ref, w_ref, phi_ref = weights.knn_weights(X, mask, k, phi, normalize)
    Xt = torch.tensor(np.nan_to_num(X), dtype=torch.float32, device="cuda")
    m = None if mask is None else torch.tensor(mask.astype(np.uint8), device="cuda")
    e, w, phi_used = cc.build_knn_weights(Xt, m, k=k, phi=phi, normalize=normalize)
    e = e.cpu().numpy()
    w = w.cpu().numpy()
    assert np.array_equal(e, E_ref)
    assert phi_used == pytest.approx(phi_ref, rel=1e-13)
    assert np.allclose(w, w_ref, rtol=1e-12, atol=0)


def test_knn_plain(cc):
    wl = gen.plain()
    _check(cc, as_f32_values(wl.X), None, wl.k, wl.phi)


def test_knn_expression_missing_median_rule(cc):
    wl = gen.expression(n=300, p=64, n_clusters=6)
    _check(cc, as_f32_values(wl.X), wl.mask, wl.k, wl.phi)
    _check(cc, as_f32_values(wl.X), wl.mask, 4, 0.0)
    _check(cc, as_f32_values(wl.X), wl.mask, 7, -0.5, normalize=True)


def test_knn_genotype_standardised(cc):
    wl = gen.genotype(n=240, p=512)
    Z = as_f32_values(prep.standardize_columns(wl.X))
    _check(cc, Z, None, wl.k, wl.phi)


@pytest.mark.parametrize("n", [2, 3, 65, 129])
def test_knn_small_and_ragged(cc, n):
    rng = np.random.default_rng(n)
    X = as_f32_values(rng.normal(size=(n, 3)))
    _check(cc, X, None, 1, 0.3)
    if n > 3:
        _check(cc, X, None, 3, 0.3)


@pytest.mark.parametrize("n", [300, 1500])
def test_knn_near_duplicates_exact(cc, n):
    """A third of the rows are copies of one row plus noise far below the
    FP32 rounding of their distances, so the FP32 Gram product cannot rank
    them.  The FP64 re-rank of the first candidates cannot be certified for
    those rows; the wider pass (every row for n = 300, 512 candidates for
    n = 1500) can, and the edge set equals the oracle's exact one."""
    rng = np.random.default_rng(7)
    p = 256
    X = rng.normal(size=(n, p)) * 3.0 + 10.0
    dup = n // 3
    X[:dup] = X[0] + rng.normal(size=(dup, p)) * 1e-4
    _check(cc, as_f32_values(X), None, 6, 0.0)


def test_knn_uncertifiable_rows_are_an_error(cc):
    """n above what the widest pass ranks exhaustively (12289 rows), with
    every row within FP32 rounding of every other: no row's neighbours can
    be certified exact, and the builder returns CC_ERR_NUMERIC instead of
    an edge set."""
    rng = np.random.default_rng(3)
    n, p = 16384, 8
    X = 1.0 + rng.normal(size=(n, p)) * 1e-4
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    with pytest.raises(cc.CCError) as ei:
        cc.build_knn_weights(Xt, None, k=6, phi=0.0)
    assert ei.value.status == 4  # CC_ERR_NUMERIC
    assert "certified" in str(ei.value)


def test_knn_ties_lower_index(cc):
    X = np.arange(9, dtype=np.float64)[:, None]  # equal spacing: every row has a tie
    _check(cc, X, None, 1, 0.0)
    _check(cc, X, None, 2, 0.0)


def test_standardize(cc):
    wl = gen.expression(n=200, p=40, n_clusters=4)
    X = as_f32_values(wl.X)
    ref = prep.standardize_columns(X, wl.mask)
    Xt = torch.tensor(np.nan_to_num(X), dtype=torch.float32, device="cuda")
    m = torch.tensor(wl.mask.astype(np.uint8), device="cuda")
    cc.standardize_columns(Xt, m)
    got = Xt.cpu().numpy().astype(np.float64)
    obs = wl.mask
    assert np.allclose(got[obs], ref[obs].astype(np.float32), rtol=2e-7, atol=2e-7)
    G = gen.genotype(n=100, p=300).X
    G[:, 7] = 1.0  # constant column
    refg = prep.standardize_columns(G)
    Gt = torch.tensor(G, dtype=torch.float64, device="cuda")
    cc.standardize_columns(Gt)
    assert np.allclose(Gt.cpu().numpy(), refg, rtol=1e-13, atol=1e-13)
    assert (Gt[:, 7] == 0).all()


@pytest.mark.parametrize("m", [0, 10, 50, 300])
def test_components(cc, m):
    rng = np.random.default_rng(m)
    n = 200
    pairs = set()
    while len(pairs) < m:
        i, j = sorted(rng.choice(n, 2, replace=False).tolist())
        pairs.add((i, j))
    E = np.array(sorted(pairs), dtype=np.int64).reshape(-1, 2)
    keep = rng.random(len(E)) < 0.8
    ref, k = graph.components(n, E, keep)
    lab, cnt = cc.components(n, torch.tensor(E.astype(np.int32), device="cuda"),
                             torch.tensor(keep.astype(np.uint8), device="cuda"))
    assert np.array_equal(lab.cpu().numpy(), ref)
    assert cnt == k
