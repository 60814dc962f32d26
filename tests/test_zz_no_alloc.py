"""The allocation-free standardisation entry point against the allocating
one, through the C ABI: equal results on two calls in a row (the second
smaller), at the largest column count it takes, the size limit, and the
non-finite check."""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_1409_2065_amd import _lib
    L = _lib.load()
    assert torch.cuda.is_available()
    return L


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _case(seed, n, p, missing, dtype):
    rng = np.random.default_rng(seed)
    X = rng.normal(3.0, 2.0, size=(n, p)) * rng.lognormal(0.0, 1.0, size=p)
    X[:, 0] = 7.0  # a constant column becomes 0
    X = torch.tensor(X, dtype=dtype, device="cuda")
    M = None
    if missing > 0:
        M = torch.tensor((rng.random((n, p)) >= missing).astype(np.uint8), device="cuda")
    return X, M


def _both(lib, X, M):
    from paper_1409_2065_amd import _lib
    n, p = X.shape
    dt = _lib.CC_DTYPE_F32 if X.dtype == torch.float32 else _lib.CC_DTYPE_F64
    a, b = X.clone(), X.clone()
    sa = lib.cc_standardize_columns(n, p, dt, _ptr(a), p, _ptr(M), p, _stream())
    sb = lib.cc_standardize_columns_noalloc(n, p, dt, _ptr(b), p, _ptr(M), p, _stream())
    torch.cuda.synchronize()
    return sa, sb, a, b


def test_noalloc_equals_allocating_entry_point(lib):
    # two calls in a row, the second smaller (fewer rows and columns): the
    # shared array keeps the first call's statistics, which must not leak
    for seed, n, p, missing, dtype in [(1, 700, 3000, 0.1, torch.float32), (2, 60, 45, 0.0, torch.float64),
                                       (3, 33, 7, 0.3, torch.float32)]:
        X, M = _case(seed, n, p, missing, dtype)
        sa, sb, a, b = _both(lib, X, M)
        assert sa == 0 and sb == 0, (seed, lib.cc_last_error_message())
        assert torch.equal(a, b), seed
        col = b[:, 1][M[:, 1] > 0] if M is not None else b[:, 1]
        assert abs(float(col.double().mean())) < 1e-5 and abs(float(col.double().std(unbiased=False)) - 1) < 1e-5


def test_noalloc_at_and_beyond_its_column_limit(lib):
    from paper_1409_2065_amd import _lib
    X, _ = _case(4, 5, 65536, 0.0, torch.float32)
    sa, sb, a, b = _both(lib, X, None)
    assert sa == 0 and sb == 0
    assert torch.equal(a, b)
    Y = torch.ones((3, 65537), dtype=torch.float32, device="cuda")
    Y0 = Y.clone()
    st = lib.cc_standardize_columns_noalloc(3, 65537, _lib.CC_DTYPE_F32, _ptr(Y), 65537, None, 65537, _stream())
    torch.cuda.synchronize()
    assert st == _lib.CC_ERR_INVALID_ARG and b"p <= 65536" in lib.cc_last_error_message()
    assert torch.equal(Y, Y0)


def test_noalloc_rejects_non_finite_observed_entries(lib):
    from paper_1409_2065_amd import _lib
    X, M = _case(5, 40, 30, 0.2, torch.float32)
    X[3, 4] = float("inf")
    M[3, 4] = 1
    X0 = X.clone()
    st = lib.cc_standardize_columns_noalloc(40, 30, _lib.CC_DTYPE_F32, _ptr(X), 30, _ptr(M), 30, _stream())
    torch.cuda.synchronize()
    assert st == _lib.CC_ERR_INVALID_ARG and b"non-finite" in lib.cc_last_error_message()
    assert torch.equal(X, X0)
    # the next call starts from a cleared count
    M[3, 4] = 0
    sa, sb, a, b = _both(lib, X, M)
    assert sa == 0 and sb == 0 and torch.equal(a, b)
