"""paper_1409_2065_amd: proximal-distance convex clustering on MI355X.

The compute path is libccmi.so (hand-written HIP kernels for gfx950) behind
the C ABI in include/ccmi.h; this package is a thin ctypes binding over it
that takes torch device tensors.  Build with
``python -m paper_1409_2065_amd.build``.
"""
from ._lib import CCError, LIB_PATH, load  # noqa: F401
from .api import (PRECISIONS, Batch, Problem, Server, build_knn_weights, components,  # noqa: F401
                  composite_weights, min_connected_k, pca, standardize_columns)

__all__ = ["Problem", "Batch", "Server", "build_knn_weights", "standardize_columns", "components", "pca",
           "min_connected_k", "composite_weights", "CCError",
           "PRECISIONS", "load", "LIB_PATH"]
