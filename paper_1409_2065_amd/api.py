"""Python face of libccmi on torch device tensors.

Every function marshals arguments (device pointers, sizes, the current HIP
stream) into one C-ABI call of libccmi; PyTorch only supplies device memory
and streams.  Inputs must be contiguous tensors on the current HIP device.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import CCError, check, default_opts

PRECISIONS = {"f32": _lib.CC_PREC_F32, "mixed": _lib.CC_PREC_MIXED, "f64": _lib.CC_PREC_F64}


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t, dtype=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t))
    if dtype is not None and t.dtype != dtype:
        t = t.to(dtype)
    if not t.is_cuda:
        t = t.cuda()
    return t.contiguous()


def _xdtype(X: torch.Tensor) -> int:
    if X.dtype == torch.float32:
        return _lib.CC_DTYPE_F32
    if X.dtype == torch.float64:
        return _lib.CC_DTYPE_F64
    raise TypeError("X must be float32 or float64")


def _mask(mask, shape):
    if mask is None:
        return None
    m = _dev(mask)
    if m.dtype != torch.uint8:
        m = m.to(torch.uint8)
    if tuple(m.shape) != tuple(shape):
        raise ValueError("mask shape must equal X shape")
    return m.contiguous()


class Problem:
    """A clustering problem resident on the GPU (cc_problem_create)."""

    def __init__(self, X, mask=None, edges=None, w=None, precision: str = "mixed"):
        X = _dev(X)
        if X.dtype not in (torch.float32, torch.float64):
            X = X.to(torch.float32)
        n, p = X.shape
        m = _mask(mask, X.shape)
        if edges is None:
            edges = torch.zeros((0, 2), dtype=torch.int32)
        e = _dev(edges, torch.int32).reshape(-1, 2)
        ei = e[:, 0].contiguous()
        ej = e[:, 1].contiguous()
        wt = _dev(w if w is not None else torch.zeros(0), torch.float64).reshape(-1)
        self._keep = (X, m, ei, ej, wt)
        self.n, self.p, self.E = int(n), int(p), int(e.shape[0])
        self.precision = precision
        lib = _lib.load()
        h = C.c_void_p()
        check(lib.cc_problem_create(n, p, _xdtype(X), _ptr(X), p, _ptr(m), p, self.E,
                                    _ptr(ei), _ptr(ej), _ptr(wt), PRECISIONS[precision],
                                    C.c_void_p(_stream()), C.byref(h)))
        self._h = h
        self._keep = None

    # -- lifetime --
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().cc_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- solving --
    def solve(self, gamma: float, **opts) -> dict:
        o = default_opts(**opts)
        info = _lib.SolveInfo()
        check(_lib.load().cc_solve(self._h, float(gamma), C.byref(o), C.byref(info)))
        return info.as_dict()

    def solve_path(self, gammas: Sequence[float], labels: bool = True, U_path: bool = False, **opts):
        g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64))
        G = g.size
        o = default_opts(**opts)
        infos = (_lib.SolveInfo * max(G, 1))()
        lab = torch.empty((G, self.n), dtype=torch.int32, device="cuda") if labels else None
        up = torch.empty((G, self.n, self.p), dtype=torch.float32, device="cuda") if U_path else None
        check(_lib.load().cc_solve_path(self._h, G, g.ctypes.data_as(_lib.P_f64), C.byref(o),
                                        _ptr(lab), _ptr(up), infos))
        return [infos[k].as_dict() for k in range(G)], lab, up

    def solve_path_pc(self, gammas: Sequence[float], V, center=None, labels: bool = True, **opts):
        """cc_solve_path_pc: the path with each gamma's U projected on the
        device onto the columns of V (p, r): returns (infos, labels,
        proj (G, n, r) float64)."""
        g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64))
        G = g.size
        V = _dev(V, torch.float64)
        if V.dim() != 2 or V.shape[0] != self.p:
            raise ValueError("V must be (p, r)")
        r = V.shape[1]
        c = None if center is None else _dev(center, torch.float64)
        if c is not None and c.numel() != self.p:
            raise ValueError("center must have p entries")
        o = default_opts(**opts)
        infos = (_lib.SolveInfo * max(G, 1))()
        lab = torch.empty((G, self.n), dtype=torch.int32, device="cuda") if labels else None
        proj = torch.empty((G, self.n, r), dtype=torch.float64, device="cuda")
        check(_lib.load().cc_solve_path_pc(self._h, G, g.ctypes.data_as(_lib.P_f64), C.byref(o),
                                           _ptr(lab), r, _ptr(V), _ptr(c), _ptr(proj), infos))
        return [infos[k].as_dict() for k in range(G)], lab, proj

    # -- results --
    def U(self, dtype=torch.float32) -> torch.Tensor:
        out = torch.empty((self.n, self.p), dtype=dtype, device="cuda")
        dt = _lib.CC_DTYPE_F32 if dtype == torch.float32 else _lib.CC_DTYPE_F64
        check(_lib.load().cc_get_U(self._h, dt, _ptr(out), self.p))
        torch.cuda.current_stream().synchronize()
        return out

    def labels(self):
        out = torch.empty(self.n, dtype=torch.int32, device="cuda")
        k = C.c_int32()
        check(_lib.load().cc_get_labels(self._h, _ptr(out), C.byref(k)))
        return out, int(k.value)

    def fused_edges(self) -> torch.Tensor:
        out = torch.empty(max(self.E, 1), dtype=torch.uint8, device="cuda")
        check(_lib.load().cc_get_fused_edges(self._h, _ptr(out)))
        torch.cuda.current_stream().synchronize()
        return out[: self.E]

    def trace(self, cap: int = 1 << 22) -> np.ndarray:
        buf = np.empty(cap, dtype=np.float64)
        cnt = C.c_int64()
        check(_lib.load().cc_get_trace(self._h, buf.ctypes.data_as(_lib.P_f64), cap, C.byref(cnt)))
        return buf[: cnt.value].copy()

    # -- kernel timing --
    def profile(self, sample_every: int) -> None:
        check(_lib.load().cc_profile(self._h, int(sample_every)))

    def kernel_stats(self):
        ms = (C.c_double * 2)()
        cnt = (C.c_int64 * 2)()
        check(_lib.load().cc_kernel_stats(self._h, ms, cnt))
        names = ("point_sweep", "edge_stage")
        return {nm: {"avg_ms": ms[q], "launches": cnt[q]} for q, nm in enumerate(names)}

    # -- state --
    def export_state(self) -> bytes:
        sz = C.c_size_t()
        check(_lib.load().cc_state_size(self._h, C.byref(sz)))
        buf = C.create_string_buffer(sz.value)
        check(_lib.load().cc_export_state(self._h, buf, sz.value))
        return buf.raw

    def import_state(self, data: bytes) -> None:
        buf = C.create_string_buffer(data, len(data))
        check(_lib.load().cc_import_state(self._h, buf, len(data)))

    def reset_state(self) -> None:
        check(_lib.load().cc_reset_state(self._h))

    def set_state(self, U, A, s) -> None:
        U = _dev(U, torch.float64)
        A = _dev(A, torch.float64)
        s = _dev(s, torch.float64).reshape(-1)
        check(_lib.load().cc_set_state(self._h, _ptr(U), _ptr(A), self.p, _ptr(s)))

    def get_state(self):
        U = torch.empty((self.n, self.p), dtype=torch.float64, device="cuda")
        A = torch.empty((self.n, self.p), dtype=torch.float64, device="cuda")
        s = torch.empty(max(self.E, 1), dtype=torch.float64, device="cuda")
        check(_lib.load().cc_get_state(self._h, _ptr(U), _ptr(A), self.p, _ptr(s)))
        torch.cuda.current_stream().synchronize()
        return U, A, s[: self.E]


def build_knn_weights(X, mask=None, k: int = 10, phi: float = 0.5, normalize: bool = False):
    """cc_build_knn_weights: returns (edges (E, 2) int32, w (E,) float64,
    phi_used), on the device."""
    X = _dev(X)
    n, p = X.shape
    m = _mask(mask, X.shape)
    cap = n * k
    ei = torch.empty(cap, dtype=torch.int32, device="cuda")
    ej = torch.empty(cap, dtype=torch.int32, device="cuda")
    w = torch.empty(cap, dtype=torch.float64, device="cuda")
    ne = C.c_int64()
    phi_used = C.c_double()
    check(_lib.load().cc_build_knn_weights(n, p, _xdtype(X), _ptr(X), p, _ptr(m), p, int(k), float(phi),
                                           1 if normalize else 0, _ptr(ei), _ptr(ej), _ptr(w), cap,
                                           C.byref(ne), C.byref(phi_used), C.c_void_p(_stream())))
    E = ne.value
    return torch.stack([ei[:E], ej[:E]], dim=1).contiguous(), w[:E].contiguous(), phi_used.value


def standardize_columns(X: torch.Tensor, mask=None) -> torch.Tensor:
    """cc_standardize_columns, in place on X; returns X."""
    if not (X.is_cuda and X.is_contiguous()):
        raise ValueError("X must be a contiguous device tensor")
    m = _mask(mask, X.shape)
    n, p = X.shape
    check(_lib.load().cc_standardize_columns(n, p, _xdtype(X), _ptr(X), p, _ptr(m), p,
                                             C.c_void_p(_stream())))
    return X


def pca(X, mask=None, r: int = 2, iters: int = 100):
    """cc_pca: (V (p, r) float64 on the device, singular values (r,) numpy,
    column means (p,) float64 on the device) of the mean-imputed, centred X."""
    X = _dev(X)
    n, p = X.shape
    m = _mask(mask, X.shape)
    V = torch.empty((p, int(r)), dtype=torch.float64, device="cuda")
    center = torch.empty(p, dtype=torch.float64, device="cuda")
    sval = np.zeros(int(r), dtype=np.float64)
    check(_lib.load().cc_pca(n, p, _xdtype(X), _ptr(X), p, _ptr(m), p, int(r), int(iters), _ptr(V),
                             sval.ctypes.data_as(_lib.P_f64), _ptr(center), C.c_void_p(_stream())))
    return V, sval, center


def min_connected_k(X, mask=None, k_max: int = 32):
    """cc_min_connected_k: (smallest k <= k_max with a connected kNN graph,
    or -1; number of components at k_max)."""
    X = _dev(X)
    n, p = X.shape
    m = _mask(mask, X.shape)
    kmin, ncomp = C.c_int32(), C.c_int32()
    check(_lib.load().cc_min_connected_k(n, p, _xdtype(X), _ptr(X), p, _ptr(m), p, int(k_max),
                                         C.byref(kmin), C.byref(ncomp), C.c_void_p(_stream())))
    return int(kmin.value), int(ncomp.value)


def composite_weights(edges, X, Y, alpha: float, phi: float = -0.5, period=None,
                      geodesic: bool = False, radius: float = 1.0, normalize: bool = False, mask=None):
    """cc_composite_weights: (w (E,) float64 on the device, phi_used) from
    d = alpha ||x_i - x_j|| + (1 - alpha) dist(y_i, y_j) over the edges
    (missing entries of X, per mask, take their observed column means)."""
    e = _dev(edges, torch.int32).reshape(-1, 2)
    ei = e[:, 0].contiguous()
    ej = e[:, 1].contiguous()
    X = _dev(X)
    Y = _dev(Y, torch.float64)
    if Y.dim() == 1:
        Y = Y.reshape(-1, 1)
    n, p = X.shape
    m = _mask(mask, X.shape)
    q = Y.shape[1]
    if Y.shape[0] != n:
        raise ValueError("X and Y need the same number of rows")
    per = None
    if period is not None:
        per = np.ascontiguousarray(np.asarray(period, dtype=np.float64).reshape(q))
    w = torch.empty(e.shape[0], dtype=torch.float64, device="cuda")
    phi_used = C.c_double()
    check(_lib.load().cc_composite_weights(
        n, e.shape[0], _ptr(ei), _ptr(ej), p, _xdtype(X), _ptr(X), p, _ptr(m), p, q, _ptr(Y), q,
        None if per is None else per.ctypes.data_as(_lib.P_f64), 1 if geodesic else 0, float(radius),
        float(alpha), float(phi), 1 if normalize else 0, _ptr(w), C.byref(phi_used),
        C.c_void_p(_stream())))
    return w, phi_used.value


def components(n: int, edges, keep=None):
    """cc_components: labels (n,) int32 (min index per component) and count."""
    e = _dev(edges, torch.int32).reshape(-1, 2)
    ei = e[:, 0].contiguous()
    ej = e[:, 1].contiguous()
    kp = None if keep is None else _dev(keep, torch.uint8)
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    cnt = C.c_int32()
    check(_lib.load().cc_components(n, e.shape[0], _ptr(ei), _ptr(ej), _ptr(kp), _ptr(lab), C.byref(cnt),
                                    C.c_void_p(_stream())))
    return lab, int(cnt.value)


__all__ = ["Problem", "build_knn_weights", "standardize_columns", "components", "CCError", "PRECISIONS"]


class Batch:
    """Many problems, each along its own gamma path, solved in the same
    launches (cc_batch_create / cc_batch_run).  The problems must outlive the
    batch; while it runs, their solver states belong to it."""

    def __init__(self, problems: Sequence[Problem], gammas: Sequence[Sequence[float]],
                 autotune: bool = True, **opts):
        if len(problems) != len(gammas):
            raise ValueError("one gamma path per problem")
        self.problems = list(problems)
        self.n_gamma = [len(g) for g in gammas]
        flat = np.ascontiguousarray(np.concatenate([np.asarray(g, dtype=np.float64) for g in gammas]))
        ng = np.asarray(self.n_gamma, dtype=np.int32)
        handles = (C.c_void_p * len(problems))(*[pr._h.value for pr in problems])
        o = default_opts(**opts)
        h = C.c_void_p()
        torch.cuda.current_stream().synchronize()
        check(_lib.load().cc_batch_create(len(problems), handles, ng.ctypes.data_as(_lib.P_i32),
                                          flat.ctypes.data_as(_lib.P_f64), C.byref(o),
                                          1 if autotune else 0, C.byref(h)))
        self._h = h

    def config(self) -> dict:
        vec, ipw, gi = C.c_int32(), C.c_int32(), C.c_int32()
        tune = (C.c_double * 9)()
        check(_lib.load().cc_batch_config(self._h, C.byref(vec), C.byref(ipw), C.byref(gi), tune))
        return {"vec": vec.value, "items_per_wave": ipw.value, "graph_iters": gi.value, "tune_us": list(tune)}

    def tuning(self):
        """The autotuner's classes (width class, size class, instances, vec,
        items per wave, us per batched iteration) and each instance's class."""
        nc = C.c_int32()
        check(_lib.load().cc_batch_tuning(self._h, 0, C.byref(nc), None, None, None))
        k = nc.value
        cls = (C.c_int32 * max(5 * k, 1))()
        us = (C.c_double * max(k, 1))()
        inst = (C.c_int32 * max(len(self.problems), 1))()
        check(_lib.load().cc_batch_tuning(self._h, k, C.byref(nc), cls, us, inst))
        names = ("width_class", "size_class", "instances", "vec", "items_per_wave")
        out = [{**{nm: cls[5 * c + q] for q, nm in enumerate(names)}, "us_per_iteration": us[c]} for c in range(k)]
        return out, [inst[b] for b in range(len(self.problems))]

    def run(self, labels: bool = True):
        """Returns (labels, infos, latency_ms): labels[b] is an (n_gamma[b], n_b)
        int32 tensor (or None), infos[b] a list of per-gamma dicts,
        latency_ms[b] the time from the start of the run to the end of b's path."""
        sizes = [pr.n * g for pr, g in zip(self.problems, self.n_gamma)]
        lab = torch.empty(max(sum(sizes), 1), dtype=torch.int32, device="cuda") if labels else None
        total = sum(self.n_gamma)
        infos = (_lib.SolveInfo * max(total, 1))()
        lat = np.zeros(len(self.problems), dtype=np.float64)
        torch.cuda.current_stream().synchronize()
        check(_lib.load().cc_batch_run(self._h, _ptr(lab), infos, lat.ctypes.data_as(_lib.P_f64)))
        out_lab, out_inf = [], []
        off = g0 = 0
        for pr, g, sz in zip(self.problems, self.n_gamma, sizes):
            out_lab.append(lab[off:off + sz].view(g, pr.n) if labels else None)
            out_inf.append([infos[g0 + k].as_dict() for k in range(g)])
            off += sz
            g0 += g
        return out_lab, out_inf, lat

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().cc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Server:
    """Continuous-batching solver (cc_server_*): requests (host data, kNN
    parameters and a gamma path) are admitted first come, first served
    within an HBM budget and share the launches of the admitted others."""

    def __init__(self, precision: str = "mixed", hbm_budget: int = 8 << 30, max_active: int = 256,
                 round_iters: int = 32, **opts):
        o = default_opts(**opts)
        h = C.c_void_p()
        check(_lib.load().cc_server_create(PRECISIONS[precision], C.byref(o), int(hbm_budget), int(max_active),
                                           int(round_iters), C.c_void_p(_stream()), C.byref(h)))
        self._h = h
        self._shape = {}

    def submit(self, X, mask=None, k: int = 10, phi: float = -0.5, gammas=(1.0,)) -> int:
        Xh = np.ascontiguousarray(np.nan_to_num(np.asarray(X, dtype=np.float32)))
        n, p = Xh.shape
        mh = None if mask is None else np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64))
        t = C.c_int64()
        check(_lib.load().cc_server_submit(self._h, n, p, Xh.ctypes.data_as(C.c_void_p),
                                           None if mh is None else mh.ctypes.data_as(C.c_void_p),
                                           int(k), float(phi), g.size, g.ctypes.data_as(_lib.P_f64),
                                           C.byref(t)))
        self._shape[t.value] = (n, p, g.size)
        return t.value

    def step(self):
        a, w, d = C.c_int32(), C.c_int32(), C.c_int32()
        check(_lib.load().cc_server_step(self._h, C.byref(a), C.byref(w), C.byref(d)))
        return a.value, w.value, d.value

    def status(self, ticket: int) -> dict:
        st = C.c_int32()
        ts, ta, td = C.c_double(), C.c_double(), C.c_double()
        check(_lib.load().cc_server_status(self._h, ticket, C.byref(st), C.byref(ts), C.byref(ta), C.byref(td)))
        return {"state": st.value, "t_submit": ts.value, "t_admit": ta.value, "t_done": td.value}

    def result(self, ticket: int, U: bool = False):
        n, p, g = self._shape[ticket]
        lab = torch.empty((g, n), dtype=torch.int32, device="cuda")
        infos = (_lib.SolveInfo * g)()
        u = torch.empty((n, p), dtype=torch.float32, device="cuda") if U else None
        check(_lib.load().cc_server_result(self._h, ticket, _ptr(lab), infos, _ptr(u)))
        return lab, [infos[k].as_dict() for k in range(g)], u

    def release(self, ticket: int) -> None:
        check(_lib.load().cc_server_release(self._h, ticket))
        self._shape.pop(ticket, None)

    def memory(self):
        """(device bytes counted against the budget, the budget)."""
        used, budget = C.c_int64(), C.c_int64()
        check(_lib.load().cc_server_memory(self._h, C.byref(used), C.byref(budget)))
        return used.value, budget.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().cc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
