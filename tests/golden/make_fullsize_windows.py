"""Writes the expected values of the full-size trajectory parity tests
(tests/test_gpu_fullsize.py) from the FP64 oracle alone.

Run from the repository root:
    python tests/golden/make_fullsize_windows.py expression
    python tests/golden/make_fullsize_windows.py genotype

Each window starts from the oracle's initial state (U_0 = X-tilde, s = 1,
A' = U_0; Section "The Proximal Distance Algorithm", readings r7) and runs
a fixed number of MM iterations with one Jacobi sweep of the block-descent
projection per iteration (proj "jacobi:1", the GPU's scheme), at the
default rho and eps = (eta rho)^2, eta = 1e-2.  Inputs are the workloads'
seeded FP32 values and the oracle's own kNN weights (Methods, "Calibration
of Weights").  Stored per window: the final shrink factors s of every edge
(fusion: s = 0, the V update's group soft-threshold), the fused-edge count
after every iteration, the labels (components of the fused edges), d and
F of the last iteration, and U and A on a seeded sample of rows (those of
edges whose fused state changed, then random ones) and, for the wide
genotype rows, of columns.

Only gen/ and oracle/ are used; nothing comes from the GPU path.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
from oracle import graph, mm, prep, weights  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# (gamma, MM iterations): gammas of the workloads' paths; the expression
# windows span the onset of fusion from the initial state
WINDOWS = {
    "expression": [(None, -3, 420), (None, -2, 360), (None, -1, 300)],
    "genotype": [(None, -1, 32)],
}


def inputs(name):
    wl = gen.make(name)
    X = np.asarray(wl.X, dtype=np.float32).astype(np.float64)
    if wl.standardize:
        X = np.asarray(prep.standardize_columns(X, wl.mask), dtype=np.float32).astype(np.float64)
    E, w, phi = weights.knn_weights(X, wl.mask, wl.k, wl.phi)
    return wl, X, E, w, phi


def run(name):
    wl, X, E, w, phi = inputs(name)
    prob = mm.Problem(X, wl.mask, E, w)
    n, p = X.shape
    out = {"edges": E.astype(np.int32), "w": w, "phi": np.float64(phi)}
    rng = np.random.default_rng(4242)
    cols = np.arange(p) if p <= 1024 else np.sort(rng.choice(p, 256, replace=False))
    out["cols"] = cols.astype(np.int32)
    for k, (_, gi, iters) in enumerate(WINDOWS[name]):
        gamma = float(wl.gammas[gi])
        rho, eps = prob.constants(gamma, mm.Opts())
        st = prob.initial_state()
        fused0 = st.s == 0.0
        ever = np.zeros(len(E), dtype=bool)
        counts = []
        t0 = time.time()
        for m in range(iters):
            st, dg = prob.iterate(gamma, rho, eps, st, "jacobi:1")
            f = st.s == 0.0
            ever |= f != fused0
            counts.append(int(f.sum()))
            if m % 50 == 0:
                print(f"[golden] {name} gamma={gamma:.4g} iteration {m}/{iters} fused={counts[-1]} "
                      f"({time.time() - t0:.0f} s)", flush=True)
        lab, ncl = graph.components(n, E, st.s == 0.0)
        touched = np.unique(E[ever].ravel())
        rows = list(touched[:32])
        rest = np.setdiff1d(np.arange(n), rows)
        rows += list(rng.choice(rest, 48 - len(rows), replace=False))
        rows = np.sort(np.asarray(rows, dtype=np.int64))
        out[f"w{k}_gamma"] = np.float64(gamma)
        out[f"w{k}_iters"] = np.int64(iters)
        out[f"w{k}_rho"] = np.float64(rho)
        out[f"w{k}_eps"] = np.float64(eps)
        out[f"w{k}_s"] = st.s
        out[f"w{k}_fused_counts"] = np.asarray(counts, dtype=np.int64)
        out[f"w{k}_labels"] = lab.astype(np.int32)
        out[f"w{k}_n_clusters"] = np.int64(ncl)
        out[f"w{k}_d"] = np.float64(dg["d"])
        out[f"w{k}_F"] = np.float64(dg["F"])
        out[f"w{k}_rows"] = rows.astype(np.int32)
        out[f"w{k}_U"] = st.U[np.ix_(rows, cols)]
        out[f"w{k}_A"] = st.A[np.ix_(rows, cols)]
        print(f"[golden] {name} gamma={gamma:.4g}: {iters} iterations, fused {counts[-1]} of {len(E)}, "
              f"first fused at iteration {next((i for i, c in enumerate(counts) if c), None)}, "
              f"{int(ever.sum())} edges changed state, {ncl} clusters", flush=True)
    path = os.path.join(HERE, f"{name}_windows.npz")
    np.savez_compressed(path, **out)
    print(f"[golden] wrote {path} ({os.path.getsize(path) / 1e6:.2f} MB)")


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["expression"]:
        run(nm)
