#!/usr/bin/env python3
"""Benchmark of the proximal-distance MM convex-clustering path on one GPU.

Workload (the expression-like configuration): n = 2000 cases, p = 500
predictors, 20 latent clusters with log-normal feature scales, 5% of the
entries missing completely at random, kNN weights with k = 15 and
phi = 0.5 / median(d^2), and a path of 30 log-spaced gammas in [1e-3, 1e2]
solved with warm starts.  All inputs are seeded and synthetic.

One step = the whole hot path over the batch: reset to the initial state,
then for every gamma the MM iterations to convergence (projection sweep,
edge norms, smoothed distance, shrinkage, U update, objective and stop test)
followed by the fused-cluster labels.  The kNN weights are built once on the
GPU before timing (reported separately).

Metric: pair-feature updates/s = sum over MM iterations of |E| * p, divided
by the wall time of the timed steps (inputs resident in HBM).

Beside it, the line carries the batched and served comparisons the metric
names (solves/s and latency, against the plain per-solve path).  Both sides
stop each gamma at a looser tolerance than the headline (--batch-tol and
--serve-tol, default 1e-4: windowed relative change <= 1e-4 * eta) or at the
iteration cap, and the line states the share of solves that passed the test
and the stopping quantity reached:
  batched  256 instances (n ~ U{50..800}, p ~ U{20..200}, 2-10 clusters,
           kNN k=10, 16 gammas each) in shared launches, tile shape
           autotuned, each gamma capped at --batch-max-iter MM iterations;
           the plain path solves the first --plain-sample instances one by
           one with the same options (its FIFO latency for all 256 is
           estimated from them and marked so);
  served   the first --serve-requests requests of the Poisson stream
           (200/s; n log-uniform in [100, 5000], p in [10, 1000], 10%
           missing, 8-32 gammas) submitted at their arrival times to the
           continuous-batching server and, separately, solved first come
           first served by the plain path; each gamma capped at
           --serve-max-iter MM iterations.

  extras   principal components (r = 2), the smallest connected k (k_max =
           128), composite-distance weights, and the path returned as U
           against its projection on two principal components.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
METRIC = "pair-feature updates/s (n=2000,p=500); solves/s + p99 latency, batched vs plain"

WORKLOAD_TEXT = {
    "expression": "expression-like n=2000 p=500, 20 clusters, log-normal scales, 5% MCAR, kNN k=15, "
                  "30-gamma path 1e-3..1e2 (warm starts), eta=1e-2, tol=1e-6",
    "genotype": "genotype-like n=1000 p=20000, Balding-Nichols F_ST=0.05, 12 groups, standardised, "
                "kNN k=20, 40-gamma path 1e-3..1e2 (warm starts), eta=1e-2, tol=1e-6",
    "plain": "plain n=200 p=10, 4 Gaussian clusters, kNN k=10, phi=0.5, gamma=1, eta=1e-2, tol=1e-6",
}


def algorithmic_bytes(n, p, E, has_mask):
    """Bytes the method itself must move per MM iteration with FP32 state,
    each array element counted once (neighbour rows are re-reads of the same
    array).  Point sweep (U update and the projection sweep) per
    point-feature: X 4, the mask 1 (with missing data), U read 4 and write 4,
    A' read 4, A write 4; per edge the neighbour slot and q factor of both
    directions, 2 x (4 + 8) B.  Edge stage per point-feature: the rows of
    the new A and of A' (4 + 4); per edge its ends, weight, shrink factor,
    norms and q (about 60 B less the point sweep's 24).  Returns
    (point-sweep bytes, whole-iteration bytes, point-sweep bytes per
    point-feature)."""
    k1 = 20 + (1 if has_mask else 0)
    point = k1 * n * p + 24 * E
    iteration = (k1 + 8) * n * p + 60 * E
    return point, iteration, k1


def implementation_bytes(n, p, E, precision, has_mask, missing=0):
    """Bytes one point-sweep launch of this implementation moves.  The mixed
    precision keeps U in FP64 and A as hi + lo: hi is the FP32 gather copy
    (its own row read, the new one written) and lo an FP32 low half, so A
    costs 4 + 4 bytes per entry beyond the gather copy.  Without missing data
    U_m follows from X and A', so U is neither read nor written (it is
    rebuilt once at the end of a solve).  With missing data and one work
    item per wave (the expression workload) U is read and written in full;
    where waves take several items it is read and written only at the
    `missing` entries, in a side array.  Same per-edge bytes as the
    algorithmic count.  Returns (bytes per launch, bytes per point-feature
    outside the side array)."""
    sx = 8 if precision == "f64" else 4
    ss = 4 if precision == "f32" else 8     # U
    sa = 8 if precision == "f64" else 4     # the stored A array
    per_pf = sx + sa + sa                   # X, A' read, A written
    if precision == "mixed":
        per_pf += 4 + 4                     # own gather row read, new one written
    side = 0
    if has_mask:
        per_pf += 1                         # mask
        if missing:
            side = 2 * ss * missing
        else:
            per_pf += 2 * ss                # U read and written
    return n * p * per_pf + side + 24 * E, per_pf


TRAFFIC_PROFILES = {
    ("expression", "mixed"): os.path.join(ROOT, "profiles", "traffic_k_point_expression_n2000_p500_mixed.md"),
    ("genotype", "mixed"): os.path.join(ROOT, "profiles", "traffic_k_point_genotype_n1000_p20000_mixed.md"),
}
KERNEL_SOURCES = ("paper_1409_2065_amd/csrc/solver.hip", "paper_1409_2065_amd/csrc/ccmi_internal.h")


def kernel_source_hash():
    """SHA-256 over the sources the sweep kernels are compiled from; a stored
    counter reading is used only while this matches the one it was taken with."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stored_traffic(workload, precision):
    """HBM bytes per k_point launch from the committed counter summary (two
    rocprofv3 --pmc passes, FETCH_SIZE and WRITE_SIZE, each scaled by what the
    same counter reads for a device copy of known size), or None when there is
    none for this workload or the kernel sources changed since it was taken."""
    path = TRAFFIC_PROFILES.get((workload, precision))
    if path is None or not os.path.exists(path):
        return None
    try:
        text = open(path).read()
        m = re.search(r"```json\n(.*?)\n```", text, re.S)
        rec = json.loads(m.group(1)) if m else {}
        if rec.get("source_sha256") != kernel_source_hash():
            return None
        return rec["fetch_kib_per_launch"] * rec["fetch_factor"] * 1024 + \
            rec["write_kib_per_launch"] * rec["write_factor"] * 1024
    except (OSError, ValueError, KeyError, TypeError):
        return None


def pmc_summary(fetch_csv, write_csv, copy_mib, command):
    """Markdown summary of two rocprofv3 counter-collection CSVs (one pass
    with FETCH_SIZE, one with WRITE_SIZE): per-kernel mean KiB per dispatch,
    the copy calibration factors, and a JSON record for the k_point kernel."""
    import csv
    from collections import defaultdict

    def per_kernel(path, counter):
        vals = defaultdict(list)
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") == counter:
                    vals[row["Kernel_Name"]].append(float(row["Counter_Value"]))
        return vals

    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    known_kib = copy_mib * 1024.0
    copy_f = max(v for k, vs in fetch.items() if "copyBuffer" in k for v in vs)
    copy_w = max(v for k, vs in write.items() if "copyBuffer" in k for v in vs)
    ff, wf = known_kib / copy_f, known_kib / copy_w
    kp = [k for k in fetch if "k_point" in k]
    if len(kp) != 1:
        raise SystemExit(f"expected one k_point kernel in the counters, found {kp}")
    kp = kp[0]
    fk = sum(fetch[kp]) / len(fetch[kp])
    wk = sum(write[kp]) / len(write[kp])
    rec = {"kernel": kp, "source_sha256": kernel_source_hash(), "dispatches": len(fetch[kp]),
           "fetch_kib_per_launch": round(fk, 3), "write_kib_per_launch": round(wk, 3),
           "copy_mib": copy_mib, "copy_fetch_kib": copy_f, "copy_write_kib": copy_w,
           "fetch_factor": round(ff, 6), "write_factor": round(wf, 6)}
    out = [f"command (pass 1): `{command.format(counter='FETCH_SIZE')}`",
           f"command (pass 2): `{command.format(counter='WRITE_SIZE')}`", "",
           f"Calibration: a device copy of {copy_mib} MiB ({known_kib:.0f} KiB each way) read "
           f"FETCH_SIZE {copy_f:.0f} KiB and WRITE_SIZE {copy_w:.0f} KiB: factors {ff:.4f} and {wf:.4f}.", "",
           "| kernel | dispatches | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | scaled MB/dispatch |",
           "|---|---:|---:|---:|---:|"]
    for k in sorted(fetch, key=lambda k: -sum(fetch[k])):
        f_ = sum(fetch[k]) / len(fetch[k])
        w_ = sum(write.get(k, [0.0])) / max(len(write.get(k, [])), 1)
        name = k.replace("|", "/")
        name = name if len(name) <= 60 else name[:57] + "..."
        out.append(f"| `{name}` | {len(fetch[k])} | {f_:.1f} | {w_:.1f} | {(f_ * ff + w_ * wf) * 1024 / 1e6:.3f} |")
    out += ["", "```json", json.dumps(rec, indent=1), "```"]
    print("\n".join(out))


def cpu_baseline(wl, seconds):
    """The oracle (default exact projection, FP64) timed on the host on a
    bounded sample: as many MM iterations at gamma = 30 as fit in `seconds`
    after its own setup (kNN weights and Cholesky factorisation; the
    standardisation for the genotype workload)."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import mm, prep, weights
    X = prep.standardize_columns(wl.X, wl.mask) if wl.standardize else wl.X
    edges, w, _ = weights.knn_weights(X, wl.mask, wl.k, wl.phi)
    prob = mm.Problem(X, wl.mask, edges, w)
    rho, eps = prob.constants(30.0, mm.Opts())
    st = prob.initial_state()
    prob._cholesky()
    st, _ = prob.iterate(30.0, rho, eps, st, "exact")  # warm caches
    it = 0
    t0 = time.perf_counter()
    while True:
        st, _ = prob.iterate(30.0, rho, eps, st, "exact")
        it += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    threads = 1
    for lib in threadpool_info():
        if lib.get("user_api") == "blas":
            threads = max(threads, int(lib.get("num_threads", 1)))
    E = edges.shape[0]
    return {
        "value": it * E * wl.p / dt,
        "unit": "pair-feature updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{it} MM iterations (exact projection) at gamma=30 on the n={wl.n}, p={wl.p} "
                  f"workload, {dt:.1f} s; setup excluded",
        "host": {**host_cpu(), "blas_threads": threads,
                 "threads_note": "the exact projection's Cholesky solve runs on the BLAS threads; "
                                 "the sparse products and elementwise steps on one thread"},
    }


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=np.float64), q))


def _accuracy(infos, tol):
    """Share of solves whose stopping test passed, and the stopping rule's
    quantity at the last test (windowed change of U and A over max(1, ||U||),
    compared against tol * eta): how far capped solves are from stopping."""
    import numpy as np
    rc = np.array([i["rel_change"] for i in infos], dtype=np.float64)
    conv = np.array([i["converged"] for i in infos], dtype=np.float64)
    return {"converged_frac": float(conv.mean()) if conv.size else 0.0,
            "rel_change_median": float(np.median(rc)) if rc.size else 0.0,
            "rel_change_max": float(rc.max()) if rc.size else 0.0,
            "stop_threshold": tol * 1e-2}


def bench_batched(args):
    """Batched instances in shared launches against the plain per-solve path."""
    import numpy as np
    import torch

    import gen
    import paper_1409_2065_amd as cc
    opts = dict(max_iter=args.batch_max_iter, tol=args.batch_tol)

    def make(b):
        w = gen.batched_instance(b)
        X = torch.tensor(w.X, dtype=torch.float32, device="cuda")
        e, wt, _ = cc.build_knn_weights(X, None, k=w.k, phi=w.phi)
        return cc.Problem(X, None, e, wt, precision="mixed"), [float(g) for g in w.gammas]

    N = args.batch_instances
    inst = [make(b) for b in range(N)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt = cc.Batch([p for p, _ in inst], [g for _, g in inst], autotune=True, **opts)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    cfg = bt.config()
    classes, _ = bt.tuning()
    t0 = time.perf_counter()
    labs, infos, lat = bt.run(labels=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # one small instance's results, for the comparison with the oracle
    ob = ORACLE_BATCH_INSTANCE if ORACLE_BATCH_INSTANCE < N else 0
    sample = {"instance": ob, "labels": labs[ob].cpu().numpy(), "infos": infos[ob],
              "U": inst[ob][0].U(torch.float64).cpu().numpy()}
    solves = sum(len(g) for _, g in inst)
    print(f"[bench] batched: {N} instances, {solves} solves in {wall:.2f}s", file=sys.stderr, flush=True)
    bt.close()
    for p, _ in inst:
        p.close()
    # the plain path: every instance solved alone, one after another in
    # order, all present at the start (the batch's own arrival pattern); the
    # latency of instance b is the time from the start to the end of its path
    times, psolves, pinfos = [], 0, []
    nplain = N if args.plain_sample <= 0 else min(args.plain_sample, N)
    for b in range(nplain):
        p, g = make(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pinfos += p.solve_path(g, labels=True, **opts)[0]
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        psolves += len(g)
        p.close()
    fifo = np.cumsum(times)
    print(f"[bench] batched, plain path: {nplain} instances in {fifo[-1]:.2f}s", file=sys.stderr, flush=True)
    plain = {"instances": nplain, "solves_per_s": psolves / float(fifo[-1]), "wall_s": float(fifo[-1]),
             "fifo_latency_ms": {"p50": 1e3 * _pct(fifo, 50), "p99": 1e3 * _pct(fifo, 99), "max": 1e3 * float(fifo[-1])},
             "accuracy": _accuracy(pinfos, args.batch_tol)}
    if nplain < N:
        plain["note"] = f"the first {nplain} of {N} instances; latencies are of those"
    return {
        "instances": N, "solves": solves, "max_iter_per_gamma": args.batch_max_iter,
        "autotuned": {"classes": [{k: (round(v, 1) if isinstance(v, float) else v) for k, v in c.items()}
                                  for c in classes],
                      "class_key": "width_class: p <= 64, <= 128, <= 256, wider; size_class: point-sweep items "
                                   "<= 512, <= 2048, more; vec: 64*vec features per wave",
                      "largest_instance": {"vec": cfg["vec"], "items_per_wave": cfg["items_per_wave"],
                                           "us_per_iteration_candidates": [round(t, 1) for t in cfg["tune_us"]]},
                      "tune_s": round(tune_s, 3)},
        "solves_per_s": solves / wall, "wall_s": wall,
        "latency_ms": {"p50": _pct(lat, 50), "p99": _pct(lat, 99), "max": float(np.max(lat))},
        "mm_iterations": int(sum(i["iters"] for inf in infos for i in inf)),
        "tol": args.batch_tol,
        "accuracy": _accuracy([i for inf in infos for i in inf], args.batch_tol),
        "plain": plain,
        "oracle_sample": sample,
    }


ORACLE_BATCH_INSTANCE = 14  # n = 82, p = 83: the oracle runs its 16-gamma path in seconds


def batched_oracle_parity(sample, args):
    """A batched instance's results against the FP64 oracle on the oracle's
    own kNN weights (same stopping rule and cap): gammas whose stopping test
    passed on both sides, whether their labels agree, and the centres' error
    after the path."""
    import numpy as np

    import gen
    from oracle import mm, weights
    b = sample["instance"]
    wl = gen.batched_instance(b)
    X = np.asarray(wl.X, dtype=np.float32).astype(np.float64)
    E, w, _ = weights.knn_weights(X, None, wl.k, wl.phi)
    t0 = time.perf_counter()
    _, oinf, oU = mm.Problem(X, None, E, w).solve_path(
        [float(g) for g in wl.gammas], mm.Opts(proj="jacobi:1", max_iter=args.batch_max_iter, tol=args.batch_tol))
    cpu_s = time.perf_counter() - t0
    conv = [k for k, oi in enumerate(oinf) if oi.converged and sample["infos"][k]["converged"]]
    labels_equal = all(np.array_equal(sample["labels"][k], oinf[k].labels) for k in conv)
    return {
        "instance": b, "n": wl.n, "p": wl.p, "gammas": len(oinf),
        "converged_both": len(conv),
        "converged_oracle_only": sum(1 for k, oi in enumerate(oinf) if oi.converged and not sample["infos"][k]["converged"]),
        "labels_equal_where_converged": bool(labels_equal),
        "U_max_rel_diff_after_path": float(np.abs(sample["U"] - oU[-1]).max() / np.abs(oU[-1]).max()),
        "bar": {"U_rel": 1e-5},
        "oracle_s": round(cpu_s, 2),
    }


def serve_stream(cc, reqs, arrivals, budget, opts, max_active=256, round_iters=32, keep=None):
    """Submits each request at its arrival time to a continuous-batching
    server and steps it until every request is done; a client reads each
    result (labels on the device, infos) as soon as its request is done and
    releases it, so its budget share returns.  Returns wall time, per-request
    latency (arrival -> labels on the device, stamped by the server at the end
    of the round that finished the path), the per-gamma infos, and the peak
    of admitted requests and of counted device bytes."""
    import torch
    N = len(reqs)
    torch.cuda.synchronize()
    srv = cc.Server("mixed", hbm_budget=budget, max_active=max_active, round_iters=round_iters, **opts)
    t0 = time.perf_counter()
    tickets, nxt = {}, 0
    open_, lat, infos, kept = {}, [0.0] * N, [None] * N, None
    peak_active, peak_used, waited_rounds = 0, 0, 0
    while True:
        now = time.perf_counter() - t0
        while nxt < N and arrivals[nxt] <= now:
            w = reqs[nxt]
            tickets[nxt] = srv.submit(w.X, w.mask, k=w.k, phi=w.phi, gammas=w.gammas)
            open_[nxt] = tickets[nxt]
            nxt += 1
        a, wt, nd = srv.step()
        peak_active = max(peak_active, a)
        peak_used = max(peak_used, srv.memory()[0])
        waited_rounds += 1 if (wt > 0 and a > 0) else 0
        if nd:
            for r, t in list(open_.items()):
                st = srv.status(t)
                if st["state"] != 2:
                    continue
                lat[r] = st["t_done"] - st["t_submit"]
                if keep is not None and r == keep:
                    lab, inf, U = srv.result(t, U=True)
                    kept = {"request": keep, "labels": lab.cpu().numpy(), "infos": inf, "U": U.double().cpu().numpy()}
                else:
                    _, inf, _ = srv.result(t)
                infos[r] = inf
                srv.release(t)
                del open_[r]
        if nxt == N and a == 0 and wt == 0 and not open_:
            break
        if a == 0 and wt == 0 and nxt < N:
            time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
    wall = time.perf_counter() - t0
    srv.close()
    return {"wall": wall, "lat": lat, "infos": [i for inf in infos for i in inf], "peak_active": peak_active,
            "peak_used": peak_used, "rounds_with_waiting": waited_rounds, "kept": kept}


def bench_served(args):
    """Requests of the Poisson stream at their arrival times.
      stream     the first --serve-requests requests at 200/s (far beyond
                 what one GPU sustains: saturated), admitted within an HBM
                 budget of --serve-budget-mib that binds;
      fifo       the first --serve-fifo of them on the server and, apart,
                 solved first come first served by the plain path;
      rate_sweep --serve-sweep-requests requests at each of the
                 --serve-rates arrival rates on the server.
    Every solve stops at tol --serve-tol or --serve-max-iter MM iterations per
    gamma on both sides; the converged share is stated."""
    import numpy as np
    import torch

    import gen
    import paper_1409_2065_amd as cc
    opts = dict(max_iter=args.serve_max_iter, tol=args.serve_tol)
    budget = args.serve_budget_mib << 20
    N = args.serve_requests
    reqs = [gen.served_instance(r) for r in range(N)]
    arr = gen.served_arrivals(200.0, N)

    def summary(res, reqs_):
        solves = sum(len(w.gammas) for w in reqs_)
        return {"requests": len(reqs_), "solves": solves, "wall_s": res["wall"],
                "solves_per_s": solves / res["wall"], "requests_per_s": len(reqs_) / res["wall"],
                "latency_s": {"p50": _pct(res["lat"], 50), "p99": _pct(res["lat"], 99), "max": float(np.max(res["lat"]))},
                "accuracy": _accuracy(res["infos"], args.serve_tol)}

    res = serve_stream(cc, reqs, arr, budget, opts)
    stream = summary(res, reqs)
    stream.update({"arrival_rate_per_s": 200.0, "hbm_budget_bytes": budget, "peak_admitted": res["peak_active"],
                   "peak_counted_bytes": res["peak_used"], "rounds_with_requests_waiting": res["rounds_with_waiting"]})
    print(f"[bench] served stream: {N} requests in {res['wall']:.2f}s", file=sys.stderr, flush=True)

    M = min(args.serve_fifo, N)
    small = int(np.argmin([w.n * w.p for w in reqs[:M]]))  # compared with the oracle
    res_m = serve_stream(cc, reqs[:M], arr[:M], budget, opts, keep=small)
    t0 = time.perf_counter()
    lat2, pinfos = [], []
    for r, w in enumerate(reqs[:M]):
        now = time.perf_counter() - t0
        if now < arr[r]:
            time.sleep(arr[r] - now)
        X = torch.tensor(np.nan_to_num(w.X), dtype=torch.float32, device="cuda")
        Mk = torch.tensor(w.mask.astype(np.uint8), device="cuda")
        e, wt, _ = cc.build_knn_weights(X, Mk, k=w.k, phi=w.phi)
        with cc.Problem(X, Mk, e, wt, precision="mixed") as pr:
            pinfos += pr.solve_path([float(g) for g in w.gammas], labels=True, **opts)[0]
        torch.cuda.synchronize()
        lat2.append(time.perf_counter() - t0 - arr[r])
    wall2 = time.perf_counter() - t0
    print(f"[bench] served head-to-head: {M} requests, server {res_m['wall']:.2f}s, plain {wall2:.2f}s",
          file=sys.stderr, flush=True)
    fifo = {"server": summary(res_m, reqs[:M]),
            "plain_fifo": summary({"wall": wall2, "lat": lat2, "infos": pinfos}, reqs[:M])}

    sweep = []
    S = min(args.serve_sweep_requests, N)
    for rate in [float(x) for x in args.serve_rates.split(",") if x]:
        r_ = serve_stream(cc, reqs[:S], gen.served_arrivals(rate, S), budget, opts)
        sweep.append({"arrival_rate_per_s": rate, **summary(r_, reqs[:S]), "peak_admitted": r_["peak_active"]})
        print(f"[bench] served at {rate}/s: {S} requests in {r_['wall']:.2f}s", file=sys.stderr, flush=True)
    return {"max_iter_per_gamma": args.serve_max_iter, "tol": args.serve_tol,
            "stream": stream, "head_to_head": fifo, "rate_sweep": sweep, "oracle_sample": res_m["kept"]}


def served_oracle_parity(sample, args):
    """A served request's results against the FP64 oracle on the oracle's own
    kNN weights of the same data and mask, with the same stopping rule and
    cap: gammas converged on both sides, their labels, U after the path."""
    import numpy as np

    import gen
    from oracle import mm, weights
    r = sample["request"]
    wl = gen.served_instance(r)
    X = np.where(wl.mask, np.asarray(np.nan_to_num(wl.X), dtype=np.float32).astype(np.float64), np.nan)
    E, w, _ = weights.knn_weights(X, wl.mask, wl.k, wl.phi)
    t0 = time.perf_counter()
    _, oinf, oU = mm.Problem(X, wl.mask, E, w).solve_path(
        [float(g) for g in wl.gammas], mm.Opts(proj="jacobi:1", max_iter=args.serve_max_iter, tol=args.serve_tol))
    cpu_s = time.perf_counter() - t0
    conv = [k for k, oi in enumerate(oinf) if oi.converged and sample["infos"][k]["converged"]]
    return {
        "request": r, "n": wl.n, "p": wl.p, "gammas": len(oinf),
        "converged_both": len(conv),
        "converged_oracle_only": sum(1 for k, oi in enumerate(oinf) if oi.converged and not sample["infos"][k]["converged"]),
        "labels_equal_where_converged": bool(all(np.array_equal(sample["labels"][k], oinf[k].labels) for k in conv)),
        "U_max_rel_diff_after_path": float(np.abs(sample["U"] - oU[-1]).max() / np.abs(oU[-1]).max()),
        "bar": {"U_rel": 1e-5},
        "oracle_s": round(cpu_s, 2),
    }


def bench_extras(X, M, edges, w, gammas, args):
    """The paper's extras on the headline workload: principal components,
    the smallest connected k, composite-distance weights, and the 30-gamma
    path (each gamma capped at --extras-max-iter iterations) returned as U
    on the host against its projection on two principal components."""
    import numpy as np
    import torch

    import paper_1409_2065_amd as cc

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, 1e3 * (time.perf_counter() - t0)

    (V, sval, center), pca_ms = timed(lambda: cc.pca(X, M, r=2, iters=100))
    (kmin, ncomp), mink_ms = timed(lambda: cc.min_connected_k(X, M, k_max=128))
    rng = np.random.default_rng(7)
    n = X.shape[0]
    Y = torch.tensor(np.stack([rng.uniform(-60, 60, n), rng.uniform(-180, 180, n)], axis=1), device="cuda")
    _, comp_ms = timed(lambda: cc.composite_weights(edges, X, Y, 0.5, -0.5, geodesic=True, radius=6371.0,
                                                    mask=M))
    opts = dict(max_iter=args.extras_max_iter, labels=True)
    with cc.Problem(X, M, edges, w, precision="mixed") as g:
        (_, _, Up), _ = timed(lambda: g.solve_path(gammas, U_path=True, **opts))
        g.reset_state()
        _, u_ms = timed(lambda: (g.solve_path(gammas, U_path=True, **opts)[2].cpu()))
        g.reset_state()
        _, pc_ms = timed(lambda: (g.solve_path_pc(gammas, V, center, **opts)[2].cpu()))
    return {
        "pca": {"r": 2, "iters": 100, "ms": pca_ms, "singular_values": [float(v) for v in sval]},
        "min_connected_k": {"k_max": 128, "k_min": kmin, "components_at_k_max": ncomp, "ms": mink_ms},
        "composite_weights": {"alpha": 0.5, "geodesic": True, "edges": int(edges.shape[0]), "ms": comp_ms},
        "path_to_host": {"gammas": len(gammas), "max_iter_per_gamma": args.extras_max_iter,
                         "U_ms": u_ms, "U_bytes": int(Up.numel() * 4),
                         "projected_ms": pc_ms, "projected_bytes": int(len(gammas) * n * 2 * 8)},
    }


def host_cpu():
    """The host the CPU baseline runs on: logical CPUs, those this process may
    use, and the CPU model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 0
    return {"nproc": os.cpu_count() or 0, "usable": usable, "model": model}


def run_workload(cc, name, precision, steps, warmup, max_iter, sample_every, log):
    """One workload's timed path: inputs on the device, kNN weights built
    (timed separately), then `steps` timed steps of reset + the warm-started
    gamma path with labels, each gamma capped at max_iter MM iterations.
    Returns the result fields and the device inputs."""
    import numpy as np
    import torch

    import gen
    dev = torch.device("cuda:0")
    wl = gen.make(name)
    n, p = wl.n, wl.p
    X = torch.tensor(np.nan_to_num(wl.X), dtype=torch.float32, device=dev)
    M = None if wl.mask is None else torch.tensor(wl.mask.astype(np.uint8), device=dev)
    if wl.standardize:
        cc.standardize_columns(X, M)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    edges, w, phi_used = cc.build_knn_weights(X, M, k=wl.k, phi=wl.phi)
    torch.cuda.synchronize()
    knn_s = time.perf_counter() - t0
    E = int(edges.shape[0])
    prob = cc.Problem(X, M, edges, w, precision=precision)
    gammas = [float(g) for g in wl.gammas]
    opts = dict(max_iter=max_iter, warm_start=1)

    def step():
        prob.reset_state()
        infos, labels, _ = prob.solve_path(gammas, labels=True, **opts)
        return infos, labels

    for k in range(warmup):
        step()
        log(f"{name}: warmup step {k + 1}/{warmup} done")
    torch.cuda.synchronize()
    prob.profile(sample_every)
    iters = 0
    converged = 0
    clusters = []
    t0 = time.perf_counter()
    for k in range(steps):
        infos, labels = step()
        log(f"{name}: timed step {k + 1}/{steps} done")
        iters += sum(i["iters"] for i in infos)
        converged += sum(i["converged"] for i in infos)
        clusters = [i["n_clusters"] for i in infos]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ks = prob.kernel_stats()
    prob.profile(0)
    prob.close()

    has_mask = M is not None
    alg_point, alg_iter, k1 = algorithmic_bytes(n, p, E, has_mask)
    impl_point, impl_pf = implementation_bytes(n, p, E, precision, has_mask)
    pt_ms = ks["point_sweep"]["avg_ms"]
    iter_ms = dt * 1e3 / max(iters, 1)
    achieved = alg_point / (pt_ms * 1e-3) / 1e9 if pt_ms > 0 else 0.0
    it_achieved = alg_iter / (iter_ms * 1e-3) / 1e9 if iter_ms > 0 else 0.0
    out = {
        "value": iters * E * p / dt,
        "ms_per_step": dt * 1e3 / steps,
        "config": {
            "workload": WORKLOAD_TEXT[name] + ("" if max_iter >= 20000 else f", at most {max_iter} MM iterations per gamma"),
            "n": n, "p": p, "edges": E, "gammas": len(gammas), "precision": precision,
            "mm_iterations_per_step": iters // max(steps, 1),
            "gammas_converged_per_step": converged // max(steps, 1),
            "clusters_along_path": clusters,
            "knn_build_s": round(knn_s, 4),
            "phi": phi_used,
            "kernel_ms": {k: round(v["avg_ms"], 5) for k, v in ks.items()},
            "iteration_ms_kernels": round(sum(v["avg_ms"] for v in ks.values()), 5),
            "iteration_ms_wall": round(iter_ms, 5),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_point (point sweep: U update + Jacobi projection sweep)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": stored_traffic(name, precision),
            "bytes_per_launch": alg_point,
            "bytes_per_point_feature": k1,
            "bytes_rule": f"{k1} B per point-feature (FP32 state: X, "
                          + ("mask, " if has_mask else "") + "U read and write, A' read, A write) + 24 B per edge",
            "precision_overhead_bytes": impl_point - alg_point,
            "implementation_bytes_per_launch": impl_point,
            "implementation_bytes_per_point_feature": impl_pf,
            "iteration": {"bytes": alg_iter, "bytes_rule": f"{k1 + 8} B per point-feature + 60 B per edge",
                          "achieved": it_achieved, "frac": it_achieved / HBM_PEAK_GBS},
        },
    }
    return out, (X, M, edges, w, gammas, wl)


def oracle_parity(cc, X, M, edges, w, wl, gamma=30.0, iters=20):
    """The error against the FP64 oracle of the configuration the headline
    times: the oracle's own kNN weights (edge set compared with the GPU's),
    then `iters` MM iterations at `gamma` from the initial state on both
    sides, the oracle with one Jacobi sweep per iteration as the GPU; max
    relative differences of U and A, the largest shrink-factor difference,
    and whether the fused edges agree."""
    import numpy as np
    import torch

    from oracle import mm, weights
    Xh = np.asarray(wl.X, dtype=np.float32).astype(np.float64)
    E, wo, _ = weights.knn_weights(Xh, wl.mask, wl.k, wl.phi)
    Eg = edges.cpu().numpy()
    same_edges = bool(Eg.shape == E.shape and np.array_equal(Eg, E))
    w_rel = float(np.abs(w.cpu().numpy() - wo).max() / np.abs(wo).max()) if same_edges else None
    t0 = time.perf_counter()
    st, info = mm.Problem(Xh, wl.mask, E, wo).solve(gamma, mm.Opts(tol=0, max_iter=iters, proj="jacobi:1"))
    cpu_s = time.perf_counter() - t0
    with cc.Problem(X, M, edges, w, precision="mixed") as g:
        g.solve(gamma, tol=0.0, max_iter=iters)
        U, A, s = (t.cpu().numpy() for t in g.get_state())
    torch.cuda.synchronize()

    def rel(a, b):
        return float(np.abs(a - b).max() / np.abs(b).max())
    return {
        "workload": "expression n=2000 p=500 (the headline's inputs)",
        "oracle": "FP64, one Jacobi sweep per MM iteration, from the initial state",
        "gamma": gamma, "mm_iterations": iters,
        "knn_edges_equal": same_edges, "weights_max_rel_diff": w_rel,
        "U_max_rel_diff": rel(U, st.U), "A_max_rel_diff": rel(A, st.A),
        "s_max_abs_diff": float(np.abs(s - st.s).max()),
        "fused_edges_equal": bool(np.array_equal(s == 0, st.s == 0)),
        "bar": {"U_A_rel": 2e-6, "s_abs": 1e-6},
        "oracle_s": round(cpu_s, 2),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "f32", "f64"])
    ap.add_argument("--workload", default="expression", choices=["expression", "genotype", "plain"],
                    help="expression (n=2000, p=500) is the headline; the others are for profiling")
    ap.add_argument("--max-iter", type=int, default=20000, help="MM iteration cap per gamma")
    ap.add_argument("--sample-every", type=int, default=8, help="kernel timing sample period")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-genotype", action="store_true")
    ap.add_argument("--genotype-steps", type=int, default=3)
    ap.add_argument("--genotype-max-iter", type=int, default=50)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch-instances", type=int, default=256)
    ap.add_argument("--batch-max-iter", type=int, default=1000)
    ap.add_argument("--batch-tol", type=float, default=1e-3)
    ap.add_argument("--plain-sample", type=int, default=0, help="instances the plain path solves (0: all)")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-fifo", type=int, default=32)
    ap.add_argument("--serve-sweep-requests", type=int, default=16)
    ap.add_argument("--serve-rates", default="2,5,10")
    ap.add_argument("--serve-budget-mib", type=int, default=1024)
    ap.add_argument("--serve-max-iter", type=int, default=1000)
    ap.add_argument("--serve-tol", type=float, default=1e-3)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras-max-iter", type=int, default=100)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first copy this many MiB device to device (counter calibration)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 counter CSVs (no GPU) and exit")
    ap.add_argument("--pmc-command", default="", help="command text recorded in the summary")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.calibrate_copy_mib, args.pmc_command)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}); "
              "feature sharding across GPUs is described in the design notes and not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1409_2065_amd as cc

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    cc.load()
    dev = torch.device("cuda:0")
    if args.calibrate_copy_mib > 0:
        src = torch.ones(args.calibrate_copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"copied {args.calibrate_copy_mib} MiB for counter calibration")
    head, (X, M, edges, w, gammas, wl) = run_workload(
        cc, args.workload, args.precision, args.steps, args.warmup, args.max_iter, args.sample_every, log)
    n, p = wl.n, wl.p
    result = {
        "metric": METRIC if args.workload == "expression" else f"pair-feature updates/s (n={n},p={p})",
        "value": head["value"],
        "unit": "pair-feature updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f64 point arithmetic and U, A as f32 hi + f32 lo, f32 pair gathers", "f32": "f32", "f64": "f64"}[args.precision],
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
    }
    if not args.no_extras and args.workload == "expression":
        result["extras"] = bench_extras(X, M, edges, w, gammas, args)
        log("extras done")
    if not args.no_genotype and args.workload == "expression":
        geno, _ = run_workload(cc, "genotype", args.precision, args.genotype_steps, 1, args.genotype_max_iter,
                               args.sample_every, log)
        result["genotype"] = {"metric": "pair-feature updates/s (n=1000,p=20000)", "unit": "pair-feature updates/s",
                              "steps": args.genotype_steps, **geno}
    batched = served = None
    if not args.no_batched:
        result["batched"] = batched = bench_batched(args)
    if not args.no_served:
        result["served"] = served = bench_served(args)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
        log("cpu baseline done")
        if not args.no_parity and args.workload == "expression":
            result["parity"] = {"expression": oracle_parity(cc, X, M, edges, w, wl)}
            if batched is not None and "oracle_sample" in batched:
                result["parity"]["batched"] = batched_oracle_parity(batched.pop("oracle_sample"), args)
            if served is not None and served.get("oracle_sample"):
                result["parity"]["served"] = served_oracle_parity(served.pop("oracle_sample"), args)
            log("parity done")
    for leg in (batched, served):
        if leg is not None:
            leg.pop("oracle_sample", None)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
