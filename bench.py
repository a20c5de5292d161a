#!/usr/bin/env python3
"""HODLRdD matvec throughput on one MI355X.

Workload: 2^18 points i.i.d. uniform in [-1,1]^3, kernel 1/r (diagonal 0),
leaf size 64, ACA tolerance 1e-10, one N(0,1) right-hand side.  The library
builds the representation once (tree, lists, ACA: setup, reported apart) and
a step is one full matvec: permutation, projections, expansions of every
level, near field evaluated on the fly, permutation back.

Two precisions are timed on the same inputs: FP64 (factors and arithmetic)
and mixed (FP32 factors, FP32 arithmetic).  `value` is the FP64 throughput;
the mixed figures are in `mixed`; `skeleton` times the same product with
the skeleton storage form (pivots and LU of K(sigma, tau), kernel evaluated
on the fly).  `multi_rhs` times the matrix-core path on
its own workload (2^19 points in 4D, 1/r^2, 32 right-hand sides, BF16
factors); `solve` times GMRES with FP64 iterative refinement on the 2^20-point
Gaussian-mixture workload; `serve` reports p50/p99 latency of a Poisson
request stream on resident point sets; `admissibility` compares the
admissibility conditions on a 4D workload.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _events(torch, n):
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


NCLASS = 6
CLASS_KERNELS = ["k_lr_group<8>", "k_lr_group<16>", "k_lr_stream<1,1,8>", "k_lr_stream<1,2,4>",
                 "k_lr_stream<4,4,*>", "k_lr_stream<8,9,*>"]


def time_matvecs(P, torch, H, X, Y, prec, warmup, steps):
    """Warm-up, then `steps` matvecs, each with 11 HIP events recorded by the
    library on the stream: the 4 stages and the launch of every block class."""
    for _ in range(warmup):
        P.hodlr_matvec(H.h, X, Y, prec)
    torch.cuda.synchronize()
    evs = [_events(torch, 5 + NCLASS) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e in evs:
        P.hodlr_matvec_events(H.h, X, Y, e, prec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(4)] for e in evs])  # ms
    # class c runs between the previous class's event (or the end of stage 1)
    # and its own
    cls = np.array([[(e[1] if c == 0 else e[4 + c]).elapsed_time(e[5 + c]) for c in range(NCLASS)]
                    for e in evs])
    lat = np.array([e[0].elapsed_time(e[4]) for e in evs])
    return wall, stages, cls, lat


def roofline(info, cls_ms, sf, sc):
    """Dominant block-class kernel: algorithmic bytes (every stored factor
    element of its blocks once, plus the x reads and contribution writes)
    over its measured average duration."""
    c = int(np.argmax(cls_ms))
    nbytes = info.class_factor_elems[c] * sf + info.class_vector_elems[c] * sc
    achieved = nbytes / (cls_ms[c] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": CLASS_KERNELS[c], "blocks": int(info.class_blocks[c]),
            "bytes_per_launch": int(nbytes), "avg_ms": float(cls_ms[c]), "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS}


def measured_traffic(workload, kernel, storage):
    """HBM bytes per launch of `kernel` from the committed counter summaries
    under profiles/ (FETCH_SIZE and WRITE_SIZE passes, scaled by a copy of
    known size), or None when none matches or the apply source has changed
    since the counters were taken."""
    import glob
    import hashlib
    with open(os.path.join(ROOT, "paper_2209_05819_amd", "csrc", "apply.hip"), "rb") as f:
        cur = hashlib.sha256(f.read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        rec = {}
        with open(path) as f:
            for line in f:
                k, sep, v = line.strip().partition(": ")
                if sep and k in ("workload", "kernel", "storage", "traffic_bytes",
                                 "apply_hip_sha256"):
                    rec[k] = v.strip()
        if (rec.get("workload"), rec.get("kernel"), rec.get("storage")) == (workload, kernel,
                                                                            storage):
            if rec.get("apply_hip_sha256") != cur:
                return None
            return float(rec["traffic_bytes"])
    return None


def multi_rhs(P, torch, W, steps, warmup, n_override=0):
    """Several right-hand sides on matrix cores: 2^19 points uniform in
    [-1,1]^4, 1/r^2, leaf 128, ACA 1e-8, 32 N(0,1) right-hand sides in FP32,
    BF16 factors, FP32 accumulation.  Error against the direct sum on
    sampled rows."""
    import oracle
    w = W.WORKLOADS["uniform4d_invr2_n524288"]
    if n_override:
        w = W.scaled(w, n_override)
    pts, q = w.points(), w.rhs()
    N, nrhs = w.N, q.shape[1]
    kern = P.make_kernel(w.kernel, h=w.h, diag=w.diag)
    t0 = time.perf_counter()
    H = P.HODLR(pts, kern, w.leaf, w.tol, domain=w.domain, storage=P.BF16)
    torch.cuda.synchronize()
    build = time.perf_counter() - t0
    info = H.info()
    print(f"[bench] multi-RHS BF16 build {build:.1f} s kappa={info.kappa}", file=sys.stderr,
          flush=True)
    X = torch.tensor(np.ascontiguousarray(q.T), dtype=torch.float32, device="cuda").t()
    Y = torch.empty((nrhs, N), dtype=torch.float32, device="cuda").t()
    wall, per, cls, lat = time_matvecs(P, torch, H, X, Y, P.FP32, warmup, steps)
    st = per.mean(axis=0)
    y = Y.t().contiguous().cpu().numpy().T
    oracle.build(force=False)
    rows = np.sort(W.rng(203).choice(N, size=min(N, 512), replace=False))
    bd = oracle.direct(pts, oracle.kernel(w.kernel, diag=w.diag), q, rows=rows)
    err = float(np.linalg.norm(y[rows] - bd) / np.linalg.norm(bd))
    fe = sum(info.factor_elems[l] for l in range(1, info.kappa + 1))
    proj_b = 2 * sum(info.mfma_proj_factor_elems)
    exp_b = 2 * info.mfma_expand_factor_elems
    # dominant pass: projections (stage 2) or expansions (stage 3); bytes
    # are the factor elements that pass reads, once
    if st[2] >= st[1]:
        pass_name, pass_b, pass_ms = "expansions (k_mexp, every level)", exp_b, st[2]
    else:
        pass_name, pass_b, pass_ms = "projections (k_mproj, every width, k_mreduce)", proj_b, st[1]
    # the longest single projection launch (panels up to 128, 256, 512
    # columns: <waves, column tiles, 64-column groups per wave> = <1,CT,2>,
    # <2,CT,2>, <2,CT,4>; the events of the launch for panels up to 64 also
    # hold the x conversion before it): its factor elements and x slices
    # (BF16, 32 columns) over its event time
    nrp = 16 * ((nrhs + 15) // 16)
    cm = cls.mean(axis=0)
    wi = 1 + int(np.argmax(cm[1:4]))
    kern_name = "k_mproj<{},{},{}>".format(*{1: (1, nrp // 16, 2), 2: (2, nrp // 16, 2),
                                             3: (2, nrp // 16, 4)}[wi])
    nb = 2 * info.mfma_proj_factor_elems[wi] + 2 * nrp * info.mfma_proj_vector_elems[wi]
    ms = float(cm[wi])
    ach = nb / (ms * 1e-3) / 1e9
    mfma_tf = 2.0 * nrp * info.mfma_proj_factor_elems[wi] / (ms * 1e-3) / 1e12
    traffic = measured_traffic(w.name, kern_name, "bf16")
    del H
    return {
        "workload": w.name, "N": N, "d": w.d, "nrhs": nrhs, "kernel": "1/r^2, diag 0",
        "leaf": w.leaf, "aca_tol": w.tol, "dtype": "bf16 factors, f32 accumulation",
        "value": N * nrhs / (wall / steps), "unit": "N*nrhs/s",
        "ms_per_step": wall / steps * 1e3,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "rel_err": err, "rel_err_ref": "direct sum on 512 sampled rows (seed 203)",
        "stage_ms": [round(float(v), 4) for v in st],
        "stages": ["permute_in", "projections (pass 1)", "expansions (pass 2)",
                   "near_field+permute_out"],
        "build_s": round(build, 2), "kappa": info.kappa, "factor_bytes": int(2 * fe),
        "roofline": {"bound": "hbm", "kernel": kern_name,
                     "jobs": int(info.mfma_proj_jobs[wi]), "bytes_per_launch": int(nb),
                     "avg_ms": ms, "achieved": ach, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                     "mfma_tflops": mfma_tf, "mfma_peak_tflops": 2500.0},
        "pass_roofline": {"pass": pass_name, "bytes": int(pass_b), "ms": float(pass_ms),
                          "achieved": pass_b / (pass_ms * 1e-3) / 1e9,
                          "frac": pass_b / (pass_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "proj_launch_ms": [round(float(v), 4) for v in cm[:4]],
    }


def multi_rhs_fp32(P, torch, W, steps, n_override=0):
    """The same 32-RHS product with FP32 factors (precision-aware truncation)
    and FP32 arithmetic on the lane-parallel block kernels, eight columns per
    pass over the factors: error against the direct sum on the same sampled
    rows, and the factor bytes streamed per product."""
    import oracle
    w = W.WORKLOADS["uniform4d_invr2_n524288"]
    if n_override:
        w = W.scaled(w, n_override)
    pts, q = w.points(), w.rhs()
    N, nrhs = w.N, q.shape[1]
    kern = P.make_kernel(w.kernel, h=w.h, diag=w.diag)
    t0 = time.perf_counter()
    H = P.HODLR(pts, kern, w.leaf, w.tol, domain=w.domain, storage=P.FP32)
    torch.cuda.synchronize()
    build = time.perf_counter() - t0
    info = H.info()
    print(f"[bench] multi-RHS FP32 build {build:.1f} s kappa={info.kappa}", file=sys.stderr,
          flush=True)
    X = torch.tensor(np.ascontiguousarray(q.T), dtype=torch.float32, device="cuda").t()
    Y = torch.empty((nrhs, N), dtype=torch.float32, device="cuda").t()
    wall, per, cls, lat = time_matvecs(P, torch, H, X, Y, P.FP32, 1, steps)
    ms = wall / steps * 1e3
    y = Y.t().contiguous().cpu().numpy().T.astype(np.float64)
    rows = np.sort(W.rng(203).choice(N, size=min(N, 512), replace=False))
    bd = oracle.direct(pts, oracle.kernel(w.kernel, diag=w.diag), q, rows=rows)
    err = float(np.linalg.norm(y[rows] - bd) / np.linalg.norm(bd))
    fe = sum(info.factor_elems[l] for l in range(1, info.kappa + 1))
    passes = (nrhs + 7) // 8
    streamed = 4 * fe * passes
    print(f"[bench] multi-RHS FP32 {ms:.2f} ms per product, rel err {err:.2e}", file=sys.stderr,
          flush=True)
    del H
    return {
        "dtype": "f32 factors, f32 arithmetic", "value": N * nrhs / (ms * 1e-3),
        "unit": "N*nrhs/s", "ms_per_step": ms,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "rel_err": err, "rel_err_ref": "direct sum on 512 sampled rows (seed 203)",
        "build_s": round(build, 2), "factor_bytes": int(4 * fe),
        "passes_over_factors": passes, "streamed_gbs": streamed / (ms * 1e-3) / 1e9,
        "stage_ms": [round(float(v), 4) for v in per.mean(axis=0)],
    }


def small_bench(P, torch, W, reps=200):
    """The small workload (4096 points uniform in [-1,1]^2, log r, leaf 64,
    ACA 1e-8, FP64, one U[-1,1] right-hand side): the autotuner's choice
    (tile shapes per block class; per-class launches with the near field on
    a second stream or all on one stream, or one persistent launch), and
    the per-call latency of the product on the three routes, launched
    eagerly and replayed from a captured HIP graph; the error against the
    direct N^2 sum on every row."""
    import oracle
    w = W.WORKLOADS["uniform2d_log_n4096"]
    pts, q = w.points(), w.rhs()[:, 0]
    N = w.N
    H = P.HODLR(pts, P.make_kernel(w.kernel, h=w.h, diag=w.diag), w.leaf, w.tol, domain=w.domain,
                level_rule=1)
    tune = P.hodlr_autotune(H.h, 1, P.FP64, P.FP64)
    P.hodlr_reserve_workspace(H.h, 1, P.FP64)
    X = torch.tensor(q, dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)

    def per_call(fn):
        ev = _events(torch, reps + 1)
        ev[0].record()
        for i in range(reps):
            fn()
            ev[i + 1].record()
        torch.cuda.synchronize()
        return np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(reps)])

    def wall_per_call(fn):
        t = np.empty(reps)
        for i in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            t[i] = (time.perf_counter() - t0) * 1e3
        return t

    routes = {}
    for name, route in (("per_class", 0), ("per_class_one_stream", 2), ("persistent", 1)):
        P.hodlr_set_route(H.h, route)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(3):
                P.hodlr_matvec(H.h, X, Y)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            P.hodlr_matvec(H.h, X, Y)
        torch.cuda.synchronize()
        eager = per_call(lambda: P.hodlr_matvec(H.h, X, Y))
        graph = per_call(g.replay)
        eager_w = wall_per_call(lambda: P.hodlr_matvec(H.h, X, Y))
        graph_w = wall_per_call(g.replay)
        routes[name] = {
            "eager_p50_ms": float(np.percentile(eager, 50)),
            "eager_p99_ms": float(np.percentile(eager, 99)),
            "graph_p50_ms": float(np.percentile(graph, 50)),
            "graph_p99_ms": float(np.percentile(graph, 99)),
            "eager_wall_p50_ms": float(np.percentile(eager_w, 50)),
            "graph_wall_p50_ms": float(np.percentile(graph_w, 50)),
        }
        del g
    P.hodlr_set_route(H.h, tune.route)
    Y = H.matvec(X)
    torch.cuda.synchronize()
    y = Y.cpu().numpy()
    bd = oracle.direct(pts, oracle.kernel(w.kernel, h=w.h, diag=w.diag), q[:, None])[:, 0]
    err = float(np.linalg.norm(y - bd) / np.linalg.norm(bd))
    info = H.info()
    del H
    best = min(min(r["eager_p50_ms"], r["graph_p50_ms"]) for r in routes.values())
    return {
        "workload": w.name, "N": N, "d": w.d, "kernel": "log r, diag 0", "leaf": w.leaf,
        "aca_tol": w.tol, "kappa": info.kappa, "dtype": "f64",
        "autotune": {"route": {0: "per_class", 1: "persistent",
                               2: "per_class_one_stream"}[tune.route],
                     "class_choice": list(tune.class_choice)[:6],
                     "class_ms": [round(v, 5) for v in list(tune.class_ms)[:6]],
                     "per_class_route_ms": tune.class_route_ms,
                     "per_class_one_stream_ms": tune.one_stream_ms,
                     "persistent_route_ms": tune.persistent_ms},
        "routes": routes,
        "gpu_time": "HIP events between back-to-back calls on the stream",
        "wall_time": "host clock, one call then a synchronisation (launch included)",
        "value": N / (best * 1e-3),
        "unit": "N*nrhs/s (back-to-back, the fastest route and launch mode)",
        "rel_err": err, "rel_err_ref": "direct N^2 sum, every row",
    }


def mixture_trees(P, torch, W, w, pts, q, steps=5):
    """The 16-RHS BF16 product on the Gaussian-mixture cloud with the
    closed-form balanced tree and with the adaptive tree: blocks, dense pairs,
    factor bytes, build and product times, error against the direct sum on
    256 sampled rows.  Returns (records, the adaptive handle)."""
    import oracle
    N, nrhs = w.N, q.shape[1]
    k = P.make_kernel(w.kernel, h=w.h, diag=w.diag)
    rows = np.sort(W.rng(211).choice(N, 256, replace=False))
    bd = oracle.direct(pts, oracle.kernel(w.kernel, h=w.h, diag=w.diag), q, rows=rows)
    X = torch.tensor(np.ascontiguousarray(q.T), dtype=torch.float32, device="cuda").t()
    out, keep = {}, None
    for name, rule in (("closed_form", 1), ("adaptive", 2)):
        t0 = time.perf_counter()
        H = P.HODLR(pts, k, w.leaf, w.tol, domain=w.domain, storage=P.BF16, level_rule=rule)
        torch.cuda.synchronize()
        build = time.perf_counter() - t0
        Y = torch.empty((nrhs, N), dtype=torch.float32, device="cuda").t()
        wall, per, _, _ = time_matvecs(P, torch, H, X, Y, P.FP32, 1, steps)
        ms = wall / steps * 1e3
        y = Y.t().contiguous().cpu().numpy().T.astype(np.float64)
        info = H.info()
        fe = sum(info.factor_elems[l] for l in range(1, info.kappa + 1))
        nblk = sum(info.stored_blocks[l] for l in range(1, info.kappa + 1))
        out[name] = {
            "kappa": info.kappa, "stored_blocks": int(nblk),
            "near_pairs": int(info.near_pairs), "factor_bytes": int(2 * fe),
            "build_s": round(build, 2), "ms_per_product": ms,
            "stage_ms": [round(float(v), 3) for v in per.mean(axis=0)],
            "value": N * nrhs / (ms * 1e-3), "unit": "N*nrhs/s",
            "rel_err": rel_err_rows(y, bd, rows),
        }
        print(f"[bench] mixture {name}: {ms:.2f} ms per 16-RHS product, "
              f"near pairs {info.near_pairs:.3e}, build {build:.1f} s", file=sys.stderr, flush=True)
        if rule == 2:
            keep = H
        else:
            del H
    return out, keep


def solve_bench(P, torch, W, n_override=0):
    """GMRES with FP64 iterative refinement: (I + K/N) U = F on the 2^20-point
    Gaussian-mixture cloud (exp(-r^2/0.25), diagonal 1 + 1e-3, leaf 64, ACA
    1e-6), 16 N(0,1) right-hand sides; FP64 residuals on FP64 factors, inner
    GMRES on BF16 factors, to a relative residual of 1e-10.  Both
    representations on the adaptive tree; the product on this cloud is
    compared between the closed-form and the adaptive tree first."""
    w = W.WORKLOADS["mixture3d_gauss_n1048576"]
    if n_override:
        w = W.scaled(w, n_override)
    pts, q = w.points(), w.rhs()
    N, nrhs = w.N, q.shape[1]
    k = P.make_kernel(w.kernel, h=w.h, diag=w.diag)
    trees, H16 = mixture_trees(P, torch, W, w, pts, q)
    t0 = time.perf_counter()
    H64 = P.HODLR(pts, k, w.leaf, w.tol, domain=w.domain, level_rule=2)
    torch.cuda.synchronize()
    build = time.perf_counter() - t0 + trees["adaptive"]["build_s"]
    F = torch.tensor(np.ascontiguousarray(q.T), dtype=torch.float64, device="cuda").t()
    U = torch.zeros((nrhs, N), dtype=torch.float64, device="cuda").t()
    o = P.default_solve_opts()
    o.tol, o.inner_tol, o.restart, o.max_outer = 1e-10, 1e-3, 30, 20
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = P.hodlr_solve(H64.h, H16.h, 1.0, 1.0 / N, F, U, o)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    print(f"[bench] solve {secs:.2f} s outer {info.outer_iters} inner {info.inner_iters} "
          f"rel {info.rel_residual:.2e}", file=sys.stderr, flush=True)
    del H16
    c4 = gram_solve(P, torch, W, w, pts, q, H64, build)
    del H64
    return {
        "workload": w.name, "system": "(I + K/N) U = F", "N": N, "nrhs": nrhs,
        "kernel": "exp(-r^2/0.25), diag 1+1e-3", "leaf": w.leaf, "aca_tol": w.tol,
        "tree": "adaptive", "tol": o.tol,
        "inner": "GMRES(30) on BF16 factors, f32 arithmetic, to 1e-3",
        "outer": "FP64 residuals on FP64 factors", "converged": bool(info.converged),
        "rel_residual": info.rel_residual, "outer_iters": info.outer_iters,
        "inner_iters": info.inner_iters, "seconds": secs,
        "value": N * nrhs / secs, "unit": "N*nrhs/s solved", "build_s": round(build, 2),
        "history": [info.history[i] for i in range(min(info.outer_iters + 1, 64))],
        "product_16rhs_bf16": trees,
        "gram_system": c4,
    }


def gram_solve(P, torch, W, w, pts, q, H64, build, restart=50, max_outer=2):
    """The Gaussian-mixture workload's own system: the Gram matrix
    K~ U = F with K(i,i) = 1 + 1e-3 (the SVM-style regularised kernel matrix),
    GMRES with iterative refinement to 1e-10, inner GMRES(restart) in FP64 on
    the FP64 factors themselves (a low-precision inner operator perturbs this
    system by more than its smallest eigenvalues), at most max_outer cycles.
    Reported as it ends: converged or not, the residual history against the
    operator, and the residual against the direct sum on 256 sampled rows."""
    import oracle
    N, nrhs = w.N, q.shape[1]
    F = torch.tensor(np.ascontiguousarray(q.T), dtype=torch.float64, device="cuda").t()
    U = torch.zeros((nrhs, N), dtype=torch.float64, device="cuda").t()
    o = P.default_solve_opts()
    o.tol, o.inner_tol, o.restart, o.max_outer = 1e-10, 1e-12, restart, max_outer
    o.lo_compute = P.FP64
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = P.hodlr_solve(H64.h, H64.h, 0.0, 1.0, F, U, o)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    u = U.t().contiguous().cpu().numpy().T
    rows = np.sort(W.rng(212).choice(N, 256, replace=False))
    oracle.build(force=False)
    ku = oracle.direct(pts, oracle.kernel(w.kernel, h=w.h, diag=w.diag), u, rows=rows)
    true_res = float(np.max(np.linalg.norm(q[rows] - ku, axis=0) /
                            np.linalg.norm(q[rows], axis=0)))
    print(f"[bench] Gram system: {secs:.1f} s, {info.inner_iters} products, converged "
          f"{bool(info.converged)}, residual {info.rel_residual:.2e} (direct sum, sampled rows: "
          f"{true_res:.2e})", file=sys.stderr, flush=True)
    return {
        "system": "K~ U = F, K(i,i) = 1 + 1e-3", "tol": o.tol,
        "inner": f"GMRES({restart}) in FP64 on the FP64 factors",
        "outer": "FP64 residuals on FP64 factors", "max_outer": max_outer,
        "converged": bool(info.converged), "rel_residual": info.rel_residual,
        "outer_iters": info.outer_iters, "inner_iters": info.inner_iters, "seconds": secs,
        "history": [info.history[i] for i in range(min(info.outer_iters + 1, 64))],
        "residual_vs_direct_sum_sampled": true_res,
        "residual_ref": "max over columns of |F - K U| / |F| on 256 sampled rows (seed 212), "
                        "K by the direct sum",
        "build_s": round(build, 2),
    }


def serve_bench(P, torch, W, full=True):
    """Serving: resident point sets (N log-uniform, d in {2,3}, kernels log r,
    1/r, Gaussian h=0.5 drawn uniformly, FP32 factors, leaf 64, ACA 1e-8);
    requests half products (nrhs 1..64) and half solves of (I + K/N) u = f
    to 1e-8, arriving as a Poisson stream at 70% of the capacity measured
    with all requests submitted at once.  Latency = queueing + running."""
    nsets, nreq, nmax = (64, 256, 18) if full else (16, 128, 16)
    g = W.rng(5)
    srv = P.Server(max_concurrent=8, max_batch_cols=64, max_points=1 << nmax)
    kinds = ["log", "inv_r", "gauss"]
    sets = []
    t0 = time.perf_counter()
    for i in range(nsets):
        N = int(round(2.0 ** g.uniform(14, nmax)))
        d = int(g.integers(2, 4))
        kn = kinds[int(g.integers(0, 3))]
        pts = W.uniform_points(N, d, 500 + i)
        k = P.make_kernel(kn, h=0.5, diag=1.0 if kn == "gauss" else 0.0)
        sets.append((srv.add_set(pts, k, 64, 1e-8, storage=P.FP32), N))
        if (i + 1) % 8 == 0:
            st = srv.stats()
            print(f"[bench] serve: {i + 1}/{nsets} sets resident, "
                  f"{st.used_bytes / 2**30:.1f} GiB of {st.budget_bytes / 2**30:.1f}, "
                  f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    build = time.perf_counter() - t0
    reqs = []
    for i in range(nreq):
        s = int(g.integers(0, nsets))
        if g.random() < 0.5:
            reqs.append((P.REQ_MATVEC, s, int(g.integers(1, 65))))
        else:
            reqs.append((P.REQ_SOLVE, s, 1))
    X = []
    for i, (kind, s, n) in enumerate(reqs):
        N = sets[s][1]
        X.append(torch.tensor(W.rng(900 + i).standard_normal((n, N)), device="cuda").t()
                 if n > 1 else torch.tensor(W.rng(900 + i).standard_normal(N), device="cuda"))
    Y = [torch.zeros_like(x) for x in X]

    def run(rate):
        t_start = time.perf_counter()
        arr = np.cumsum(W.rng(11).exponential(1.0 / rate, size=nreq)) if rate else np.zeros(nreq)
        ids = []
        for i, (kind, s, n) in enumerate(reqs):
            while time.perf_counter() - t_start < arr[i]:
                pass
            kw = dict(alpha=1.0, beta=1.0 / sets[s][1], tol=1e-8) if kind == P.REQ_SOLVE else {}
            ids.append(srv.submit(kind, sets[s][0], X[i], Y[i], **kw))
        lat = np.array([sum(srv.wait(r)) for r in ids]) / 1e3   # ms
        return time.perf_counter() - t_start, lat

    run(None)   # warm-up
    wall0, _ = run(None)
    cap = nreq / wall0
    print(f"[bench] serve: capacity {cap:.1f} requests/s (all submitted at once)",
          file=sys.stderr, flush=True)
    st0 = srv.stats()
    wall, lat = run(0.7 * cap)
    st1 = srv.stats()
    cols = sum(n * sets[s][1] for kind, s, n in reqs if kind == P.REQ_MATVEC)
    srv.close()
    return {
        "sets": nsets, "requests": nreq, "N_range": [14, nmax], "storage": "fp32 factors",
        "capacity_req_per_s": cap, "arrival_rate_req_per_s": 0.7 * cap,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "throughput_req_per_s": nreq / wall, "matvec_N_nrhs_per_s": cols / wall,
        "launches": int(st1.launches - st0.launches),
        "batched_requests": int(st1.batched_requests - st0.batched_requests),
        "multiset_launches": int(st1.multiset_launches - st0.multiset_launches),
        "max_concurrent": int(st1.max_concurrent), "failed": int(st1.failed),
        "build_s": round(build, 1),
    }


def class_gbs(info, cls_ms, sf, sc):
    """achieved GB/s of every block class (algorithmic bytes over its time)"""
    out = []
    for c in range(NCLASS):
        nb = info.class_factor_elems[c] * sf + info.class_vector_elems[c] * sc
        out.append(round(nb / (cls_ms[c] * 1e-3) / 1e9, 1) if cls_ms[c] > 0 and nb else 0.0)
    return out


def adm_bench(P, torch, W, N=1 << 15):
    """The admissibility conditions side by side (the comparison of sec. 6.1:
    4D, log r, ACA 1e-6): N points uniform in [-1,1]^4, leaf 128, one N(0,1)
    right-hand side, FP64; per condition the build time, factor bytes,
    largest rank, product time and error against the direct sum on 256
    sampled rows."""
    import oracle
    pts = W.uniform_points(N, 4, 3)
    q = W.rhs_normal(N, 1, 103)[:, 0]
    k = P.make_kernel("log")
    rows = np.sort(W.rng(203).choice(N, 256, replace=False))
    oracle.build(force=False)
    bd = oracle.direct(pts, oracle.kernel("log"), q, rows=rows)
    X = torch.tensor(q, device="cuda")
    out = []
    for adm, name in ((-1, "far field only (H, strong)"), (0, "vertex sharing (HODLRdD)"),
                      (1, "edges (d' <= 1)"), (2, "d' <= 2"), (3, "every pair (HODLR, weak)")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H = P.HODLR(pts, k, 128, 1e-6, domain=(np.full(4, -1.0), 2.0), adm_dim=adm)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        info = H.info()
        Y = H.matvec(X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            H.matvec(X, out=Y)
        torch.cuda.synchronize()
        tm = (time.perf_counter() - t0) / 5
        y = Y.cpu().numpy()
        out.append({
            "adm_dim": adm, "condition": name, "build_s": round(tb, 3),
            "factor_bytes": int(8 * sum(info.factor_elems[l] for l in range(1, info.kappa + 1))),
            "rank_max": int(max(info.rank_max[l] for l in range(1, info.kappa + 1))),
            "near_pairs": int(info.near_pairs), "matvec_ms": tm * 1e3,
            "rel_err": float(np.linalg.norm(y[rows] - bd) / np.linalg.norm(bd)),
        })
        del H
    return {"workload": f"{N} points uniform in [-1,1]^4, log r, leaf 128, ACA 1e-6, FP64",
            "conditions": out}


def skeleton_bench(P, torch, w, pts, q, steps, warmup, level_rule, bd, rows):
    """The skeleton storage form on the main workload: FP64, the kernel
    evaluated on the fly for K(I, tau) and K(sigma, J)."""
    t0 = time.perf_counter()
    H = P.HODLR(pts, P.make_kernel(w.kernel, h=w.h, diag=w.diag), w.leaf, w.tol,
                domain=w.domain, level_rule=level_rule, skeleton=True)
    torch.cuda.synchronize()
    build = time.perf_counter() - t0
    info = H.info()
    X = torch.tensor(q, dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    wall, per, _, lat = time_matvecs(P, torch, H, X, Y, P.FP64, warmup, steps)
    y = Y.cpu().numpy()
    se = sum(info.factor_elems[l] for l in range(1, info.kappa + 1))
    del H
    return {
        "value": w.N / (wall / steps), "unit": "N*nrhs/s", "ms_per_step": wall / steps * 1e3,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "stage_ms": [round(float(v), 4) for v in per.mean(axis=0)],
        "stored_bytes": int(8 * se), "device_bytes": int(info.device_bytes),
        "build_s": round(build, 2), "rel_err": rel_err_rows(y, bd, rows),
        "dtype": "f64",
    }


def factor_bytes(info, elem):
    return sum(info.factor_elems[l] for l in range(1, info.kappa + 1)) * elem


def rel_err_rows(y, ref, rows):
    return float(np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref))


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, pts, q, level_rule, budget_s=30.0, reps=5):
    """The oracle timed on the host: its matvec over the target rows of one
    level-1 box (all levels' blocks of those rows), after compressing exactly
    the blocks those rows need; median of up to `reps` runs within a budget,
    on all host threads and on one."""
    import oracle
    oracle.build(force=False)
    k = oracle.kernel(w.kernel, diag=w.diag)
    t0 = time.perf_counter()
    o = oracle.OracleHODLR(pts, w.leaf, level_rule, domain=w.domain)
    start, _, _ = o.boxes(1)
    r0, r1 = int(start[0]), int(start[1])
    o.compress(k, w.tol, rows=(r0, r1))
    t_setup = time.perf_counter() - t0
    all_threads = oracle.num_threads()

    def timed(threads):
        oracle.set_threads(threads)
        times, b = [], None
        for _ in range(reps):
            t1 = time.perf_counter()
            b = o.matvec(k, q, rows=(r0, r1))
            times.append(time.perf_counter() - t1)
            if sum(times) > budget_s:
                break
        return float(np.median(times)), len(times), b

    tm, nrep, b = timed(all_threads)
    t1c, nrep1, _ = timed(1)
    oracle.set_threads(all_threads)
    rows = o.perm()[r0:r1]
    return {
        "value": (r1 - r0) * 1 / tm,
        "unit": "N*nrhs/s",
        "cores": all_threads,
        "kind": "oracle",
        "cpu_model": _cpu_model(),
        "sample": f"oracle matvec (FP64, every ordered block) over the {r1 - r0} target rows of "
                  f"level-1 box 0 (all levels' blocks of those rows), median of {nrep} on "
                  f"{all_threads} threads and of {nrep1} on 1 thread; the oracle's OpenMP loop "
                  f"runs over the target boxes of each level; setup (tree, lists, ACA of those "
                  f"blocks) {t_setup:.1f} s not timed",
        "seconds_per_matvec": tm,
        "value_1_core": (r1 - r0) / t1c,
        "seconds_per_matvec_1_core": t1c,
        "parallel_speedup": t1c / tm,
    }, rows, b[rows]


def depth_rule_bench(P, torch, w, pts, q, bd, rows, steps, warmup):
    """The main workload with the max-count depth rule (the smallest level
    whose fullest box holds at most leaf points) beside the closed form:
    depth, blocks, dense pairs, bytes, build and FP64 product time, error."""
    t0 = time.perf_counter()
    H = P.HODLR(pts, P.make_kernel(w.kernel, h=w.h, diag=w.diag), w.leaf, w.tol,
                domain=w.domain, level_rule=0)
    torch.cuda.synchronize()
    build = time.perf_counter() - t0
    info = H.info()
    X = torch.tensor(q, dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    wall, per, _, lat = time_matvecs(P, torch, H, X, Y, P.FP64, warmup, steps)
    y = Y.cpu().numpy()
    del H
    return {
        "rule": "max-count", "kappa": info.kappa,
        "stored_blocks": int(sum(info.stored_blocks[l] for l in range(1, info.kappa + 1))),
        "near_pairs": int(info.near_pairs), "factor_bytes": int(factor_bytes(info, 8)),
        "build_s": round(build, 2), "ms_per_step": wall / steps * 1e3,
        "value": w.N / (wall / steps), "unit": "N*nrhs/s", "dtype": "f64",
        "stage_ms": [round(float(v), 4) for v in per.mean(axis=0)],
        "rel_err": rel_err_rows(y, bd, rows),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform3d_invr_n262144")
    ap.add_argument("--n", type=int, default=0, help="override N (smaller runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--level-rule", type=int, default=1,
                    help="1: depth from the closed form (balanced tree); 0: fullest box rule")
    ap.add_argument("--no-multi-rhs", action="store_true",
                    help="skip the 32-RHS BF16 matrix-core workload")
    ap.add_argument("--multi-rhs-n", type=int, default=0, help="override its N")
    ap.add_argument("--no-multi-rhs-fp32", action="store_true",
                    help="skip the multi-RHS product with FP32 factors")
    ap.add_argument("--no-solve", action="store_true", help="skip the GMRES-IR solve")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the small 2D workload (eager and graph-replayed latency)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-skeleton", action="store_true", help="skip the skeleton form")
    ap.add_argument("--no-adm", action="store_true",
                    help="skip the comparison of admissibility conditions")
    ap.add_argument("--serve-small", action="store_true",
                    help="serving reduced to 16 sets up to 2^16 points and 128 requests")
    ap.add_argument("--no-depth-rule", action="store_true",
                    help="skip the main workload under the max-count depth rule")
    ap.add_argument("--solve-n", type=int, default=0, help="override the solve's N")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; "
              "run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2209_05819_amd as P
    from paper_2209_05819_amd import workloads as W

    w = W.WORKLOADS[args.workload]
    if args.n:
        w = W.scaled(w, args.n)
    pts = w.points()
    q = w.rhs()[:, 0].copy()
    N = w.N
    kern = P.make_kernel(w.kernel, h=w.h, diag=w.diag)
    print(f"[bench] workload {w.name} N={N} d={w.d}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    H64 = P.HODLR(pts, kern, w.leaf, w.tol, domain=w.domain, level_rule=args.level_rule)
    torch.cuda.synchronize()
    build64 = time.perf_counter() - t0
    info = H64.info()
    print(f"[bench] FP64 build {build64:.2f} s kappa={info.kappa}", file=sys.stderr, flush=True)

    X = torch.tensor(q, dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    wall, per, cls, lat = time_matvecs(P, torch, H64, X, Y, P.FP64, args.warmup, args.steps)
    y64 = Y.cpu().numpy()
    ms_step = wall / args.steps * 1e3
    stage_ms = per.mean(axis=0)
    cls_ms = cls.mean(axis=0)
    print(f"[bench] FP64 {ms_step:.3f} ms/step stages {np.round(stage_ms, 3).tolist()}",
          file=sys.stderr, flush=True)

    fb64 = factor_bytes(info, 8)
    roof64 = roofline(info, cls_ms, 8, 8)
    roof64["traffic"] = measured_traffic(w.name, roof64["kernel"], "fp64")
    # whole product: every stored factor element once plus x in and y out
    vec_bytes = 8 * (2 * N)
    matvec_gbs = (fb64 + vec_bytes) / (lat.mean() * 1e-3) / 1e9
    apply_gbs = fb64 / (stage_ms[1] * 1e-3 + stage_ms[2] * 1e-3) / 1e9

    mixed = None
    if not args.no_mixed:
        t0 = time.perf_counter()
        H32 = P.HODLR(pts, kern, w.leaf, w.tol, domain=w.domain, level_rule=args.level_rule,
                      storage=P.FP32)
        torch.cuda.synchronize()
        build32 = time.perf_counter() - t0
        info32 = H32.info()
        Y32 = torch.empty_like(X)
        wall32, per32, cls32, lat32 = time_matvecs(P, torch, H32, X, Y32, P.FP32, args.warmup,
                                                   args.steps)
        y32 = Y32.cpu().numpy()
        fb32 = factor_bytes(info32, 4)
        st32 = per32.mean(axis=0)
        mixed = {
            "value": N / (wall32 / args.steps),
            "ms_per_step": wall32 / args.steps * 1e3,
            "p50_ms": float(np.percentile(lat32, 50)),
            "p99_ms": float(np.percentile(lat32, 99)),
            "dtype": "f32 factors, f32 arithmetic",
            "stage_ms": [round(float(v), 4) for v in st32],
            "factor_bytes": int(fb32),
            "build_s": round(build32, 2),
            "speedup_vs_fp64": (N / (wall32 / args.steps)) / (N / (wall / args.steps)),
            "class_ms": [round(float(v), 4) for v in cls32.mean(axis=0)],
            "class_gbs": class_gbs(info32, cls32.mean(axis=0), 4, 4),
            "roofline": roofline(info32, cls32.mean(axis=0), 4, 4),
            "apply_roofline": {"achieved": fb32 / ((st32[1] + st32[2]) * 1e-3) / 1e9,
                               "frac": fb32 / ((st32[1] + st32[2]) * 1e-3) / 1e9 / HBM_PEAK_GBS},
        }
        del H32

    # accuracy on sampled rows against the plain definition (direct sum)
    import oracle
    oracle.build(force=False)
    g = W.rng(203)
    rows = np.sort(g.choice(N, size=min(N, 1024), replace=False))
    bd = oracle.direct(pts, oracle.kernel(w.kernel, diag=w.diag), q, rows=rows)
    err64 = rel_err_rows(y64, bd, rows)
    if mixed is not None:
        mixed["rel_err"] = rel_err_rows(y32, bd, rows)

    skel = None
    if not args.no_skeleton:
        skel = skeleton_bench(P, torch, w, pts, q, args.steps, args.warmup, args.level_rule, bd,
                              rows)

    depth = None
    if not args.no_depth_rule and args.level_rule == 1:
        depth = depth_rule_bench(P, torch, w, pts, q, bd, rows, max(5, args.steps // 2),
                                 args.warmup)
        print(f"[bench] max-count depth: kappa {depth['kappa']}, {depth['ms_per_step']:.2f} ms, "
              f"build {depth['build_s']} s", file=sys.stderr, flush=True)

    mrhs = None
    if not args.no_multi_rhs:
        mrhs = multi_rhs(P, torch, W, max(3, args.steps // 4), 1, args.multi_rhs_n)
        if not args.no_multi_rhs_fp32:
            mrhs["fp32_factors"] = multi_rhs_fp32(P, torch, W, 3, args.multi_rhs_n)

    small = None
    if not args.no_small:
        small = small_bench(P, torch, W)
        for name, r in small["routes"].items():
            print(f"[bench] small workload, {name}: eager {r['eager_p50_ms']:.4f} ms "
                  f"(wall {r['eager_wall_p50_ms']:.3f}), graph {r['graph_p50_ms']:.4f} ms "
                  f"(wall {r['graph_wall_p50_ms']:.3f})", file=sys.stderr, flush=True)
        print(f"[bench] small workload: autotuner kept {small['autotune']['route']}, "
              f"rel err {small['rel_err']:.2e}", file=sys.stderr, flush=True)

    solve = None
    if not args.no_solve:
        solve = solve_bench(P, torch, W, args.solve_n)

    serve = None
    if not args.no_serve:
        serve = serve_bench(P, torch, W, not args.serve_small)

    adm = None
    if not args.no_adm:
        adm = adm_bench(P, torch, W)

    cpu = None
    if not args.no_cpu_baseline:
        cpu, crow, cb = cpu_baseline(w, pts, q, args.level_rule)
        cpu_err = float(np.linalg.norm(y64[crow] - cb) / np.linalg.norm(cb))
        cpu["gpu_vs_oracle_rel_err"] = cpu_err

    if args.copy_calibration:
        # plain elementwise pass over 1 GiB (reads 1 GiB, writes 1 GiB), for
        # scaling the HBM traffic counters of the same run
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()

    out = {
        "metric": "HODLRdD matvec N*nrhs/s at stated rel err, FP64 vs mixed; p50/p99 latency",
        "value": N / (wall / args.steps),
        "unit": "N*nrhs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "N": N, "d": w.d, "kernel": "1/r, diag 0" if w.kernel ==
                   "inv_r" else w.kernel, "leaf": w.leaf, "aca_tol": w.tol, "nrhs": 1,
                   "level_rule": "max-count" if args.level_rule == 0 else "closed-form",
                   "storage": "one factor pair per unordered block pair"},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "rel_err": err64,
        "rel_err_ref": "direct sum on 1024 sampled rows (seed 203)",
        "stage_ms": [round(float(v), 4) for v in stage_ms],
        "stages": ["permute_in", "block_classes+split_projection", "split_expansion",
                   "gather+near_field+permute_out"],
        "build_s": round(build64, 2),
        "build_ms_tree_lists_aca": [round(info.build_ms[i], 1) for i in range(3)],
        "kappa": info.kappa,
        "stored_blocks": int(sum(info.stored_blocks[l] for l in range(1, info.kappa + 1))),
        "rank_max": int(max([info.rank_max[l] for l in range(1, info.kappa + 1)] or [0])),
        "factor_bytes": int(fb64),
        "near_pairs": int(info.near_pairs),
        "class_ms": [round(float(v), 4) for v in cls_ms],
        "class_kernels": CLASS_KERNELS,
        "class_gbs": class_gbs(info, cls_ms, 8, 8),
        "roofline": roof64,
        "apply_roofline": {"achieved": apply_gbs, "frac": apply_gbs / HBM_PEAK_GBS,
                           "bytes": int(fb64), "what": "all stored factors once over stages 2+3"},
        "matvec_roofline": {"achieved": matvec_gbs, "frac": matvec_gbs / HBM_PEAK_GBS,
                            "bytes": int(fb64 + vec_bytes)},
        "mixed": mixed,
        "skeleton": skel,
        "depth_rule_max_count": depth,
        "multi_rhs": mrhs,
        "solve": solve,
        "small": small,
        "serve": serve,
        "admissibility": adm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
