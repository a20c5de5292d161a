"""The persistent product (one launch walks every stage as an ordered queue
of work) against the per-class launches and the direct sum, alone, under
graph capture, and for several handles in one launch (needs an MI355X).

The persistent route applies every class-5 block (blocks of 1025 to 4608
rows and columns), and the class-4 blocks wider than a side the autotuner
may choose, by segmented projections; everything else runs the same
per-item arithmetic on both routes: the products agree to 1e-13 relative
(FP64) or 1e-5 (FP32).  Route 2, the per-class launches without the second
stream, gives the same bits as route 0.
"""
import sys

import numpy as np
import pytest

from paper_2209_05819_amd import workloads as W
from test_gpu_parity import _pts, _rel

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_05819_amd as P
    P.lib()
    return P


def _dev(torch, q, dt):
    q = np.asarray(q)
    if q.ndim == 1:
        return torch.tensor(q, dtype=dt, device="cuda")
    return torch.tensor(np.ascontiguousarray(q.T), dtype=dt, device="cuda").t()


def _host(Y):
    return (Y.t().contiguous().cpu().numpy().T if Y.dim() == 2 else Y.cpu().numpy()).astype(
        np.float64)


def _routes(P, torch, H, q, dt, comp):
    """The product on route 0 (per-class, near field on a second stream),
    1 (persistent) and 2 (per-class, one stream)."""
    X = _dev(torch, q, dt)
    out = []
    for route in (0, 1, 2):
        P.hodlr_set_route(H.h, route)
        Y = torch.full_like(X, float("nan"))
        H.matvec(X, compute_prec=comp, out=Y)
        torch.cuda.synchronize()
        out.append(_host(Y))
    P.hodlr_set_route(H.h, -1)
    return out


CASES = [
    # d, N, leaf, kernel, h, diag, tol, dist, storage, symmetric, rule
    (2, 4096, 64, "log", 1.0, 0.0, 1e-8, "uniform", "fp64", True, 1),
    (3, 20000, 64, "inv_r", 1.0, 0.0, 1e-10, "uniform", "fp64", True, 1),
    (3, 20000, 64, "inv_r", 1.0, 0.0, 1e-8, "uniform", "fp32", True, 1),
    (3, 12000, 64, "inv_r", 1.0, 0.0, 1e-8, "uniform", "fp64", False, 1),
    (1, 9000, 32, "exp", 0.3, 0.0, 1e-10, "uniform", "fp64", True, 1),
    (4, 9000, 128, "inv_r2", 1.0, 0.0, 1e-8, "uniform", "fp32", True, 1),
    (3, 16000, 64, "gauss", 0.5, 1.001, 1e-6, "mixture", "fp64", True, 2),
    (2, 60000, 64, "log", 1.0, 0.0, 1e-8, "uniform", "fp64", True, 1),
]


@pytest.mark.parametrize("d,N,leaf,kern,h,diag,tol,dist,st,sym,rule", CASES)
def test_persistent_equals_per_class(P, orc, d, N, leaf, kern, h, diag, tol, dist, st, sym,
                                     rule):
    import torch
    _say(f"[persist] d={d} N={N} {kern} {st} sym={sym} rule={rule}")
    pts = _pts(d, N, 950 + d, dist)
    storage = P.FP64 if st == "fp64" else P.FP32
    H = P.HODLR(pts, P.make_kernel(kern, h=h, diag=diag), leaf, tol, storage=storage,
                symmetric=sym, level_rule=rule)
    comp = storage
    dt = torch.float64 if st == "fp64" else torch.float32
    rel = 1e-13 if st == "fp64" else 1e-5
    for nrhs in (1, 3, 7, 11):
        q = W.rhs_normal(N, nrhs, 61 + nrhs)
        q = q[:, 0] if nrhs == 1 else q
        yc, yp, y1 = _routes(P, torch, H, q, dt, comp)
        assert np.all(np.isfinite(yp))
        err = _rel(yp, yc)
        _say(f"  nrhs={nrhs}: persistent vs per-class {err:.2e}")
        assert err <= rel
        # the same launches on one stream: the same sums in the same order
        assert np.array_equal(y1, yc)
    # the persistent product against the direct sum
    q = W.rhs_normal(N, 1, 70)[:, 0]
    rows = np.sort(W.rng(71).choice(N, min(N, 800), replace=False))
    bd = orc.direct(pts, orc.kernel(kern, h=h, diag=diag), q, rows=rows)
    P.hodlr_set_route(H.h, 1)
    Y = H.matvec(_dev(torch, q, dt), compute_prec=comp)
    torch.cuda.synchronize()
    err = _rel(_host(Y)[rows], bd)
    _say(f"  persistent vs direct sum {err:.2e}")
    assert err <= (tol if st == "fp64" else 1e-5)


def test_persistent_repeats_and_graph_replays(P):
    """Repeated launches reuse the self-resetting counters: every call gives
    the same bits; a captured launch replayed between eager work does too."""
    import torch
    pts = W.uniform_points(4096, 2, 1)
    H = P.HODLR(pts, P.make_kernel("log"), 64, 1e-8)
    P.hodlr_set_route(H.h, 1)
    X = torch.tensor(W.rhs_normal(4096, 1, 2)[:, 0], device="cuda")
    Y0 = H.matvec(X)
    torch.cuda.synchronize()
    for _ in range(5):
        Y = H.matvec(X)
        torch.cuda.synchronize()
        assert torch.equal(Y, Y0)
    Yg = torch.empty_like(X)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        P.hodlr_matvec(H.h, X, Yg)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        P.hodlr_matvec(H.h, X, Yg)
    for _ in range(3):
        Yg.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Yg, Y0)


@pytest.mark.parametrize("st", ["fp64", "fp32"])
def test_batch_of_handles_equals_separate_products(P, st):
    """Products on different point sets (2D and 3D, three kernels, different
    N and column counts) in one persistent launch, against each handle's own
    product."""
    import torch
    storage = P.FP64 if st == "fp64" else P.FP32
    dt = torch.float64 if st == "fp64" else torch.float32
    rel = 1e-13 if st == "fp64" else 1e-5
    specs = [(W.uniform_points(12000, 3, 81), "inv_r", 0.0, 3),
             (W.uniform_points(6000, 2, 82), "log", 0.0, 1),
             (W.gaussian_mixture(9000, 3, 83), "gauss", 1.001, 8),
             (W.uniform_points(3000, 2, 84), "gauss", 1.0, 2)]
    hs, Xs, Ys, refs = [], [], [], []
    for i, (pts, kern, diag, nr) in enumerate(specs):
        H = P.HODLR(pts, P.make_kernel(kern, h=0.5, diag=diag), 64, 1e-8, storage=storage)
        P.hodlr_set_route(H.h, 0)
        q = W.rhs_normal(pts.shape[0], nr, 90 + i)
        X = _dev(torch, q[:, 0] if nr == 1 else q, dt)
        refs.append(_host(H.matvec(X, compute_prec=storage)))
        hs.append(H)
        Xs.append(X)
        Ys.append(torch.full_like(X, float("nan")))
    torch.cuda.synchronize()
    P.hodlr_matvec_batch([H.h for H in hs], Xs, Ys)
    torch.cuda.synchronize()
    for i in range(len(hs)):
        err = _rel(_host(Ys[i]), refs[i])
        _say(f"[batch {st}] slot {i}: {err:.2e}")
        assert err <= rel


@pytest.mark.parametrize("d,N,kern,tol,st", [(2, 4096, "log", 1e-8, "fp64"),
                                             (3, 30000, "inv_r", 1e-10, "fp64"),
                                             (3, 30000, "inv_r", 1e-8, "fp32")])
def test_autotuner_keeps_the_product(P, d, N, kern, tol, st):
    """The autotuner times every tile shape of every block class and the
    three routes and keeps the fastest; the product after tuning equals the
    default one (the shapes change only the order of the sums)."""
    import torch
    storage = P.FP64 if st == "fp64" else P.FP32
    dt = torch.float64 if st == "fp64" else torch.float32
    rel = 1e-13 if st == "fp64" else 1e-5
    pts = W.uniform_points(N, d, 990 + d)
    H = P.HODLR(pts, P.make_kernel(kern), 64, tol, storage=storage)
    X = _dev(torch, W.rhs_normal(N, 1, 991)[:, 0], dt)
    y0 = _host(H.matvec(X, compute_prec=storage))
    t = P.hodlr_autotune(H.h, 1, P.FP64 if st == "fp64" else P.FP32, storage)
    _say(f"[autotune] d={d} N={N} {st}: route {t.route}, shapes {list(t.class_choice)[:6]}, "
         f"per-class {t.class_route_ms:.4f} ms, one stream {t.one_stream_ms:.4f} ms, "
         f"persistent {t.persistent_ms:.4f} ms")
    assert t.route in (0, 1, 2) and t.class_route_ms > 0 and t.persistent_ms > 0
    assert t.one_stream_ms > 0
    times = {0: t.class_route_ms, 2: t.one_stream_ms, 1: t.persistent_ms}
    assert times[t.route] == min(times.values())
    y1 = _host(H.matvec(X, compute_prec=storage))
    assert _rel(y1, y0) <= rel
    with pytest.raises(P.HodlrError, match="EINVAL"):
        P.hodlr_set_route(H.h, 3)
