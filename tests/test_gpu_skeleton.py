"""Skeleton storage form of eqs. keq1/keq2 (needs an MI355X).

A handle in skeleton form stores each block's ACA pivots and the LU of
K(sigma, tau) and evaluates K(I, tau), K(sigma, J) inside the product.  Built
from the same points and tolerance as a U/V handle, the GPU's ACA takes the
same pivots (same ranks), and the skeleton identity
U V = K(I, tau) K(sigma, tau)^-1 K(sigma, J) makes the two products equal up
to rounding; the product is within the ACA tolerance of the direct sum.
"""
import sys

import numpy as np
import pytest

from paper_2209_05819_amd import workloads as W
from test_gpu_parity import _gpu_matvec, _pts, _rel

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


SKEL_CASES = [
    # d, N, leaf, kernel, h, diag, tol, symmetric, dist
    (3, 20000, 64, "inv_r", 1.0, 0.0, 1e-10, True, "uniform"),
    (2, 8000, 64, "log", 1.0, 0.0, 1e-8, True, "uniform"),
    (4, 10000, 128, "inv_r2", 1.0, 0.0, 1e-8, True, "uniform"),
    (3, 12000, 64, "gauss", 0.5, 1.001, 1e-6, False, "mixture"),
    (1, 5000, 32, "exp", 0.3, 0.0, 1e-10, True, "uniform"),
]


@pytest.mark.parametrize("d,N,leaf,kern,h,diag,tol,sym,dist", SKEL_CASES)
def test_skeleton_equals_uv_and_direct(P, orc, d, N, leaf, kern, h, diag, tol, sym, dist):
    _say(f"[skel] d={d} N={N} {kern} sym={sym}")
    pts = _pts(d, N, 700 + d, dist)
    k = P.make_kernel(kern, h=h, diag=diag)
    Huv = P.HODLR(pts, k, leaf, tol, symmetric=sym)
    Hsk = P.HODLR(pts, k, leaf, tol, symmetric=sym, skeleton=True)
    iuv, isk = Huv.info(), Hsk.info()
    for l in range(1, iuv.kappa + 1):
        nnz = int(iuv.il_entries[l])
        assert np.array_equal(P.hodlr_export_ranks(Huv.h, l, nnz),
                              P.hodlr_export_ranks(Hsk.h, l, nnz)), f"level {l}"
    fe_uv = sum(iuv.factor_elems[l] for l in range(1, iuv.kappa + 1))
    fe_sk = sum(isk.factor_elems[l] for l in range(1, isk.kappa + 1))
    assert fe_sk < fe_uv
    q = W.rhs_normal(N, 2, 51)
    buv = _gpu_matvec(P, Huv, q)
    bsk = _gpu_matvec(P, Hsk, q)
    d_uv = _rel(bsk, buv)
    rows = np.sort(W.rng(52).choice(N, 500, replace=False))
    bd = orc.direct(pts, orc.kernel(kern, h=h, diag=diag), q, rows=rows)
    err = _rel(bsk[rows], bd)
    _say(f"  |skel - uv| {d_uv:.2e}  skel vs direct {err:.2e}  stored {fe_sk:.3e} vs {fe_uv:.3e}")
    assert d_uv <= 1e-11
    assert err <= tol
    # columns are independent passes
    b1 = _gpu_matvec(P, Hsk, np.ascontiguousarray(q[:, 1]))
    assert np.array_equal(b1, bsk[:, 1])


def test_skeleton_errors(P):
    import torch
    pts = W.uniform_points(2000, 2, 3)
    k = P.make_kernel("log")
    for st in (P.BF16, P.FP32):
        with pytest.raises(P.HodlrError, match="EINVAL"):
            P.HODLR(pts, k, 32, 1e-6, skeleton=True, storage=st)
    with pytest.raises(P.HodlrError, match="EINVAL"):
        P.HODLR(pts, k, 32, 1e-6, skeleton=True, skip_aca=True)
    H = P.HODLR(pts, k, 32, 1e-6, skeleton=True)
    X = torch.ones(2000, dtype=torch.float64, device="cuda")
    with pytest.raises(P.HodlrError, match="EINVAL"):
        H.matvec(X, compute_prec=P.FP32)
    nnz = int(H.info().il_entries[1])
    with pytest.raises(P.HodlrError, match="EUNSUPPORTED"):
        P.hodlr_export_factors(H.h, 1, nnz)
    with pytest.raises(P.HodlrError, match="EUNSUPPORTED"):
        P.hodlr_import_factors(H.h, 1, np.zeros(nnz, dtype=np.int32), np.zeros(1), np.zeros(1))
