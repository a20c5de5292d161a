"""The cooperative ACA (the largest blocks spread over many workgroups of one
cooperative launch) against the oracle and the direct sum (needs an MI355X).

A threshold in the environment sends blocks of these small test problems to
the cooperative kernel, which the library otherwise uses for blocks of at
least 16384 rows plus columns.  The product must meet the ACA tolerance
against the direct sum, the ranks must agree with the oracle's ACA of the
same blocks, and the skeleton form built from the cooperative pivots must
reproduce the U/V product.
"""
import os
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


@pytest.fixture
def coop_min(monkeypatch):
    def set_(v):
        monkeypatch.setenv("HODLR_ACA_COOP_MIN", str(v))
    return set_


CASES = [
    # d, N, leaf, kernel, h, diag, tol, dist, threshold
    (3, 20000, 64, "inv_r", 1.0, 0.0, 1e-10, "uniform", 1024),
    (2, 4096, 64, "log", 1.0, 0.0, 1e-8, "uniform", 256),
    (3, 16000, 64, "gauss", 0.5, 1.001, 1e-6, "mixture", 2000),
    (1, 6000, 32, "exp", 0.3, 0.0, 1e-10, "uniform", 500),
]


@pytest.mark.parametrize("d,N,leaf,kern,h,diag,tol,dist,thr", CASES)
def test_cooperative_aca_against_oracle(P, orc, coop_min, d, N, leaf, kern, h, diag, tol, dist,
                                        thr):
    _say(f"[aca coop] d={d} N={N} {kern} tol={tol} threshold {thr}")
    pts = _pts(d, N, 900 + d, dist)
    ko = orc.kernel(kern, h=h, diag=diag)
    coop_min(thr)
    H = P.HODLR(pts, P.make_kernel(kern, h=h, diag=diag), leaf, tol)
    q = W.rhs_normal(N, 2, 41)
    bd = orc.direct(pts, ko, q)
    bg = _gpu_matvec(P, H, q)
    err = _rel(bg, bd)
    o = orc.OracleHODLR(pts, leaf, 1)
    o.compress(ko, tol)
    nco = 0
    for l in range(1, o.kappa + 1):
        r_or = o.ranks(l)
        r_gpu, _, _ = P.hodlr_export_factors(H.h, l, len(r_or))
        ptr, col = o.il(l)
        rows = np.repeat(np.arange(len(ptr) - 1), np.diff(ptr))
        fwd = rows < col
        st, _, _ = o.boxes(l)
        size = (np.diff(st)[rows] + np.diff(st)[col])[fwd]
        big = size >= thr
        nco += int(big.sum())
        if big.any():
            diff = np.abs(r_gpu[fwd][big].astype(int) - r_or[fwd][big].astype(int))
            assert np.mean(diff <= 2) >= 0.9, f"level {l}"
    _say(f"  {nco} blocks cooperative, rel err vs direct {err:.3e}")
    assert nco > 0
    assert err <= tol


def test_cooperative_pivots_give_the_skeleton(P, coop_min):
    """The skeleton form takes ACA's pivots: built from the cooperative
    kernel's, it must reproduce the U/V product of the same handle's ranks."""
    pts = W.uniform_points(12000, 3, 77)
    k = P.make_kernel("inv_r")
    coop_min(1000)
    Huv = P.HODLR(pts, k, 64, 1e-10)
    Hsk = P.HODLR(pts, k, 64, 1e-10, skeleton=True)
    q = W.rhs_normal(12000, 1, 42)[:, 0]
    d = _rel(_gpu_matvec(P, Hsk, q), _gpu_matvec(P, Huv, q))
    _say(f"[aca coop] skeleton vs U/V {d:.2e}")
    assert d <= 1e-11


def test_cooperative_and_single_workgroup_agree(P, coop_min):
    """The same blocks compressed by one workgroup each and cooperatively:
    the two products agree to twice the tolerance, and most ranks match."""
    pts = W.uniform_points(20000, 3, 78)
    k = P.make_kernel("inv_r")
    coop_min(1 << 30)
    H1 = P.HODLR(pts, k, 64, 1e-10)
    coop_min(1024)
    H2 = P.HODLR(pts, k, 64, 1e-10)
    q = W.rhs_normal(20000, 1, 43)[:, 0]
    assert _rel(_gpu_matvec(P, H2, q), _gpu_matvec(P, H1, q)) <= 2e-10
    nnz = int(H1.info().il_entries[1])
    r1 = P.hodlr_export_ranks(H1.h, 1, nnz)
    r2 = P.hodlr_export_ranks(H2.h, 1, nnz)
    assert np.mean(np.abs(r1.astype(int) - r2.astype(int)) <= 2) >= 0.9
