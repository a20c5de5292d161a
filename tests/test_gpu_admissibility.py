"""Admissibility variants (needs an MI355X): far field only (adm_dim = -1),
hyper-surfaces up to a given dimension, and every pair (adm_dim = d-1, HODLR).
Lists bit-exact against the oracle; products with the oracle's factors to
FP64 rounding; the full pipeline within the ACA tolerance of the direct sum.
"""
import sys

import numpy as np
import pytest

from paper_2209_05819_amd import workloads as W
from test_gpu_parity import _gpu_matvec, _pts, _rel, _symmetrize

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


LIST_CASES = [
    # d, N, leaf, rule, adm
    (2, 4000, 32, 0, -1), (2, 4000, 32, 1, 1), (3, 12000, 40, 0, -1), (3, 12000, 40, 1, 1),
    (3, 9000, 30, 0, 2), (4, 8000, 50, 0, -1), (4, 8000, 50, 1, 2), (4, 6000, 40, 0, 3),
    (1, 3000, 20, 0, -1),
]


@pytest.mark.parametrize("d,N,leaf,rule,adm", LIST_CASES)
def test_lists_bit_exact_for_every_admissibility(P, orc, d, N, leaf, rule, adm):
    _say(f"[adm] lists d={d} N={N} adm={adm}")
    pts = _pts(d, N, 600 + d, "uniform")
    o = orc.OracleHODLR(pts, leaf, rule, adm_dim=adm)
    H = P.HODLR(pts, P.make_kernel("inv_r"), leaf, 1e-6, level_rule=rule, skip_aca=True,
                adm_dim=adm)
    assert H.info().kappa == o.kappa
    for l in range(1, o.kappa + 1):
        p0, col0 = o.il(l)
        p1, col1 = P.hodlr_export_il(H.h, l, len(p0) - 1)
        assert np.array_equal(p0, p1) and np.array_equal(col0, col1), f"level {l}"
    p0, col0 = o.near()
    p1, col1 = P.hodlr_export_near(H.h, len(p0) - 1)
    assert np.array_equal(p0, p1) and np.array_equal(col0, col1)


@pytest.mark.parametrize("d,N,leaf,kern,adm", [
    (2, 4000, 32, "log", -1), (3, 6000, 48, "inv_r", -1), (3, 6000, 48, "gauss", 2),
    (2, 3000, 32, "log", 1),
])
def test_apply_with_oracle_factors_for_every_admissibility(P, orc, d, N, leaf, kern, adm):
    _say(f"[adm] apply d={d} N={N} {kern} adm={adm}")
    pts = _pts(d, N, 610 + d, "uniform")
    diag = 1.0 if kern == "gauss" else 0.0
    ko = orc.kernel(kern, h=0.5, diag=diag)
    o = orc.OracleHODLR(pts, leaf, 1, adm_dim=adm)
    o.compress(ko, 1e-9)
    H = P.HODLR(pts, P.make_kernel(kern, h=0.5, diag=diag), leaf, 1e-9, level_rule=1,
                skip_aca=True, adm_dim=adm)
    for l in range(1, o.kappa + 1):
        r, U, V = _symmetrize(o, l)
        o.set_factors(l, r, U, V)
        P.hodlr_import_factors(H.h, l, r, U, V)
    q = W.rhs_normal(N, 2, 13)
    assert _rel(_gpu_matvec(P, H, q), o.matvec(ko, q)) <= 1e-13


@pytest.mark.parametrize("d,N,leaf,kern,adm,tol", [
    (3, 15000, 64, "inv_r", -1, 1e-8), (2, 8000, 64, "log", 1, 1e-8),
    (4, 10000, 128, "inv_r2", 1, 1e-6),
])
def test_pipeline_for_every_admissibility(P, orc, d, N, leaf, kern, adm, tol):
    _say(f"[adm] pipeline d={d} N={N} {kern} adm={adm}")
    pts = _pts(d, N, 620 + d, "uniform")
    ko = orc.kernel(kern)
    H = P.HODLR(pts, P.make_kernel(kern), leaf, tol, adm_dim=adm)
    q = W.rhs_normal(N, 1, 14)[:, 0]
    rows = np.sort(W.rng(15).choice(N, 800, replace=False))
    bd = orc.direct(pts, ko, q, rows=rows)
    bg = _gpu_matvec(P, H, q)[rows]
    err = _rel(bg, bd)
    _say(f"  rel err {err:.2e}")
    assert err <= tol


def test_admissibility_out_of_range(P):
    with pytest.raises(P.HodlrError, match="EINVAL"):
        P.HODLR(W.uniform_points(500, 2, 1), P.make_kernel("log"), 16, 1e-6, adm_dim=2)
