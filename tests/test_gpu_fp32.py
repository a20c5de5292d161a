"""FP32 factor storage and FP32 arithmetic on the single-RHS and few-RHS
paths, element by element against the oracle (needs an MI355X).

The oracle's own FP64 ACA factors are imported (the import stores them as
they are, without the truncation FP32 builds apply), so the differences from
the oracle's product are the roundings of the FP32 path: U and V rounded to
FP32 (u = 2^-24 each), x rounded to FP32 (u), and FP32 arithmetic in the
projections t = V x, the expansions U t, the sum of a row's contributions
over levels and entries, and the near field (kernel evaluation and the sum
over a leaf's near sources).  Each of those sums has at most L terms per
output element, L = (largest block side) + (largest rank) + (most
interaction-list entries over the levels of a row) + (most near-field
sources of a leaf); by the probabilistic rounding-error bound of Higham and
Mary (SIAM J. Sci. Comput. 41, 2019) a sum of L rounded terms is within
lambda sqrt(L) u of its terms' absolute sum except with probability about
2 exp(-lambda^2 / 2); lambda = 6 makes a failure by chance negligible over
every element of these tests.  Elementwise:

    |y_gpu - y| <= (3 + 6 sqrt(L)) u z,   z = sum |U| (|V| |x|) + K |x|,

z computed by the oracle with |U|, |V| and |x| (positive kernels, so the
near-field part is K |x|).
"""
import sys

import numpy as np
import pytest

from paper_2209_05819_amd import workloads as W
from test_gpu_bf16 import _abs_product
from test_gpu_parity import _gpu_matvec, _pts, _rel, _symmetrize

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


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


def _sum_length(o):
    """L: the longest accumulation an output element goes through."""
    side = rank = entries = 0
    for l in range(1, o.kappa + 1):
        start, _, _ = o.boxes(l)
        ptr, _ = o.il(l)
        side = max(side, int(np.diff(start).max()))
        r = o.ranks(l)
        rank = max(rank, int(r.max()) if len(r) else 0)
        entries += int(np.diff(ptr).max()) if len(ptr) > 1 else 0
    start, _, _ = o.boxes(o.kappa)
    sizes = np.diff(start)
    nptr, ncol = o.near()
    near = max(int(sizes[ncol[nptr[A]:nptr[A + 1]]].sum()) for A in range(len(nptr) - 1))
    return side + rank + entries + near


FP32_CASES = [
    # d, N, leaf, kernel, tol, rule, dist, sym, nrhs
    (3, 20000, 64, "inv_r", 1e-10, 1, "uniform", True, 1),
    (3, 20000, 64, "inv_r", 1e-10, 1, "uniform", False, 1),
    (3, 12000, 64, "inv_r", 1e-10, 1, "uniform", True, 6),
    (2, 6000, 64, "log", 1e-8, 0, "uniform", True, 1),
    (4, 9000, 128, "inv_r2", 1e-8, 1, "uniform", True, 3),
    # several passes of eight columns, the last one ragged
    (4, 9000, 128, "inv_r2", 1e-8, 1, "uniform", True, 20),
    (3, 12000, 64, "inv_r", 1e-10, 1, "uniform", False, 11),
    (3, 6000, 48, "gauss", 1e-6, 0, "mixture", True, 1),
]


@pytest.mark.parametrize("d,N,leaf,kern,tol,rule,dist,sym,nrhs", FP32_CASES)
def test_fp32_apply_with_oracle_factors(P, orc, d, N, leaf, kern, tol, rule, dist, sym, nrhs):
    _say(f"[fp32] d={d} N={N} {kern} sym={sym} nrhs={nrhs}")
    pts = _pts(d, N, 450 + d, dist)
    diag = 1.001 if kern == "gauss" else 0.0
    ko = orc.kernel(kern, h=0.5, diag=diag)
    o = orc.OracleHODLR(pts, leaf, rule)
    o.compress(ko, tol)
    H = P.HODLR(pts, P.make_kernel(kern, h=0.5, diag=diag), leaf, tol, level_rule=rule,
                skip_aca=True, symmetric=sym, storage=P.FP32)
    for l in range(1, o.kappa + 1):
        if sym:
            r, U, V = _symmetrize(o, l)
            o.set_factors(l, r, U, V)
        r, U, V = o.factors(l)
        P.hodlr_import_factors(H.h, l, r, U, V)
    L = _sum_length(o)
    c = (3 + 6 * np.sqrt(L)) * U32
    q = W.rhs_normal(N, nrhs, 23)
    qq = q[:, 0] if nrhs == 1 else q
    bo = o.matvec(ko, qq)
    z = _abs_product(o, ko, qq)
    for xdt in ("f32", "f64"):
        bg = _gpu_matvec(P, H, qq, x_dtype=xdt, compute=P.FP32)
        dev = np.abs(bg - bo)
        ratio = float(np.max(dev / (U32 * z)))
        _say(f"  x={xdt} L={L} rel err vs oracle {_rel(bg, bo):.3e}, "
             f"max |dy|/(u z) {ratio:.1f} (bound {c / U32:.0f})")
        assert np.all(dev <= c * z)
        assert _rel(bg, bo) <= 1e-5


def test_fp32_truncation_meets_the_mixed_tolerance(P, orc):
    """FP32 builds drop the trailing ACA terms below the storage's resolution:
    fewer stored elements than the FP64 build of the same points, and the
    product within 1e-5 of the direct sum (the mixed-precision tolerance)."""
    pts = W.uniform_points(20000, 3, 501)
    k = P.make_kernel("inv_r")
    H64 = P.HODLR(pts, k, 64, 1e-10)
    H32 = P.HODLR(pts, k, 64, 1e-10, storage=P.FP32)
    i64, i32 = H64.info(), H32.info()
    f64 = sum(i64.factor_elems[l] for l in range(1, i64.kappa + 1))
    f32 = sum(i32.factor_elems[l] for l in range(1, i32.kappa + 1))
    q = W.rhs_normal(20000, 1, 502)[:, 0]
    bd = orc.direct(pts, orc.kernel("inv_r"), q)
    err = _rel(_gpu_matvec(P, H32, q, x_dtype="f32", compute=P.FP32), bd)
    _say(f"[fp32] truncation: stored elements {f32:.3e} vs {f64:.3e} (FP64), rel err {err:.2e}")
    assert f32 < 0.9 * f64
    assert err <= 1e-5
