"""BF16 factor storage and the matrix-core multi-RHS apply (needs an MI355X).

The oracle's own FP64 ACA factors are imported, so the only differences from
the oracle's product are the roundings of the BF16 path.  Their first-order
bound, elementwise: rounding U and V to BF16 (relative u = 2^-8 each), x to
BF16 and the projections t = V x to BF16 (matrix-core path) give

    |y_gpu - y| <= (4 u + FP32 accumulation) * z,   z = sum |U| (|V| |x|) + near field K |x|,

with FP32 accumulation over at most ~10^4 terms below 0.25 u.  z is computed
by the oracle itself, with |U|, |V| and |x| (positive kernels only, so the
near-field part of z is the oracle's own K |x|).
"""
import sys

import numpy as np
import pytest

from paper_2209_05819_amd import workloads as W
from test_gpu_parity import _gpu_matvec, _pts, _rel, _symmetrize

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -8
C_BOUND = 4.25 * U_BF16


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


def _abs_product(o, ko, q):
    """sum over blocks |U| (|V| |q|) + near field K |q|, by the oracle."""
    saved = [o.factors(l) for l in range(1, o.kappa + 1)]
    for l, (r, U, V) in enumerate(saved, start=1):
        o.set_factors(l, r, np.abs(U), np.abs(V))
    z = o.matvec(ko, np.abs(q))
    for l, (r, U, V) in enumerate(saved, start=1):
        o.set_factors(l, r, U, V)
    return z


BF16_CASES = [
    # d, N, leaf, kernel, tol, rule, dist, sym, nrhs
    (3, 20000, 64, "inv_r", 1e-10, 1, "uniform", True, 1),
    (3, 20000, 64, "inv_r", 1e-10, 1, "uniform", True, 16),
    (3, 20000, 64, "inv_r", 1e-10, 1, "uniform", True, 32),
    (3, 20000, 64, "inv_r", 1e-10, 1, "uniform", False, 20),
    (4, 9000, 128, "inv_r2", 1e-8, 1, "uniform", True, 40),
    (3, 6000, 48, "gauss", 1e-6, 0, "mixture", True, 7),
    (2, 4096, 64, "inv_r", 1e-8, 0, "uniform", True, 33),
]


@pytest.mark.parametrize("d,N,leaf,kern,tol,rule,dist,sym,nrhs", BF16_CASES)
def test_bf16_apply_with_oracle_factors(P, orc, d, N, leaf, kern, tol, rule, dist, sym, nrhs):
    _say(f"[bf16] d={d} N={N} {kern} sym={sym} nrhs={nrhs}")
    pts = _pts(d, N, 400 + d, dist)
    diag = 1.001 if kern == "gauss" else 0.0
    ko = orc.kernel(kern, h=0.5, diag=diag)
    o = orc.OracleHODLR(pts, leaf, rule)
    o.compress(ko, tol)
    H = P.HODLR(pts, P.make_kernel(kern, h=0.5, diag=diag), leaf, tol, level_rule=rule,
                skip_aca=True, symmetric=sym, storage=P.BF16)
    for l in range(1, o.kappa + 1):
        if sym:
            r, U, V = _symmetrize(o, l)
            o.set_factors(l, r, U, V)
        r, U, V = o.factors(l)
        P.hodlr_import_factors(H.h, l, r, U, V)
    q = W.rhs_normal(N, nrhs, 19)
    qq = q[:, 0] if nrhs == 1 else q
    bo = o.matvec(ko, qq)
    z = _abs_product(o, ko, qq)
    for xdt in ("f32", "f64"):
        bg = _gpu_matvec(P, H, qq, x_dtype=xdt, compute=P.FP32)
        dev = np.abs(bg - bo)
        ratio = float(np.max(dev / (C_BOUND * z)))
        _say(f"  x={xdt} rel err vs oracle {_rel(bg, bo):.3e}, max |dy|/(4.25u z) {ratio:.3f}")
        assert np.all(dev <= C_BOUND * z)
        assert _rel(bg, bo) <= 1e-2


def test_bf16_multi_rhs_columns_consistent(P, orc):
    """Each column of a 32-column product equals, within the same bound, the
    product of that column alone on the single-RHS path."""
    _say("[bf16] columns")
    pts = W.uniform_points(12000, 3, 41)
    H = P.HODLR(pts, P.make_kernel("inv_r"), 64, 1e-10, storage=P.BF16)
    q = W.rhs_normal(12000, 32, 42)
    bm = _gpu_matvec(P, H, q, x_dtype="f32", compute=P.FP32)
    o = orc.OracleHODLR(pts, 64, 1)
    ko = orc.kernel("inv_r")
    o.compress(ko, 1e-10)
    for c in (0, 13, 31):
        b1 = _gpu_matvec(P, H, np.ascontiguousarray(q[:, c]), x_dtype="f32", compute=P.FP32)
        z = _abs_product(o, ko, np.ascontiguousarray(q[:, c]))
        # both within 4.25 u z of the exact product: within 8.5 u z of each other
        assert np.all(np.abs(bm[:, c] - b1) <= 2 * C_BOUND * z * 1.05)


def test_bf16_pipeline_against_direct_sum(P, orc):
    _say("[bf16] pipeline")
    w = W.scaled(W.WORKLOADS["uniform4d_invr2_n524288"], 16000)
    pts, q = w.points(), w.rhs()[:, :32]
    ko = orc.kernel("inv_r2")
    H = P.HODLR(pts, P.make_kernel("inv_r2"), w.leaf, w.tol, domain=w.domain, storage=P.BF16)
    bg = _gpu_matvec(P, H, q, x_dtype="f32", compute=P.FP32)
    rows = np.sort(W.rng(7).choice(16000, 600, replace=False))
    bd = orc.direct(pts, ko, q, rows=rows)
    o = orc.OracleHODLR(pts, w.leaf, 1, domain=w.domain)
    o.compress(ko, w.tol)
    z = _abs_product(o, ko, q)[rows]
    err = np.linalg.norm(bg[rows] - bd) / np.linalg.norm(bd)
    bound = (w.tol * np.linalg.norm(bd) + C_BOUND * np.linalg.norm(z)) / np.linalg.norm(bd)
    _say(f"  bf16 pipeline rel err {err:.3e} (bound {bound:.3e})")
    assert err <= bound
